"""Pins of the oracle's traceback (the alignment returned with each hit, Section 2.2).

* every reported hit of several workloads (three scoring schemes, narrow and wide
  bands, indels): the path consumes exactly the hit's query and bank spans, its
  '=' / 'X' agree with the bases, it stays inside the band centred on band_d0, it
  starts and ends on a matched pair, and rescoring it move by move (a gap run of g
  costing open + g extend) gives the hit's score;
* hand-worked paths: an exact copy, one substitution, a deletion and an insertion
  inside homopolymer runs, where the path, walked back from the end, takes the
  diagonal while it scores as well and so puts the gap at its leftmost place;
* hits that are not alignments of the query are refused.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth


def rescore(ops, match, mismatch, gap_open, gap_extend):
    score, prev = 0, ""
    for op in ops:
        if op == "=":
            score += match
        elif op == "X":
            score -= mismatch
        else:
            score -= gap_extend + (gap_open if op != prev else 0)
        prev = op
    return score


def check_path(ix, q: bytes, prm, hit, ops, seq: bytes):
    qs, qe, ds, de = (int(hit[f]) for f in ("q_start", "q_end", "d_start", "d_end"))
    assert sum(op in "=XI" for op in ops) == qe - qs
    assert sum(op in "=XD" for op in ops) == de - ds
    assert ops[0] == "=" and ops[-1] == "="
    i, j = qs, ds
    up = bytes(q).upper().replace(b"U", b"T")
    for op in ops:
        if op in "=X":
            assert (up[i] == seq[j]) == (op == "=")
            assert abs((j - i) - int(hit["band_d0"])) <= prm.band
            i, j = i + 1, j + 1
        elif op == "I":
            i += 1
        else:
            j += 1
    assert rescore(ops, prm.match, prm.mismatch, prm.gap_open, prm.gap_extend) == int(hit["score"])


@pytest.mark.parametrize("kw,seed", [(dict(), 1), (dict(band=3), 2),
                                     (dict(match=2, mismatch=1, gap_open=1, gap_extend=1), 3),
                                     (dict(gap_open=0, gap_extend=3, band=10), 4)])
def test_every_reported_path(ggo, kw, seed):
    db = synth.random_db(70 + seed, n_seqs=120, lmin=0, lmax=1500)
    qs = synth.random_queries(70 + seed, db, n=15, lmin=20, lmax=800, frac_homolog=1.0,
                              ident_lo=0.8, ident_hi=0.98, indel_rate=0.03)
    ix = ggo.Index(db.seqs, db.off, 8)
    prm = ggo.params(0, max_gap=16, min_hsp_len=16, **kw)
    n = gaps = 0
    for i in range(qs.n):
        q = bytes(qs.query(i))
        rc, hits, m, _ = ix.search(q, prm)
        for h in hits:
            ops = ix.traceback(q, prm, h)
            check_path(ix, q, prm, h, ops, bytes(db.seq(int(h["seq_id"]))).upper())
            n += 1
            gaps += ops.count("I") + ops.count("D")
    assert n > 20 and gaps > 0


def one_seq_index(ggo, bank: bytes, k=5):
    seqs = np.frombuffer(bank, np.uint8).copy()
    return ggo.Index(seqs, np.array([0, len(bank)], np.int64), k)


def top_path(ggo, ix, q: bytes, prm):
    rc, hits, m, _ = ix.search(q, prm)
    assert rc == 0 and m >= 1
    return hits[0], ix.traceback(q, prm, hits[0])


def test_hand_worked_paths(ggo):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, 77])))
    x = rng.choice(list(b"ACG"), 60).astype(np.uint8).tobytes()  # no T: the T runs stay unique
    y = rng.choice(list(b"ACG"), 60).astype(np.uint8).tobytes()
    prm = ggo.params(5, max_gap=10, min_hsp_len=10)
    # exact copy
    bank = x + b"TTTTTT" + y
    ix = one_seq_index(ggo, bank)
    h, ops = top_path(ggo, ix, bank, prm)
    assert ops == "=" * len(bank) and int(h["score"]) == len(bank)
    # one substitution in the middle of the copy
    q = x + b"TTATTT" + y
    h, ops = top_path(ggo, ix, q, prm)
    assert ops == "=" * 62 + "X" + "=" * 63
    # the query lacks one T of the bank's run: the gap goes before the run's pairs
    q = x + b"TTTTT" + y
    h, ops = top_path(ggo, ix, q, prm)
    assert ops == "=" * 60 + "D" + "=" * 65
    assert int(h["score"]) == 125 - 7
    # the query has one T more than the bank's run
    q = x + b"TTTTTTT" + y
    h, ops = top_path(ggo, ix, q, prm)
    assert ops == "=" * 60 + "I" + "=" * 66
    # a two-base deletion costs open + 2 extend, and is one gap
    q = x + b"TTTT" + y
    h, ops = top_path(ggo, ix, q, prm)
    assert ops == "=" * 60 + "DD" + "=" * 64 and int(h["score"]) == 124 - 9


def test_not_an_alignment_is_refused(ggo):
    db = synth.small_db(n_seqs=100)
    qs = synth.small_queries(db)
    ix = ggo.Index(db.seqs, db.off, 11)
    prm = ggo.params(5)
    q = bytes(qs.query(0))
    rc, hits, m, _ = ix.search(q, prm)
    h = hits[0].copy()
    h["score"] += 1
    with pytest.raises(ValueError):
        ix.traceback(q, prm, h)
    h = hits[0].copy()
    h["q_end"] = len(q) + 1
    with pytest.raises(ValueError):
        ix.traceback(q, prm, h)
    h = hits[0].copy()
    h["seq_id"] = db.n_seqs
    with pytest.raises(ValueError):
        ix.traceback(q, prm, h)
