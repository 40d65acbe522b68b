"""End-to-end pins for the oracle's search (Section 2.2, all seven phases).

* sensitivity: every planted homolog of the small uniform workload (2,000
  sequences, 500 bp queries at 95% identity) whose full, unbanded Smith-Waterman
  score against its source region is >= 50 is reported in its top 20, on its
  source sequence, overlapping the source region;
* uniform random queries report nothing;
* the phases composed by hand from the stage functions give the same result;
* input errors, short queries, truncation and determinism.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth


@pytest.fixture(scope="module")
def c0(ggo):
    db = synth.small_db()
    q = synth.small_queries(db)
    return db, q, ggo.Index(db.seqs, db.off, 11)


def test_planted_homologs_found(ggo, c0):
    db, qs, ix = c0
    prm = ggo.params(20)
    full = ggo.params(0, band=100_000)
    checked = 0
    for i in range(qs.n):
        if not qs.kind[i]:
            continue
        q = qs.query(i)
        s, a, b = int(qs.src_seq[i]), int(qs.src_start[i]), int(qs.src_end[i])
        qc = ggo.encode(q)
        sc = ix.seq_codes(s)
        ref, _ = ggo.bsw(qc, sc, (s, 0, len(qc), a, b, a, a), full)
        rc, res, n, _ = ix.search(q, prm)
        assert rc == 0
        if ref["score"] < 50:
            continue
        checked += 1
        on_src = res[(res["seq_id"] == s) & (res["d_start"] < b) & (res["d_end"] > a)]
        assert len(on_src) >= 1, i
        # indels split a homolog into ungapped boxes; each sits on the true diagonal band
        assert np.all(np.abs((on_src["d_start"] - a) - on_src["q_start"]) <= 3 * 4)
    assert checked == 10


def test_random_queries_report_nothing(ggo, c0):
    db, qs, ix = c0
    prm = ggo.params(20)
    for i in range(qs.n):
        if qs.kind[i]:
            continue
        rc, res, n, st = ix.search(qs.query(i), prm)
        assert rc == 0 and n == 0
        assert st["n_hits"] > 0  # chance k-mer hits exist but never chain


def test_composed_stages_equal_search(ggo, c0):
    db, qs, ix = c0
    prm = ggo.params(20)
    for i in range(0, qs.n, 3):
        q = qs.query(i)
        qc = ggo.encode(q)
        hits = ggo.group(ix.hits(qc))
        cands = ggo.chain(hits, 11, prm.max_gap, prm.min_hsp_len)
        bx = [ggo.extend(qc, ix.seq_codes(int(c["seq"])), c, prm) for c in cands]
        bx = np.array(bx, dtype=ggo.BOX_DTYPE) if bx else np.zeros(0, ggo.BOX_DTYPE)
        sel = ggo.select(ggo.merge(bx), prm.max_hits)
        out = [ggo.bsw(qc, ix.seq_codes(int(b["seq"])), b, prm)[0] for b in sel]
        out = ggo.report(np.array(out, dtype=ggo.HIT_DTYPE)) if out else np.zeros(0, ggo.HIT_DTYPE)
        rc, res, n, _ = ix.search(q, prm)
        assert rc == 0 and n == len(out)
        assert res.tobytes() == out.tobytes()


def test_edge_cases(ggo, c0):
    db, qs, ix = c0
    prm = ggo.params(20)
    rc, res, n, _ = ix.search(b"ACGTACGTAC", prm)  # shorter than k
    assert (rc, n) == (0, 0)
    rc, res, n, _ = ix.search(b"", prm)
    assert (rc, n) == (0, 0)
    rc, res, n, _ = ix.search(b"ACGTNACGTACGTACGT", prm)
    assert rc == 1
    q = qs.query(0)
    rc, full, n, _ = ix.search(q, prm)
    assert rc == 0 and n >= 2
    rc, part, n2, _ = ix.search(q, prm, cap=1)
    assert rc == 5 and n2 == n and part.tobytes() == full[:1].tobytes()
    # N <= 0 keeps every box
    rc, every, n_all, st = ix.search(q, ggo.params(0))
    assert rc == 0 and n_all >= n and st["n_selected"] == st["n_merged"]
    # lowercase and U are the same letters
    low = bytes(q).lower().replace(b"t", b"u")
    rc, same, _, _ = ix.search(low, prm)
    assert same.tobytes() == full.tobytes()


def test_deterministic(ggo, c0):
    db, qs, ix = c0
    prm = ggo.params(20)
    a = [ix.search(qs.query(i), prm)[1].tobytes() for i in range(qs.n)]
    b = [ix.search(qs.query(i), prm)[1].tobytes() for i in range(qs.n)]
    assert a == b
