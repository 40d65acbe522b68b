"""Pins of the oracle's two index options: both strands and the repeat cutoff.

Both strands: sequence n + s of the index is the reverse complement of sequence s.
* the index equals the plain index over the bank followed by reverse complements
  computed here with a byte translation table;
* a query that is the reverse complement of a bank region is found whole on
  sequence n + s, at the region's mirrored coordinates, with the score of an exact
  copy; the one-strand index does not find it;
* the bank and its reverse complement hold the same 2n strands with ids swapped,
  so every query's full result set is the same up to that swap.

Repeat cutoff (max_posting): lists longer than the cutoff are dropped whole.
* lists equal a brute-force dictionary of the windows with long lists removed;
* hits equal the plain index's hits on the query windows whose list is kept;
* a cutoff at or above the longest list gives the plain index.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

COMP = bytes.maketrans(b"ACGTUacgtu", b"TGCAAtgcaa")


def revcomp(b: bytes) -> bytes:
    return bytes(b).translate(COMP)[::-1]


def base4(window: bytes) -> int:
    v = 0
    for ch in window.upper():
        v = v * 4 + "ACGT".index(chr(ch).replace("U", "T"))
    return v


def both_strand_bank(db):
    parts = [bytes(db.seq(s)) for s in range(db.n_seqs)]
    parts += [revcomp(p) for p in parts]
    off = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([len(p) for p in parts], out=off[1:])
    return np.frombuffer(b"".join(parts), np.uint8).copy(), off


@pytest.mark.parametrize("k,mask", [(5, None), (11, None), (0, "1101")])
def test_both_strand_index_is_the_bank_plus_reverse_complements(ggo, k, mask):
    db = synth.random_db(21, n_seqs=40, lmin=0, lmax=400)
    seqs2, off2 = both_strand_bank(db)
    a = ggo.Index(db.seqs, db.off, k, mask=mask, strands=2)
    b = ggo.Index(seqs2, off2, k, mask=mask)
    assert a.strands == 2 and a.n_seqs == 2 * db.n_seqs
    assert np.array_equal(a.list_off(), b.list_off())
    for x, y in zip(a.postings(), b.postings()):
        assert np.array_equal(x, y)


def test_reverse_complement_query_found_on_the_reverse_strand(ggo):
    db = synth.small_db(n_seqs=200)
    n = db.n_seqs
    ix2 = ggo.Index(db.seqs, db.off, 11, strands=2)
    ix1 = ggo.Index(db.seqs, db.off, 11)
    src = next(s for s in range(n) if len(db.seq(s)) >= 700)
    n_s = len(db.seq(src))
    q = revcomp(bytes(db.seq(src)[100:700]))
    rc, h, m, st = ix2.search(q, ggo.params(5))
    assert rc == 0 and m >= 1
    top = h[0]
    assert (int(top["seq_id"]), int(top["score"])) == (n + src, 600)
    assert (int(top["q_start"]), int(top["q_end"])) == (0, 600)
    assert (int(top["d_start"]), int(top["d_end"])) == (n_s - 700, n_s - 100)
    assert st["n_kmers"] == 600 - 11 + 1
    rc, h1, m1, _ = ix1.search(q, ggo.params(5))
    assert rc == 0 and all(int(x["score"]) < 100 for x in h1)
    # the forward copy of the region is found on the forward strand
    rc, hf, mf, _ = ix2.search(bytes(db.seq(src)[100:700]), ggo.params(5))
    assert (int(hf[0]["seq_id"]), int(hf[0]["score"]), int(hf[0]["d_start"])) == (src, 600, 100)


def test_strand_swap_symmetry(ggo):
    db = synth.random_db(22, n_seqs=60, lmin=0, lmax=800)
    qs = synth.random_queries(22, db, n=12, lmin=20, lmax=500, frac_homolog=0.9,
                              ident_lo=0.85, ident_hi=1.0, indel_rate=0.01)
    rparts = [revcomp(bytes(db.seq(s))) for s in range(db.n_seqs)]
    roff = np.zeros(db.n_seqs + 1, np.int64)
    np.cumsum([len(p) for p in rparts], out=roff[1:])
    rseqs = np.frombuffer(b"".join(rparts), np.uint8).copy()
    n = db.n_seqs
    a = ggo.Index(db.seqs, db.off, 8, strands=2)
    b = ggo.Index(rseqs, roff, 8, strands=2)
    prm = ggo.params(0, max_gap=16, min_hsp_len=16)
    found = 0
    for i in range(qs.n):
        ra, rb = a.search(qs.query(i), prm), b.search(qs.query(i), prm)
        assert ra[0] == rb[0] == 0
        swap = lambda s: s + n if s < n else s - n  # noqa: E731
        ta = sorted(tuple(int(x) for x in r) for r in ra[1].tolist())
        tb = sorted((swap(int(r[0])),) + tuple(int(x) for x in r[1:]) for r in rb[1].tolist())
        assert ta == tb
        for f in ("n_hits", "n_cands", "n_merged", "n_cells"):
            assert ra[3][f] == rb[3][f]
        found += len(ta)
    assert found > 0


def brute_lists(db, k):
    lists = {}
    for s in range(db.n_seqs):
        b = bytes(db.seq(s))
        for pos in range(0, len(b) - k + 1, k):
            lists.setdefault(base4(b[pos:pos + k]), []).append((s, pos))
    return lists


@pytest.mark.parametrize("k,cut", [(4, 3), (4, 12), (6, 2), (6, 5)])
def test_cutoff_lists_brute_force(ggo, k, cut):
    db = synth.repeat_db(23, n_seqs=60, lmin=0, lmax=500)
    lists = brute_lists(db, k)
    assert max(len(v) for v in lists.values()) > cut  # some list is dropped
    ix = ggo.Index(db.seqs, db.off, k, max_posting=cut)
    off = ix.list_off()
    seq, pos = ix.postings()
    assert ix.n_post == sum(len(v) for v in lists.values() if len(v) <= cut)
    for c in range(4 ** k):
        want = lists.get(c, [])
        got = list(zip(seq[off[c]:off[c + 1]].tolist(), pos[off[c]:off[c + 1]].tolist()))
        assert got == (want if len(want) <= cut else []), c


@pytest.mark.parametrize("strands", [1, 2])
def test_cutoff_hits_are_the_kept_windows_hits(ggo, strands):
    k, cut = 6, 4
    db = synth.repeat_db(24, n_seqs=50, lmin=0, lmax=600)
    qs = synth.random_queries(24, db, n=10, lmin=10, lmax=300, frac_homolog=1.0,
                              ident_lo=0.9, ident_hi=1.0, indel_rate=0.0)
    plain = ggo.Index(db.seqs, db.off, k, strands=strands)
    cutix = ggo.Index(db.seqs, db.off, k, strands=strands, max_posting=cut)
    plen = np.diff(plain.list_off())
    dropped = 0
    for i in range(qs.n):
        q = bytes(qs.query(i))
        hp = plain.hits(ggo.encode(q))
        hc = cutix.hits(ggo.encode(q))
        keep = [plen[base4(q[t:t + k])] <= cut for t in range(len(q) - k + 1)]
        want = sorted((int(s), int(d), int(p)) for s, d, p in
                      zip(hp["seq"], hp["diag"], hp["qpos"]) if keep[p])
        got = sorted(zip(hc["seq"].tolist(), hc["diag"].tolist(), hc["qpos"].tolist()))
        assert got == want
        dropped += len(hp) - len(hc)
    assert dropped > 0


def test_cutoff_above_longest_list_is_the_plain_index(ggo):
    db = synth.repeat_db(25, n_seqs=40, lmin=0, lmax=500)
    qs = synth.random_queries(25, db, n=8, lmin=20, lmax=300, frac_homolog=1.0,
                              ident_lo=0.9, ident_hi=1.0, indel_rate=0.01)
    a = ggo.Index(db.seqs, db.off, 7)
    top = int(np.diff(a.list_off()).max())
    b = ggo.Index(db.seqs, db.off, 7, max_posting=top)
    assert np.array_equal(a.list_off(), b.list_off())
    prm = ggo.params(10, max_gap=14, min_hsp_len=14)
    for i in range(qs.n):
        ra, rb = a.search(qs.query(i), prm), b.search(qs.query(i), prm)
        assert ra[1].tobytes() == rb[1].tobytes()
    c = ggo.Index(db.seqs, db.off, 7, max_posting=top - 1)
    assert c.n_post < a.n_post


def test_bad_options(ggo):
    db = synth.random_db(26, n_seqs=5, lmin=10, lmax=50)
    for kw in (dict(strands=0), dict(strands=3), dict(max_posting=-1)):
        with pytest.raises(ValueError):
            ggo.Index(db.seqs, db.off, 5, **kw)
    bad = db.seqs.copy()
    bad[3] = ord("N")
    with pytest.raises(ValueError):
        ggo.Index(bad, db.off, 5, strands=2)
