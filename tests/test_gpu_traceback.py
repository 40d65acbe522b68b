"""GPU traceback (gg_traceback) against the oracle's, byte for byte: every reported
hit of workloads with indels under several scoring schemes and bands (0, 5, the
default 32 whose 65 band slots spill into each lane's second slot, and 63), a
masked and a two-strand index, long alignments, and the error paths."""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


def compare_all(ggo, G, gix, oix, qs, prm_g, prm_o):
    n_hits = n_gaps = 0
    for i in range(qs.n):
        q = bytes(qs.query(i))
        rc, hits, n = gix.search(q, prm_g, cap=1000)
        assert rc == 0
        if n == 0:
            continue
        rc, ops = gix.traceback(q, prm_g, hits)
        assert rc == G.GG_OK, G.STATUS[rc]
        for h, got in zip(hits, ops):
            want = oix.traceback(q, prm_o, tuple(int(x) for x in h.tolist()))
            assert got == want, (i, tuple(h.tolist()))
            n_gaps += got.count("I") + got.count("D")
        n_hits += n
    return n_hits, n_gaps


@pytest.mark.parametrize("kw,seed", [(dict(), 81), (dict(band=0), 82), (dict(band=5), 83),
                                     (dict(band=63), 84),
                                     (dict(match=2, mismatch=1, gap_open=1, gap_extend=1), 85),
                                     (dict(gap_open=0, gap_extend=3, band=17), 86)])
def test_traceback_matches_oracle(ggo, kw, seed):
    G = gpu()
    db = synth.random_db(seed, n_seqs=200, lmin=0, lmax=2500)
    qs = synth.random_queries(seed, db, n=30, lmin=20, lmax=1500, frac_homolog=0.9,
                              ident_lo=0.8, ident_hi=0.99, indel_rate=0.03)
    gix, oix = G.Index(db.seqs, db.off, 8), ggo.Index(db.seqs, db.off, 8)
    n_hits, n_gaps = compare_all(ggo, G, gix, oix, qs, G.params(0, max_gap=16, min_hsp_len=16, **kw),
                                 ggo.params(0, max_gap=16, min_hsp_len=16, **kw))
    assert n_hits > 30
    if kw.get("band", 32) > 0:
        assert n_gaps > 0


@pytest.mark.parametrize("kw", [dict(mask="111010010100110111"), dict(strands=2)])
def test_traceback_on_index_options(ggo, kw):
    G = gpu()
    db = synth.random_db(87, n_seqs=200, lmin=0, lmax=2500)
    qs = synth.random_queries(87, db, n=30, lmin=20, lmax=1500, frac_homolog=0.9,
                              ident_lo=0.85, ident_hi=0.99, indel_rate=0.02)
    k = 0 if "mask" in kw else 11
    gix, oix = G.Index(db.seqs, db.off, k, **kw), ggo.Index(db.seqs, db.off, k, **kw)
    n_hits, _ = compare_all(ggo, G, gix, oix, qs, G.params(10), ggo.params(10))
    assert n_hits > 10


def test_long_alignments(ggo):
    G = gpu()
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, 88])))
    bank = rng.choice(list(b"ACGT"), 12_000).astype(np.uint8)
    off = np.array([0, len(bank)], np.int64)
    src = bank[2_000:7_000]
    q = synth.mutate(src, 0.03, 0.0005, rng)
    gix, oix = G.Index(bank, off, 11), ggo.Index(bank, off, 11)
    rc, hits, n = gix.search(q.tobytes(), G.params(5), cap=10)
    assert rc == 0 and n >= 1 and int(hits[0]["q_end"] - hits[0]["q_start"]) > 3_000
    rc, ops = gix.traceback(q.tobytes(), G.params(5), hits[:n])
    assert rc == 0
    for h, got in zip(hits[:n], ops):
        assert got == oix.traceback(q.tobytes(), ggo.params(5), tuple(int(x) for x in h.tolist()))


def test_traceback_errors(ggo):
    G = gpu()
    db = synth.small_db(n_seqs=200)
    qs = synth.small_queries(db)
    gix = G.Index(db.seqs, db.off, 11)
    q = bytes(qs.query(0))
    prm = G.params(5)
    rc, hits, n = gix.search(q, prm, cap=10)
    assert rc == 0 and n >= 2
    hits = hits[:n].copy()
    # a wrong score: that hit is refused, the others are still traced
    bad = hits.copy()
    bad["score"][0] += 1
    rc, ops = gix.traceback(q, prm, bad)
    assert rc == G.GG_EINVAL and ops[0] == "" and all(len(o) > 0 for o in ops[1:])
    # a hit outside the query is refused before any GPU work
    bad = hits.copy()
    bad["q_end"][0] = len(q) + 5
    assert gix.traceback(q, prm, bad)[0] == G.GG_EINVAL
    # a bank span past its sequence is refused on the device
    bad = hits.copy()
    bad["d_end"][0] = 10 ** 8
    rc, ops = gix.traceback(q, prm, bad)
    assert rc == G.GG_EINVAL and ops[0] == ""
    # too small an output buffer
    h = np.ascontiguousarray(hits)
    off = np.zeros(n + 1, np.int64)
    ln = np.zeros(n, np.int32)
    buf = np.zeros(4, np.uint8)
    qa = np.frombuffer(q, np.uint8).copy()
    rc = G.lib().gg_traceback(gix.handle, G._ptr(qa), len(qa), G.C.byref(prm), G._ptr(h), n,
                              G._ptr(buf), 4, G._ptr(off), G._ptr(ln))
    assert rc == G.GG_ETRUNC and off[n] == int(((h["q_end"] - h["q_start"]) +
                                                (h["d_end"] - h["d_start"])).sum())
