"""GPU parity of spaced-seed masks (Section 2.1) against the oracle, bit-exact.

The masked index (windows of the mask's length m at multiples of m, coded on the
bases under its 1s) and the masked search (overlapping query windows of m bases,
runs and lengths measured with m) must give the oracle's postings, hits, work
counts and report under every grouping strategy, in the graph-replayed form and
in the served form; an all-ones mask must equal the plain index.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu

PAPER_MASK = "111010010100110111"
FIELDS = ("n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out")


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


def as_rows(a):
    return [tuple(int(x) for x in r) for r in a.tolist()]


def oracle_all(oix, qs, prm_o, cap=100000):
    res, stats = [], []
    for i in range(qs.n):
        rc, h, n, st = oix.search(qs.query(i), prm_o, cap=cap)
        assert rc == 0
        res.append(h)
        stats.append(st)
    return res, stats


def check_batch(G, gix, qs, prm, want, wst, cap=100000, stats=True):
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm, cap=cap, stats=stats)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"
        if stats:
            for f in FIELDS:
                assert int(st[i][f]) == wst[i][f], (i, f)


def workload(seed, n_seqs=300, n_q=40):
    db = synth.random_db(seed, n_seqs=n_seqs, lmin=0, lmax=3000)
    qs = synth.random_queries(seed, db, n=n_q, lmin=0, lmax=1500, frac_homolog=0.8,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    return db, qs


@pytest.mark.parametrize("mask,seed,n_seqs,n_q", [
    (PAPER_MASK, 31, 300, 40), ("1101", 32, 100, 40), ("0110111", 33, 300, 40),
    ("1" * 9 + "0", 34, 300, 40), ("11", 35, 20, 10)])
def test_masked_index_and_search(ggo, monkeypatch, mask, seed, n_seqs, n_q):
    G = gpu()
    db, qs = workload(seed, n_seqs, n_q)
    oix, gix = ggo.Index(db.seqs, db.off, mask=mask), G.Index(db.seqs, db.off, mask=mask)
    info = gix.info()
    assert info["n_postings"] == oix.n_post and info["k"] == mask.count("1")
    m = len(mask)
    for kw in (dict(), dict(max_gap=3 * m, min_hsp_len=2 * m), dict(max_gap=0, min_hsp_len=m)):
        want, wst = oracle_all(oix, qs, ggo.params(20, **kw))
        for grouping in ("sort", "bucket", "probe"):
            monkeypatch.setenv("GG_GROUPING", grouping)
            check_batch(G, gix, qs, G.params(20, **kw), want, wst)


def test_all_ones_mask_equals_plain_index(monkeypatch):
    G = gpu()
    db, qs = workload(36)
    a, b = G.Index(db.seqs, db.off, 11), G.Index(db.seqs, db.off, mask="1" * 11)
    assert a.info() == b.info()
    monkeypatch.setenv("GG_GROUPING", "sort")
    prm = G.params(20)
    ra, rb = a.search_batch(qs.buf, qs.off, prm, stats=True), b.search_batch(qs.buf, qs.off, prm,
                                                                           stats=True)
    assert ra[0] == rb[0] == 0
    for i in range(qs.n):
        assert as_rows(ra[1][i]) == as_rows(rb[1][i])
        assert all(int(ra[3][i][f]) == int(rb[3][i][f]) for f in FIELDS)


def test_masked_graph_and_served_forms(ggo, monkeypatch):
    """Batches without statistics replay one captured graph per index; a masked
    index captures its own (its window span and mask are part of the graph), and
    the served form reads the same index."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db, qs = workload(37)
    oix = ggo.Index(db.seqs, db.off, mask=PAPER_MASK)
    gix = G.Index(db.seqs, db.off, mask=PAPER_MASK)
    plain = G.Index(db.seqs, db.off, 11)
    want, wst = oracle_all(oix, qs, ggo.params(10))
    prm = G.params(10)
    gix.profile(True)
    plain.search_batch(qs.buf, qs.off, prm, cap=1000)
    check_batch(G, gix, qs, prm, want, wst, cap=1000, stats=False)
    assert gix.profile_read("graph")["units"] >= 1
    gix.set_hit_budget(16 * max(max(int(s["n_hits"]) for s in wst), 1))
    check_batch(G, gix, qs, prm, want, wst, cap=1000, stats=False)
    gix.set_hit_budget(0)
    gix.profile(False)
    sv = G.Server(gix, prm, max_slots=8)
    try:
        tickets = [sv.submit(qs.query(i)) for i in range(qs.n)]
        for i, t in enumerate(tickets):
            rc, h, n = sv.poll(t, cap=1000, timeout_us=-1)
            assert rc == 0 and as_rows(h) == as_rows(want[i])
    finally:
        sv.close()


def test_masked_exact_copy_and_edges(ggo):
    G = gpu()
    db = synth.small_db(n_seqs=200)
    gix = G.Index(db.seqs, db.off, mask=PAPER_MASK)
    oix = ggo.Index(db.seqs, db.off, mask=PAPER_MASK)
    src = next(s for s in range(db.n_seqs) if len(db.seq(s)) >= 700)
    q = bytes(db.seq(src)[100:700])
    rc, h, n = gix.search(q, G.params(5))
    assert rc == 0 and n >= 1
    assert (int(h[0]["seq_id"]), int(h[0]["score"]), int(h[0]["q_start"]), int(h[0]["q_end"]),
            int(h[0]["d_start"]), int(h[0]["d_end"])) == (src, 600, 0, 600, 100, 700)
    # queries shorter than the mask, exactly its length, and one base longer
    for p in (b"", b"ACGT" * 4 + b"A", q[:18], q[:19]):
        orc, oh, on, _ = oix.search(p, ggo.params(5))
        rc, gh, gn = gix.search(p, G.params(5))
        assert rc == orc == 0 and as_rows(gh) == as_rows(oh)


def test_bad_masks_rejected():
    G = gpu()
    db = synth.random_db(6, n_seqs=5, lmin=10, lmax=50)
    for bad in ["", "0000", "12", "1" * 17, "1" + "0" * 40 + "1"]:
        with pytest.raises(G.GGError):
            G.Index(db.seqs, db.off, mask=bad)


@pytest.mark.parametrize("grouping", ["sort", "bucket", "probe"])
def test_paper_mask_on_the_bank_workload(ggo, monkeypatch, grouping):
    """The paper's mask on the bank-like workload (many hit tiles per query), whole
    and with a hit budget that cuts the largest queries into sequence ranges."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", grouping)
    db = synth.mid_db(n_seqs=20_000)
    qs = synth.mid_queries(db, n=60)
    oix = ggo.Index(db.seqs, db.off, mask=PAPER_MASK)
    gix = G.Index(db.seqs, db.off, mask=PAPER_MASK)
    for kw in (dict(), dict(max_gap=54, min_hsp_len=36)):
        want, wst = oracle_all(oix, qs, ggo.params(50, **kw))
        check_batch(G, gix, qs, G.params(50, **kw), want, wst)
        hits = max(int(s["n_hits"]) for s in wst)
        gix.set_hit_budget(16 * (hits // 5))
        check_batch(G, gix, qs, G.params(50, **kw), want, wst)
        gix.set_hit_budget(0)
