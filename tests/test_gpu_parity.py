"""GPU parity: the HIP path (through the C ABI) against the oracle, bit-exact.

Every integer field of every reported hit, the hit order and the per-query work
counts must be identical.  Inputs are the seeded synthetic workloads; sizes span
several gather / sort tiles with ragged tails, plus edge cases.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


def as_rows(a):
    return [tuple(int(x) for x in r) for r in a.tolist()]


def oracle_all(ggo, oix, qs, prm_o, cap=100000):
    res, stats = [], []
    for i in range(qs.n):
        rc, h, n, st = oix.search(qs.query(i), prm_o, cap=cap)
        assert rc == 0
        res.append(h)
        stats.append(st)
    return res, stats


def check_batch(G, gix, qs, prm_g, want, want_stats, cap=100000):
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm_g, cap=cap, stats=True)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"
        for f in ("n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out"):
            assert int(st[i][f]) == want_stats[i][f], (i, f)


@pytest.fixture(scope="module")
def c0(ggo):
    G = gpu()
    db = synth.small_db()
    qs = synth.small_queries(db)
    return G, db, qs, G.Index(db.seqs, db.off, 11), ggo.Index(db.seqs, db.off, 11)


def test_small_batch_and_single(ggo, c0):
    G, db, qs, gix, oix = c0
    want, wst = oracle_all(ggo, oix, qs, ggo.params(20))
    check_batch(G, gix, qs, G.params(20), want, wst)
    for i in range(qs.n):
        rc, h, n = gix.search(qs.query(i), G.params(20), cap=1000)
        assert rc == 0 and as_rows(h) == as_rows(want[i])
    info = gix.info()
    assert info["n_postings"] == oix.n_post and info["k"] == 11


@pytest.mark.parametrize("k,band,max_hits,seed", [
    (4, 32, 20, 1), (6, 5, 0, 2), (8, 0, 3, 3), (11, 63, 50, 4), (12, 32, 1, 5), (7, 17, -1, 6),
    (4, 10, 0, 7)])
def test_random_banks(ggo, k, band, max_hits, seed):
    G = gpu()
    db = synth.random_db(seed, n_seqs=300, lmin=0, lmax=3000)
    qs = synth.random_queries(seed, db, n=40, lmin=0, lmax=1500, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix, gix = ggo.Index(db.seqs, db.off, k), G.Index(db.seqs, db.off, k)
    kw = dict(band=band, max_gap=3 * k - 2 * (seed % 2), min_hsp_len=2 * k)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(max_hits, **kw))
    check_batch(G, gix, qs, G.params(max_hits, **kw), want, wst)
    if k == 4:  # more than one LDS segment of runs per query: the global-sort paths ran
        assert max(s["n_cands"] for s in wst) > 1024
        if max_hits <= 0:
            assert max(s["n_selected"] for s in wst) > 1024


def test_scoring_variants(ggo, c0):
    G, db, qs, gix, oix = c0
    for kw in (dict(match=2, mismatch=1, gap_open=1, gap_extend=1, xdrop=10),
               dict(match=1, mismatch=1, gap_open=0, gap_extend=3, xdrop=5, max_gap=0,
                    min_hsp_len=11),
               dict(max_gap=100, min_hsp_len=0, band=1)):
        want, wst = oracle_all(ggo, oix, qs, ggo.params(7, **kw))
        check_batch(G, gix, qs, G.params(7, **kw), want, wst)


def test_waves_under_small_budget(ggo, monkeypatch):
    """With stored hits (radix-sort grouping), a small hit budget forces one query
    per wave, then cuts the largest queries into ranges of sequences; results
    must not change.  Only a single sequence over the budget is refused."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    db = synth.mid_db(n_seqs=20_000)
    qs = synth.mid_queries(db, n=60)
    oix, gix = ggo.Index(db.seqs, db.off, 11), G.Index(db.seqs, db.off, 11)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(50))
    check_batch(G, gix, qs, G.params(50), want, wst)
    hits = max(int(s["n_hits"]) for s in wst)
    gix.set_hit_budget(16 * hits)
    check_batch(G, gix, qs, G.params(50), want, wst)
    gix.set_hit_budget(16 * (hits // 7))
    check_batch(G, gix, qs, G.params(50), want, wst)
    gix.set_hit_budget(16)
    rc, _, _, _ = gix.search_batch(qs.buf, qs.off, G.params(50))
    assert rc == G.GG_EBUDGET


@pytest.mark.parametrize("grouping", ["probe", "bucket", "sort"])
def test_pieces_by_sequence_range(ggo, monkeypatch, grouping):
    """Queries over the hit budget are searched in ranges of sequence ids (with
    every grouping strategy, all boxes kept or the top 3, host and device
    results); the merged selection equals the unsplit oracle."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", grouping)
    db = synth.random_db(12, n_seqs=500, lmin=50, lmax=3000)
    qs = synth.random_queries(12, db, n=24, lmin=100, lmax=2500, frac_homolog=0.8,
                              ident_lo=0.85, ident_hi=1.0, indel_rate=0.01)
    oix, gix = ggo.Index(db.seqs, db.off, 6), G.Index(db.seqs, db.off, 6)
    for top in (3, 0):
        want, wst = oracle_all(ggo, oix, qs, ggo.params(top))
        hits = max(int(s["n_hits"]) for s in wst)
        gix.set_hit_budget(16 * (hits // 9))
        check_batch(G, gix, qs, G.params(top), want, wst)
    cap = 4
    dq = G.DeviceBuffer(len(qs.buf))
    dq.upload(qs.buf)
    dout = G.DeviceBuffer(qs.n * cap * G.HIT_DTYPE.itemsize)
    dn = G.DeviceBuffer(qs.n * 4)
    rc, st = gix.search_batch_device(dq, qs.off, G.params(0), dout, dn, cap, stats=True)
    assert rc in (G.GG_OK, G.GG_ETRUNC)
    n = dn.download(np.zeros(qs.n, np.int32))
    got = dout.download(np.zeros(qs.n * cap, G.HIT_DTYPE))
    for i in range(qs.n):
        assert int(n[i]) == len(want[i])
        m = min(cap, len(want[i]))
        assert as_rows(got[i * cap: i * cap + m]) == as_rows(want[i][:m])


def test_edge_cases(ggo, c0):
    G, db, qs, gix, oix = c0
    prm = G.params(20)
    # empty batch, empty query, shorter than k, lowercase and U
    rc, res, n, _ = gix.search_batch(b"", np.array([0]), prm)
    assert rc == 0 and len(res) == 0
    parts = [b"", b"ACGTACGTAC", bytes(qs.query(0)).lower().replace(b"t", b"u"), b"A" * 11,
             bytes(qs.query(3))]
    off = np.cumsum([0] + [len(p) for p in parts])
    rc, res, n, _ = gix.search_batch(b"".join(parts), off, prm)
    assert rc == 0
    for i, p in enumerate(parts):
        orc, oh, on, _ = oix.search(p, ggo.params(20))
        assert as_rows(res[i]) == as_rows(oh)
    # bad byte anywhere fails the call
    rc, _, _ = gix.search(b"ACGTNACGTACGTACGTAC", prm)
    assert rc == G.GG_EINVAL
    # truncation: first cap hits, full count
    rc, full, nfull = gix.search(qs.query(0), prm, cap=1000)
    assert rc == 0 and nfull >= 2
    rc, part, n = gix.search(qs.query(0), prm, cap=1)
    assert rc == G.GG_ETRUNC and n == nfull and as_rows(part) == as_rows(full[:1])
    # parameters outside the supported range
    assert gix.search(qs.query(0), G.params(20, band=64))[0] == G.GG_EINVAL
    assert gix.search(qs.query(0), G.params(20, match=0))[0] == G.GG_EINVAL


def test_index_build_errors():
    G = gpu()
    with pytest.raises(G.GGError):
        G.Index(b"ACGTN", np.array([0, 5]), 3)
    with pytest.raises(G.GGError):
        G.Index(b"ACGT", np.array([0, 4]), 17)
    ix = G.Index(b"ACGTACGT" * 4, np.array([0, 0, 3, 32]), 3)  # empty and short sequences
    assert ix.info()["n_postings"] == 10


def test_deterministic_repeat(c0):
    G, db, qs, gix, oix = c0
    a = gix.search_batch(qs.buf, qs.off, G.params(20))[1]
    b = gix.search_batch(qs.buf, qs.off, G.params(20))[1]
    assert all(x.tobytes() == y.tobytes() for x, y in zip(a, b))


def test_server_matches_plain(c0):
    G, db, qs, gix, oix = c0
    prm = G.params(20)
    want = [gix.search(qs.query(i), prm, cap=1000)[1] for i in range(qs.n)]
    sv = G.Server(gix, prm, max_slots=8)
    try:
        tickets = [sv.submit(qs.query(i)) for i in range(qs.n)]
        for i, t in enumerate(tickets):
            rc, h, n = sv.poll(t, cap=1000, timeout_us=-1)
            assert rc == 0 and as_rows(h) == as_rows(want[i])
        assert sv.poll(tickets[0], timeout_us=0)[0] == G.GG_ENOTFOUND
    finally:
        sv.close()


@pytest.mark.slow
def test_mid_full_bank_every_query(ggo):
    """The mid-size workload exactly as the benchmark's device-resident leg runs it:
    the 200,000-sequence bank, all 1,000 queries in one gg_search_batch_device call
    (no statistics, so every wave is a replay of the captured graph, with the
    lone-diagonal filter), launch choices sort / 16 lane steps.  Every hit of every
    query equals the oracle's; the work counts of a call with statistics equal the
    oracle's too."""
    from concurrent.futures import ThreadPoolExecutor

    G = gpu()
    db = synth.mid_db()
    qs = synth.mid_queries(db)
    gix = G.Index(db.seqs, db.off, 11)
    gix.set_tuning("sort", 256)
    cap = 50
    dq = G.DeviceBuffer(len(qs.buf))
    dq.upload(qs.buf)
    dout = G.DeviceBuffer(qs.n * cap * G.HIT_DTYPE.itemsize)
    dn = G.DeviceBuffer(qs.n * 4)
    gix.profile(True)
    rc, _ = gix.search_batch_device(dq, qs.off, G.params(50), dout, dn, cap)
    waves = gix.profile_read("graph")["units"]
    gix.profile(False)
    assert rc in (G.GG_OK, G.GG_ETRUNC) and waves >= 1
    n = dn.download(np.zeros(qs.n, np.int32))
    got = dout.download(np.zeros(qs.n * cap, G.HIT_DTYPE))
    rc, _, n2, st = gix.search_batch(qs.buf, qs.off, G.params(50), cap=cap, stats=True)
    assert rc in (G.GG_OK, G.GG_ETRUNC) and np.array_equal(n, n2)
    oix = ggo.Index(db.seqs, db.off, 11)
    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(lambda i: oix.search(qs.query(i), ggo.params(50), cap=cap),
                          range(qs.n)))
    for i, (orc, oh, on, ost) in enumerate(res):
        assert orc in (0, 5) and on == int(n[i]), i
        m = min(cap, on)
        assert as_rows(got[i * cap: i * cap + m]) == as_rows(oh), i
        for f in ("n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out"):
            assert int(st[i][f]) == ost[f], (i, f)
    for b in (dq, dout, dn):
        b.close()


def test_device_resident_form(ggo, c0):
    """gg_search_batch_device (queries and hits in GPU memory) equals the oracle."""
    G, db, qs, gix, oix = c0
    want, wst = oracle_all(ggo, oix, qs, ggo.params(20))
    cap = 8
    dq = G.DeviceBuffer(len(qs.buf))
    dq.upload(qs.buf)
    dout = G.DeviceBuffer(qs.n * cap * G.HIT_DTYPE.itemsize)
    dn = G.DeviceBuffer(qs.n * 4)
    for rep in range(2):  # the second call reuses the workspace
        rc, st = gix.search_batch_device(dq, qs.off, G.params(20), dout, dn, cap, stats=True)
        assert rc in (G.GG_OK, G.GG_ETRUNC)
        n = dn.download(np.zeros(qs.n, np.int32))
        got = dout.download(np.zeros(qs.n * cap, G.HIT_DTYPE))
        for i in range(qs.n):
            assert int(n[i]) == len(want[i])
            m = min(cap, len(want[i]))
            assert as_rows(got[i * cap: i * cap + m]) == as_rows(want[i][:m])
            assert int(st[i]["n_cells"]) == wst[i]["n_cells"]
        assert (rc == G.GG_ETRUNC) == any(len(w) > cap for w in want)


@pytest.mark.parametrize("grouping", ["probe", "bucket", "sort", "sort-onesweep"])
def test_grouping_strategies_agree(ggo, monkeypatch, grouping):
    """Runs found by probing neighbour windows, by sorting hits in LDS slices, or
    by global radix sorting (the default; per-pass histograms or one-sweep
    look-back) are the same runs."""
    G = gpu()
    db = synth.random_db(11, n_seqs=400, lmin=50, lmax=4000)
    qs = synth.random_queries(11, db, n=30, lmin=100, lmax=3000, frac_homolog=0.8,
                              ident_lo=0.85, ident_hi=1.0, indel_rate=0.01)
    oix, gix = ggo.Index(db.seqs, db.off, 8), G.Index(db.seqs, db.off, 8)
    for kw in (dict(), dict(max_gap=0, min_hsp_len=8), dict(max_gap=40, min_hsp_len=30)):
        want, wst = oracle_all(ggo, oix, qs, ggo.params(10, **kw))
        monkeypatch.setenv("GG_GROUPING", grouping.split("-")[0])
        monkeypatch.setenv("GG_SORT", "onesweep" if grouping.endswith("onesweep") else "classic")
        check_batch(G, gix, qs, G.params(10, **kw), want, wst)


def test_autotune_and_lane_steps(ggo, monkeypatch):
    """The autotuner keeps one of its candidates, every candidate returned the same
    hits (it checks), and the kept choice, like the extreme lane-step settings
    (a wave resumes almost every walk / lanes finish every walk), equals the
    oracle."""
    G = gpu()
    monkeypatch.delenv("GG_GROUPING", raising=False)
    db = synth.mid_db(n_seqs=20_000)
    qs = synth.mid_queries(db, n=80)
    oix, gix = ggo.Index(db.seqs, db.off, 11), G.Index(db.seqs, db.off, 11)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(50))
    assert gix.tuning() == {"grouping": "sort", "lane_steps": 256, "wave_log2": 25, "graph": 1,
                            "graph_query_log2": 0}
    got = gix.autotune(qs.buf, qs.off, G.params(50))
    assert got["grouping"] in G.GROUPINGS and got["lane_steps"] in (0, 64, 256, 4096)
    assert got["sample_ms"] > 0
    assert {k: gix.tuning()[k] for k in ("grouping", "lane_steps")} == {
        k: got[k] for k in ("grouping", "lane_steps")}
    check_batch(G, gix, qs, G.params(50), want, wst)
    for steps in (0, 1, 16, 17, 4096):
        gix.set_tuning("sort", steps)
        check_batch(G, gix, qs, G.params(50), want, wst)
    with pytest.raises(G.GGError):
        gix.set_tuning("sort", -1)


def graph_waves(gix):
    return gix.profile_read("graph")["units"]


@pytest.mark.parametrize("k,band,max_hits,seed", [(11, 32, 20, 21), (8, 17, 5, 22), (4, 32, 3, 23)])
def test_graph_replayed_batches(ggo, monkeypatch, k, band, max_hits, seed):
    """Batches without per-query statistics run as replays of one captured graph
    (one replay per wave, sizes read on the device).  With one wave, with many
    waves (small hit budget), host and device results, a reused graph and a
    recaptured one all equal the oracle; k = 4 gives queries with more runs than
    the per-query LDS sorts hold, whose waves are run again without the graph."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.random_db(seed, n_seqs=300, lmin=0, lmax=3000)
    qs = synth.random_queries(seed, db, n=40, lmin=0, lmax=1500, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix, gix = ggo.Index(db.seqs, db.off, k), G.Index(db.seqs, db.off, k)
    kw = dict(band=band, max_gap=3 * k, min_hsp_len=2 * k)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(max_hits, **kw))
    prm = G.params(max_hits, **kw)

    def check(tag):
        rc, got, n, _ = gix.search_batch(qs.buf, qs.off, prm, cap=1000)
        assert rc == 0, tag
        for i in range(qs.n):
            assert as_rows(got[i]) == as_rows(want[i]), (tag, i)

    gix.profile(True)
    check("one wave")
    assert graph_waves(gix) >= 1
    check("graph reused")
    hits = max(int(s["n_hits"]) for s in wst)
    gix.set_hit_budget(16 * max(hits, 1))  # about one query per wave
    before = graph_waves(gix)
    check("many waves")
    assert graph_waves(gix) - before > 2
    gix.set_hit_budget(0)
    check("recaptured")
    cap = 3
    dq = G.DeviceBuffer(len(qs.buf))
    dq.upload(qs.buf)
    dout = G.DeviceBuffer(qs.n * cap * G.HIT_DTYPE.itemsize)
    dn = G.DeviceBuffer(qs.n * 4)
    rc, _ = gix.search_batch_device(dq, qs.off, prm, dout, dn, cap)
    assert rc == (G.GG_ETRUNC if any(len(w) > cap for w in want) else G.GG_OK)
    n = dn.download(np.zeros(qs.n, np.int32))
    got = dout.download(np.zeros(qs.n * cap, G.HIT_DTYPE))
    for i in range(qs.n):
        assert int(n[i]) == len(want[i])
        m = min(cap, len(want[i]))
        assert as_rows(got[i * cap: i * cap + m]) == as_rows(want[i][:m])
    gix.profile(False)
    if k == 4:
        assert max(s["n_cands"] for s in wst) > 1024


@pytest.mark.parametrize("k,wave_log2,qlog2", [(4, 20, 0), (8, 11, 0), (11, 25, 0), (8, 25, 10),
                                               (11, 25, 12)])
def test_graph_waves_around_large_queries(ggo, monkeypatch, k, wave_log2, qlog2):
    """Queries with more hits than a graph wave holds, and queries whose kept hits,
    runs or selections outgrow a per-query LDS sort, take the regular path after
    the replays; the other queries stay in the graph waves.  Every result equals
    the oracle, graph waves run, and the regular path runs only for those queries
    (heavy and flagged queries are packed into sub-batches of their own)."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.repeat_db(60 + k, n_seqs=300, lmin=100, lmax=4000, frac_repeat=0.3)
    qs = synth.random_queries(60 + k, db, n=60, lmin=50, lmax=2500, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix, gix = ggo.Index(db.seqs, db.off, k), G.Index(db.seqs, db.off, k)
    kw = dict(max_gap=3 * k, min_hsp_len=2 * k)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(10, **kw))
    gix.set_tuning("sort", 256, wave_log2, 1, qlog2)
    assert gix.tuning()["wave_log2"] == wave_log2 and gix.tuning()["graph_query_log2"] == qlog2
    gix.profile(True)
    rc, got, n, _ = gix.search_batch(qs.buf, qs.off, G.params(10, **kw), cap=1000)
    waves, regular = gix.profile_read("graph")["units"], gix.profile_read("extend")["launches"]
    gix.profile(False)
    assert rc == 0
    for i in range(qs.n):
        assert as_rows(got[i]) == as_rows(want[i]), i
    assert waves >= 1
    limit = min(1 << wave_log2, 1 << qlog2) if qlog2 else 1 << wave_log2
    big = [int(s["n_hits"]) > limit or int(s["n_cands"]) > 1024 for s in wst]
    # a regular wave runs only for these queries (and those the filter's kept-hit
    # limit flags, which the counts above do not show): the heavy ones share
    # waves, and so do the flagged ones
    flaggable = sum(1 for s in wst if int(s["n_hits"]) > 8192)
    assert regular <= sum(big) + flaggable
    if k == 4:
        assert any(big)


def test_graph_off_by_tuning(ggo, monkeypatch):
    """Tuning graph = 0: no batch replays the graph, results unchanged."""
    G = gpu()
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.random_db(70, n_seqs=200, lmin=100, lmax=3000)
    qs = synth.random_queries(70, db, n=30, lmin=50, lmax=1500, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix, gix = ggo.Index(db.seqs, db.off, 11), G.Index(db.seqs, db.off, 11)
    want, _ = oracle_all(ggo, oix, qs, ggo.params(10))
    for graph in (1, 0):
        gix.set_tuning("sort", 256, 0, graph, 0)
        gix.profile(True)
        rc, got, n, _ = gix.search_batch(qs.buf, qs.off, G.params(10), cap=1000)
        waves = gix.profile_read("graph")["units"]
        gix.profile(False)
        assert rc == 0 and (waves > 0) == bool(graph)
        for i in range(qs.n):
            assert as_rows(got[i]) == as_rows(want[i]), (graph, i)


def test_long_merge_groups(ggo):
    """A tandem repeat gives one (query, sequence) pair thousands of runs, more than
    one thread merges alone; the long groups are merged by whole waves and must
    equal the oracle, with the selection prefilter active (N > 0) and not (N = 0)."""
    G = gpu()
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, 90])))
    unit = rng.choice(list(b"ACGT"), 7).astype(np.uint8)
    rep = np.resize(unit, 20_000)
    flank = rng.choice(list(b"ACGT"), 3_000).astype(np.uint8)
    other = rng.choice(list(b"ACGT"), 5_000).astype(np.uint8)
    seqs = np.concatenate([flank, rep, flank[::-1], other])
    off = np.array([0, len(flank) + len(rep) + len(flank), len(seqs)], np.int64)
    parts = [np.resize(np.roll(unit, 3), 2_000), np.concatenate([flank[500:1500], rep[:900]]),
             other[1_000:3_000]]
    qoff = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([len(p) for p in parts], out=qoff[1:])
    qs = synth.QuerySet(np.concatenate(parts), qoff, np.zeros(len(parts), np.int8),
                        np.full(len(parts), -1), np.zeros(len(parts)), np.zeros(len(parts)))
    oix, gix = ggo.Index(seqs, off, 11), G.Index(seqs, off, 11)
    for n in (20, 0):
        want, wst = oracle_all(ggo, oix, qs, ggo.params(n))
        assert max(s["n_cands"] for s in wst) > 2_000
        check_batch(G, gix, qs, G.params(n), want, wst)


@pytest.mark.parametrize("band", [1, 5, 32])
def test_tie_heavy_two_letter_banks(ggo, band):
    """Banks and queries over two letters, scored +2/-1 with gaps 1 + g: many
    local alignments tie in score, so the reported spans turn on the aligner's
    tie rules (gap open before extend, start from the diagonal, then the left gap,
    then the upper gap, first maximum in row-major order)."""
    G = gpu()
    fold = np.frombuffer(b"A" * 256, dtype=np.uint8).copy()
    fold[ord("C")] = fold[ord("T")] = ord("C")
    db0 = synth.random_db(40 + band, n_seqs=200, lmin=20, lmax=600)
    qs0 = synth.random_queries(40 + band, db0, n=40, lmin=10, lmax=300, frac_homolog=0.8,
                               ident_lo=0.75, ident_hi=0.95, indel_rate=0.05)
    db = synth.Database(fold[db0.seqs], db0.off)
    qs = qs0.subset(np.arange(qs0.n))
    qs.buf = fold[qs.buf]
    kw = dict(match=2, mismatch=1, gap_open=1, gap_extend=1, xdrop=6, band=band, max_gap=8,
              min_hsp_len=12)
    oix, gix = ggo.Index(db.seqs, db.off, 6), G.Index(db.seqs, db.off, 6)
    want, wst = oracle_all(ggo, oix, qs, ggo.params(30, **kw))
    assert sum(len(w) for w in want) > 200
    check_batch(G, gix, qs, G.params(30, **kw), want, wst)
