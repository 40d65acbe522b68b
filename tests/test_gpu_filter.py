"""GPU parity of the lone-diagonal filter, bit-exact against the oracle.

When the minimum HSP length M exceeds the seed span, a hit alone on its
(sequence, diagonal) cannot be part of a kept run (Section 2.2), so the GPU path
drops such hits per query before grouping and sorts the rest in LDS.  The oracle
groups and chains every hit.  Checked here: results and every per-query count
equal the oracle's with the filter on and off, in the host-driven and the
graph-replayed forms; a query whose real diagonal groups hold more hits than the
LDS sort takes (a 50 kb copy of a bank sequence) goes through the radix sort
instead, and its graph-replayed wave is run again by the host; with M at or below
the span the filter stays off and runs of one hit are kept.  Each case runs with
the two kernels apart (the default, GG_FUSE=0) and with the filter fused into the
gather (GG_FUSE=1: keys built from the postings, no key stored before the filter).
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu

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


def check_stats(G, gix, qs, prm, want, wst, cap=100000):
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm, cap=cap, stats=True)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        for f in FIELDS:
            assert int(st[i][f]) == wst[i][f], (i, f, int(st[i][f]), wst[i][f])
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"


def check_graph(G, gix, qs, prm, want, cap=1000):
    rc, got, n, _ = gix.search_batch(qs.buf, qs.off, prm, cap=cap)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"


def filter_units(gix):
    return gix.profile_read("filter")["units"] + gix.profile_read("gather_filter")["units"]


FUSE = pytest.mark.parametrize("fuse", ["1", "0"])


@FUSE
def test_filter_on_and_off_on_the_bank_workload(ggo, monkeypatch, fuse):
    G = gpu()
    monkeypatch.setenv("GG_FUSE", fuse)
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.mid_db(n_seqs=20_000)
    qs = synth.mid_queries(db, n=80)
    oix, gix = ggo.Index(db.seqs, db.off, 11), G.Index(db.seqs, db.off, 11)
    want, wst = oracle_all(oix, qs, ggo.params(50))
    prm = G.params(50)
    gix.profile(True)
    check_stats(G, gix, qs, prm, want, wst)
    assert filter_units(gix) > 0  # the filter ran
    assert gix.profile_read("gather_filter")["units"] > 0 if fuse == "1" else True
    assert qs.lengths().max() > 2 * 3832  # queries whose offsets are staged sparsely
    check_graph(G, gix, qs, prm, want)
    assert gix.profile_read("graph")["units"] >= 1
    gix.profile(False)
    monkeypatch.setenv("GG_FILTER", "0")
    gix.profile(True)
    check_stats(G, gix, qs, prm, want, wst)
    check_graph(G, gix, qs, prm, want)
    assert filter_units(gix) == 0
    gix.profile(False)


def copy_bank(seed):
    """A 60 kb sequence among short random ones, and queries: a 50 kb copy of its
    start (about 4,500 hits on one diagonal), a mutated 8 kb copy, random ones and
    an empty one."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, seed])))
    acgt = np.frombuffer(b"ACGT", np.uint8)
    big = acgt[rng.integers(0, 4, 60_000)]
    small = synth.random_db(seed, n_seqs=200, lmin=0, lmax=2000)
    seqs = np.concatenate([small.seqs, big])
    off = np.concatenate([small.off, [small.off[-1] + len(big)]]).astype(np.int64)
    mut = big[20_000:28_000].copy()
    pos = rng.choice(len(mut), 400, replace=False)
    mut[pos] = acgt[(np.searchsorted(acgt, mut[pos]) + rng.integers(1, 4, len(pos))) % 4]
    parts = [big[:50_000].tobytes(), mut.tobytes(), b""]
    parts += [acgt[rng.integers(0, 4, int(n))].tobytes() for n in rng.integers(50, 3000, 8)]
    qoff = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([len(p) for p in parts], out=qoff[1:])
    buf = np.frombuffer(b"".join(parts), np.uint8).copy()
    n = len(parts)
    qs = synth.QuerySet(buf, qoff, np.zeros(n, np.int8), np.full(n, -1, np.int32),
                        np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.float32))
    return seqs, off, qs


@FUSE
def test_query_over_the_lds_sort(ggo, monkeypatch, fuse):
    G = gpu()
    monkeypatch.setenv("GG_FUSE", fuse)
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    seqs, off, qs = copy_bank(61)
    oix, gix = ggo.Index(seqs, off, 11), G.Index(seqs, off, 11)
    want, wst = oracle_all(oix, qs, ggo.params(20))
    assert wst[0]["n_hits"] > 4096 + 200  # the copy's diagonal alone holds more
    prm = G.params(20)
    check_stats(G, gix, qs, prm, want, wst)
    check_graph(G, gix, qs, prm, want)


@pytest.mark.parametrize("k,min_len", [(11, 11), (8, 6)])
def test_runs_of_one_hit_kept(ggo, monkeypatch, k, min_len):
    """M <= span: a single hit is a run long enough to keep; the filter stays off."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.random_db(62 + k, n_seqs=150, lmin=0, lmax=2000)
    qs = synth.random_queries(62 + k, db, n=20, lmin=0, lmax=600, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix, gix = ggo.Index(db.seqs, db.off, k), G.Index(db.seqs, db.off, k)
    kw = dict(max_gap=2 * k, min_hsp_len=min_len)
    want, wst = oracle_all(oix, qs, ggo.params(10, **kw))
    assert sum(s["n_cands"] for s in wst) > sum(1 for w in want for _ in w)
    prm = G.params(10, **kw)
    gix.profile(True)
    check_stats(G, gix, qs, prm, want, wst)
    check_graph(G, gix, qs, prm, want)
    assert filter_units(gix) == 0
    gix.profile(False)
