"""GPU parity of the merge step (Section 2.2: overlapping HSPs of one sequence
merged in a single pass) on queries whose runs outgrow the per-query LDS sorts,
bit-exact against the oracle.

Tandem repeats of one short unit, two tracts to a bank sequence, and one tract
in a query give each (query, sequence) pair as many runs as the tracts allow, in
two or more merged boxes: groups of up to 256 runs (sorted and swept by one wave
each), up to 1,024 (one block each) and beyond (the global record sort).  The
windowed merge of the sort grouping is also run with its sweep one thread per
group (GG_MERGE=serial) and with every box through the global sort
(GG_MERGE=global).  Every grouping strategy is run: the
sort and bucket groupings emit runs in (query, sequence) order, and any order that
is not falls back to the global sort.  Both the host-driven batch (with per-query
counts) and the graph-replayed one (whose waves overflow the LDS sorts and run
again on the host) must equal the oracle, for N = 20 and N = 0 (every box).
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


def repeat_bank():
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, 91])))
    acgt = np.frombuffer(b"ACGT", np.uint8)
    unit = acgt[rng.integers(0, 4, 5)]
    seqs, off = [], [0]
    for L in (40, 120, 300, 700, 1500, 4000, 9000):  # two tracts per sequence
        s = np.concatenate([acgt[rng.integers(0, 4, 400)], np.resize(unit, L),
                            acgt[rng.integers(0, 4, 300)], np.resize(np.roll(unit, 1), L // 3),
                            acgt[rng.integers(0, 4, 400)]])
        seqs.append(s)
        off.append(off[-1] + len(s))
    parts = []
    for T in (600, 1500):
        parts.append(np.concatenate([acgt[rng.integers(0, 4, 200)], np.resize(np.roll(unit, 2), T),
                                     acgt[rng.integers(0, 4, 200)]]).tobytes())
    parts += [acgt[rng.integers(0, 4, 700)].tobytes(), b""]
    qoff = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([len(p) for p in parts], out=qoff[1:])
    n = len(parts)
    qs = synth.QuerySet(np.frombuffer(b"".join(parts), np.uint8).copy(), qoff, np.zeros(n, np.int8),
                        np.full(n, -1, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                        np.zeros(n, np.float32))
    return np.concatenate(seqs), np.array(off, np.int64), qs


@pytest.fixture(scope="module")
def bank(ggo):
    seqs, off, qs = repeat_bank()
    return seqs, off, qs, ggo.Index(seqs, off, 11)


@pytest.mark.parametrize("grouping", ["sort", "bucket", "probe"])
@pytest.mark.parametrize("N", [20, 0])
def test_merge_groups_of_every_size(ggo, bank, monkeypatch, grouping, N):
    G = gpu()
    seqs, off, qs, oix = bank
    monkeypatch.setenv("GG_GROUPING", grouping)
    monkeypatch.delenv("GG_GRAPH", raising=False)
    want, wst = [], []
    for i in range(qs.n):
        rc, h, n, st = oix.search(qs.query(i), ggo.params(N), cap=100000)
        assert rc == 0
        want.append(h)
        wst.append(st)
    assert wst[1]["n_cands"] > 5000 and wst[0]["n_cands"] > 1024
    gix = G.Index(seqs, off, 11)
    prm = G.params(N)
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm, cap=100000, stats=True)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        for f in FIELDS:
            assert int(st[i][f]) == wst[i][f], (i, f, int(st[i][f]), wst[i][f])
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"
    if N > 0:  # graph-replayed form (its wave overflows and runs again on the host)
        rc, got, n, _ = gix.search_batch(qs.buf, qs.off, prm, cap=1000)
        assert rc == 0, G.STATUS[rc]
        for i in range(qs.n):
            assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"


@pytest.mark.parametrize("merge", ["serial", "global"])
@pytest.mark.parametrize("N", [20, 0])
def test_merge_sweep_forms(ggo, bank, monkeypatch, merge, N):
    G = gpu()
    seqs, off, qs, oix = bank
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.setenv("GG_MERGE", merge)
    monkeypatch.delenv("GG_GRAPH", raising=False)
    gix = G.Index(seqs, off, 11)
    prm = G.params(N)
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm, cap=100000, stats=True)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        rc, h, _, wst = oix.search(qs.query(i), ggo.params(N), cap=100000)
        assert rc == 0
        assert int(st[i]["n_merged"]) == wst["n_merged"], (i, merge)
        assert as_rows(got[i]) == as_rows(h), f"query {i}, GG_MERGE={merge}"
