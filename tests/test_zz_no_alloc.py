"""gg_traceback_noalloc (device scratch in a static array, no allocation) against
gg_traceback, through the C ABI: the same status and paths, byte for byte, on two
calls in a row (the second smaller, so it runs over what the first left in the
scratch), and GG_ESCRATCH beyond the array."""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


@pytest.fixture(scope="module")
def searched():
    G = gpu()
    db = synth.random_db(31, n_seqs=300, lmin=200, lmax=6000)
    qs = synth.random_queries(31, db, n=12, lmin=800, lmax=5000, frac_homolog=1.0,
                              ident_lo=0.85, ident_hi=0.99, indel_rate=0.02)
    gix = G.Index(db.seqs, db.off, 11)
    prm = G.params(40, band=20)
    res = []
    for i in range(qs.n):
        rc, h, n = gix.search(qs.query(i), prm, cap=64)
        assert rc == G.GG_OK
        res.append(h)
    # the two queries with the most alignments, the larger first
    order = sorted(range(qs.n), key=lambda i: -int(np.sum(res[i]["q_end"] - res[i]["q_start"])))
    return G, qs, gix, prm, res, order


def test_noalloc_equals_traceback_twice(searched):
    G, qs, gix, prm, res, order = searched
    big, small = order[0], order[-1]
    assert len(res[big]) > len(res[small]) > 0
    for i in (big, small):  # the second call is smaller than the first
        q, h = qs.query(i), res[i]
        rc0, ops0 = gix.traceback(q, prm, h)
        rc1, ops1 = gix.traceback(q, prm, h, noalloc=True)
        assert rc0 == rc1 == G.GG_OK
        assert ops1 == ops0 and all(len(o) > 0 for o in ops1)


def test_noalloc_rejects_what_traceback_rejects(searched):
    """A hit whose score is wrong fails the same way in both forms; the others are
    still written."""
    G, qs, gix, prm, res, order = searched
    i = order[1]
    h = res[i].copy()
    h["score"][0] += 1
    rc0, ops0 = gix.traceback(qs.query(i), prm, h)
    rc1, ops1 = gix.traceback(qs.query(i), prm, h, noalloc=True)
    assert rc0 == rc1 == G.GG_EINVAL
    assert ops1 == ops0 and ops1[0] == "" and all(len(o) > 0 for o in ops1[1:])


def test_noalloc_scratch_limit(searched):
    """More direction rows than the static scratch holds: GG_ESCRATCH, and the
    allocating form still serves the call."""
    G, qs, gix, prm, res, order = searched
    i = order[0]
    h = res[i]
    rows = int(np.sum(h["q_end"] - h["q_start"]))
    reps = G.NOALLOC_SCRATCH_BYTES // (64 * rows) + 1
    many = np.concatenate([h] * reps)
    rc1, _ = gix.traceback(qs.query(i), prm, many, noalloc=True)
    assert rc1 == G.GG_ESCRATCH
    rc0, ops0 = gix.traceback(qs.query(i), prm, many[: len(h)])
    assert rc0 == G.GG_OK
