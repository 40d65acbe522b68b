"""The served form under concurrency and a hit budget, through the C ABI.

* submits from one thread while several others wait on tickets (blocking polls),
  two of them on the same ticket: one collects it, the other is told it is gone;
* destroy while polls are waiting: they return, the server goes away cleanly;
* admission by exact hit counts under a small budget: the bytes in flight never
  exceed it, queries over it run alone in sequence ranges, and every result
  equals the oracle's.
"""
import threading
import time

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


@pytest.fixture(scope="module")
def bank(ggo):
    G = gpu()
    db = synth.random_db(21, n_seqs=600, lmin=100, lmax=4000)
    qs = synth.random_queries(21, db, n=120, lmin=30, lmax=2500, frac_homolog=0.7,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.01)
    gix = G.Index(db.seqs, db.off, 8)
    oix = ggo.Index(db.seqs, db.off, 8)
    prm = dict(max_gap=20, min_hsp_len=16)
    want = []
    for i in range(qs.n):
        rc, h, n, st = oix.search(qs.query(i), ggo.params(10, **prm), cap=1000)
        assert rc == 0
        want.append((h, int(st["n_hits"])))
    return G, db, qs, gix, G.params(10, **prm), want


def test_submit_while_polling(bank):
    G, db, qs, gix, prm, want = bank
    sv = G.Server(gix, prm, max_slots=8)
    tickets = [None] * qs.n
    ready = [threading.Event() for _ in range(qs.n)]
    results = {}
    lock = threading.Lock()

    def submitter():
        for i in range(qs.n):
            tickets[i] = sv.submit(qs.query(i))
            ready[i].set()
            if i % 7 == 0:
                time.sleep(0.001)

    def poller(k):
        for i in range(k, qs.n, 4):
            ready[i].wait()
            rc, h, n = sv.poll(tickets[i], cap=1000, timeout_us=-1)
            with lock:
                results.setdefault(i, []).append((rc, as_rows(h)))

    def twin(i):
        # a second blocking poll of a ticket another thread also waits on
        ready[i].wait()
        rc, h, n = sv.poll(tickets[i], cap=1000, timeout_us=-1)
        with lock:
            results.setdefault(i, []).append((rc, as_rows(h)))

    try:
        ths = [threading.Thread(target=submitter)]
        ths += [threading.Thread(target=poller, args=(k,)) for k in range(4)]
        ths += [threading.Thread(target=twin, args=(i,)) for i in (5, 50, 110)]
        for t in ths:
            t.start()
        for t in ths:
            t.join(120)
            assert not t.is_alive()
        for i in range(qs.n):
            got = results[i]
            ok = [r for r in got if r[0] == G.GG_OK]
            gone = [r for r in got if r[0] == G.GG_ENOTFOUND]
            assert len(ok) == 1 and len(ok) + len(gone) == len(got), (i, [r[0] for r in got])
            assert ok[0][1] == as_rows(want[i][0]), i
        info = sv.info()
        assert info["submitted"] == info["completed"] == qs.n
        assert info["inflight_slots"] == 0 and info["inflight_bytes"] == 0
        assert info["peak_inflight_slots"] <= 8
    finally:
        sv.close()


def test_destroy_while_polls_wait(bank):
    G, db, qs, gix, prm, want = bank
    sv = G.Server(gix, prm, max_slots=4)
    tickets = [sv.submit(qs.query(i)) for i in range(qs.n)]
    status = []
    lock = threading.Lock()

    def waiter(t):
        rc, h, n = sv.poll(t, cap=1000, timeout_us=-1)
        with lock:
            status.append(rc)

    ths = [threading.Thread(target=waiter, args=(tickets[-1 - j],)) for j in range(6)]
    for t in ths:
        t.start()
    t0 = time.time()
    # every waiter is inside gg_serve_poll or has returned from it
    while sv.info()["calls_inside"] + len(status) < len(ths) and time.time() - t0 < 30:
        time.sleep(0.001)
    sv.close()  # gg_server_destroy with polls waiting
    for t in ths:
        t.join(60)
        assert not t.is_alive()
    assert len(status) == 6
    assert all(rc in (G.GG_OK, G.GG_ENOTFOUND) for rc in status)


def test_admission_by_hit_bytes(bank):
    """A budget of a third of the largest query's hit bytes: that query and others
    over the budget run alone in sequence ranges; the bytes in flight never exceed
    the budget; every result equals the oracle's."""
    G, db, qs, gix, prm, want = bank
    hits = np.array([w[1] for w in want], dtype=np.int64)
    budget = int(16 * hits.max() // 3)
    sv = G.Server(gix, prm, hit_budget_bytes=budget, max_slots=64)
    try:
        tickets = [sv.submit(qs.query(i)) for i in range(qs.n)]
        for i, t in enumerate(tickets):
            rc, h, n = sv.poll(t, cap=1000, timeout_us=-1)
            assert rc == G.GG_OK and as_rows(h) == as_rows(want[i][0]), i
        info = sv.info()
        assert info["budget_bytes"] == budget
        assert 0 < info["peak_inflight_bytes"] <= budget
        assert info["over_budget"] == int((16 * hits > budget).sum()) > 0
        assert info["completed"] == qs.n and info["batches"] >= info["over_budget"]
    finally:
        sv.close()


def test_submit_rejects_bad_bytes(bank):
    G, db, qs, gix, prm, want = bank
    sv = G.Server(gix, prm, max_slots=2)
    try:
        with pytest.raises(G.GGError):
            sv.submit(b"ACGTNACGT")
        t = sv.submit(b"acgu" * 20)
        rc, h, n = sv.poll(t, cap=10, timeout_us=-1)
        assert rc == G.GG_OK
        assert sv.info()["submitted"] == 1
    finally:
        sv.close()
