"""The parallel form of the merge sweep (Section 2.2 phase 4: overlapping HSPs of
one sequence merged in a single pass), as the merge kernels run it, checked on
the CPU against the plain one-pass sweep.

The kernels take a window's sorted boxes eight per thread over 256 threads.
Tentative merged-box starts are the group's first box and every box that does
not join the box before it; rounds of a segmented scan of the tentative
segments' unions drop each start that joins the union before it, until a round
drops none.  Groups longer than one window go in chunks of 2,048 boxes, the
union of the segment open at a chunk's end carried into the next.  This test
replays those rounds in Python (same thread layout, same carry rules) on boxes
shaped like extension output, including starts that fall on chunk boundaries,
and requires the merged boxes to equal the one-pass sweep's exactly.
"""
import random

import pytest

THREADS, PER, CHUNK = 256, 8, 2048
NONE = (2**31 - 1, -2**31, 2**31 - 1, -2**31, 2**31 - 1, -2**31)


def join(a, b):
    return (min(a[0], b[0]), max(a[1], b[1]), min(a[2], b[2]), max(a[3], b[3]),
            min(a[4], b[4]), max(a[5], b[5]))


def takes(cur, b):
    """The sweep's test: box b (qs, qe, ds, de, ...) joins the union cur."""
    return b[0] < cur[1] and b[2] < cur[3] and cur[2] < b[3]


def one_pass(boxes):
    out, cur = [], boxes[0]
    for b in boxes[1:]:
        if takes(cur, b):
            cur = join(cur, b)
        else:
            out.append(cur)
            cur = b
    out.append(cur)
    return out


def rounds_form(boxes, max_rounds=64):
    n = len(boxes)
    out = [None] * n
    open_u, nseg, rounds_used = NONE, 0, 0
    for c0 in range(0, n, CHUNK):
        m = min(CHUNK, n - c0)
        F = [[False] * PER for _ in range(THREADS)]
        V = [[False] * PER for _ in range(THREADS)]
        for t in range(THREADS):
            for r in range(PER):
                j = t * PER + r
                if j >= m:
                    break
                V[t][r] = True
                i = c0 + j
                F[t][r] = i == 0 or not takes(boxes[i - 1], boxes[i])
        for rnd in range(max_rounds):
            summ = []
            for t in range(THREADS):
                sf, sa = False, NONE
                for r in range(PER):
                    if V[t][r]:
                        b = boxes[c0 + t * PER + r]
                        sf, sa = (True, b) if F[t][r] else (sf, join(sa, b))
                summ.append((sf, sa))
            carries, seen, acc = [], False, NONE
            for t in range(THREADS):
                carries.append(acc if seen else join(open_u, acc))
                sf, sa = summ[t]
                acc = sa if sf else join(acc, sa)
                seen = seen or sf
            changed = False
            for t in range(THREADS):
                run = carries[t]
                for r in range(PER):
                    if not V[t][r]:
                        continue
                    b = boxes[c0 + t * PER + r]
                    first = c0 == 0 and t == 0 and r == 0
                    if F[t][r] and not first and takes(run, b):
                        F[t][r] = False
                        changed = True
                    run = b if F[t][r] else join(run, b)
            rounds_used = max(rounds_used, rnd + 1)
            if not changed:
                break
        else:
            raise AssertionError("rounds did not settle")
        if c0 > 0 and F[0][0]:
            out[nseg - 1] = open_u
        before = 0
        for t in range(THREADS):
            run = carries[t]
            for r in range(PER):
                if not V[t][r]:
                    continue
                j = t * PER + r
                b = boxes[c0 + j]
                run = b if F[t][r] else join(run, b)
                k = nseg - 1 + before + sum(F[t][:r + 1])
                if j + 1 >= m:
                    if c0 + m == n:
                        out[k] = run
                    last_open, last_n = run, k + 1
                elif F[t][r + 1] if r + 1 < PER else F[t + 1][0]:
                    out[k] = run
            before += sum(F[t])
        open_u, nseg = last_open, last_n
    return out[:nseg], rounds_used


def extension_like(rng, n, spread):
    """n boxes of one (query, sequence) group, sorted in merge order (qs, ds, qe, de):
    most on a few nearby diagonals (repeats), some far off."""
    boxes = []
    for _ in range(n):
        qs = rng.randint(0, spread)
        length = rng.randint(5, 200)
        d = rng.randint(-50, 50) if rng.random() < 0.8 else rng.randint(-5000, 5000)
        boxes.append((qs, qs + length, qs + d, qs + length + d, d, d))
    boxes.sort(key=lambda b: (b[0], b[2], b[1], b[3]))
    return boxes


@pytest.mark.parametrize("n,spread,seed", [(1, 100, 1), (37, 100, 2), (2047, 3000, 3),
                                           (2048, 3000, 4), (2049, 3000, 5), (5000, 3000, 6),
                                           (7000, 3000, 16), (4500, 200000, 7)])
def test_rounds_equal_one_pass(n, spread, seed):
    boxes = extension_like(random.Random(seed), n, spread)
    got, _ = rounds_form(boxes)
    assert got == one_pass(boxes)


def test_start_on_a_chunk_boundary():
    """A merged box made of a chunk's last box alone, the next chunk starting a new
    one: the carried segment is closed by the start at the next chunk's first box."""
    boxes = []
    for i in range(2 * CHUNK + 10):
        if i == CHUNK - 1:
            boxes.append((10 * i, 10 * i + 3, 10 * i + 100000, 10 * i + 100003, 100000, 100000))
        else:
            boxes.append((10 * i, 10 * i + 25, 10 * i, 10 * i + 25, 0, 0))
    want = one_pass(boxes)
    assert len(want) == 3
    got, _ = rounds_form(boxes)
    assert got == want


def test_tentative_starts_dropped_over_rounds():
    """Small boxes inside one big box, none overlapping the one before it: each is
    a tentative start that joins only the big box's union.  A thread drops its own
    in one pass, and each later thread's in the round after the thread before it
    has dropped them, so it takes several rounds to settle."""
    boxes = [(0, 1000, 0, 1000, 0, 0)]
    for i in range(1, 60):
        boxes.append((2 * i, 2 * i + 1, 2 * i, 2 * i + 1, 0, 0))
    want = one_pass(boxes)
    assert len(want) == 1
    got, used = rounds_form(boxes)
    assert got == want
    assert used >= 5
