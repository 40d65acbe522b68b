"""Pins for the oracle's banded Smith-Waterman (O9, Section 2.2 phase 6).

* exhaustive enumeration of every local alignment path on tiny inputs, with and
  without the band (tests/brute.py shares no code with the oracle);
* the reduction to maximum-sum segments along diagonals (Kadane) when gaps are
  prohibitively expensive;
* closed forms for identical sequences, one substitution and one gap;
* the band centre d0 = floor((dmin + dmax) / 2) and the half-width W.
"""
import json
import os

import numpy as np
import pytest

from brute import enumerate_local

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def codes(text):
    return np.array(["ACGT".index(c) for c in text], dtype=np.uint8)


def rand_text(rng, n, alphabet="ACGT"):
    return "".join(rng.choice(list(alphabet), size=n))


def box_of(qs, qe, ds, de, dmin=None, dmax=None, seq=0):
    d = ds - qs
    return (seq, qs, qe, ds, de, d if dmin is None else dmin, d if dmax is None else dmax)


SCHEMES = [
    dict(match=1, mismatch=3, gap_open=5, gap_extend=2),
    dict(match=2, mismatch=1, gap_open=1, gap_extend=1),
    dict(match=3, mismatch=2, gap_open=0, gap_extend=2),
]


@pytest.mark.parametrize("scheme", range(len(SCHEMES)))
def test_unbanded_equals_enumeration(ggo, scheme):
    sc = SCHEMES[scheme]
    prm = ggo.params(0, band=64, **sc)
    rng = np.random.default_rng(100 + scheme)
    for trial in range(25):
        q = rand_text(rng, int(rng.integers(1, 7)), "ACG" if trial % 2 else "AC")
        s = rand_text(rng, int(rng.integers(1, 7)), "ACG" if trial % 2 else "AC")
        best, spans = enumerate_local(q, s, **sc)
        hit, cells = ggo.bsw(codes(q), codes(s), box_of(0, len(q), 0, len(s)), prm)
        assert cells == len(q) * len(s)
        assert hit["score"] == best, (q, s)
        if best > 0:
            assert (hit["q_start"], hit["q_end"], hit["d_start"], hit["d_end"]) in spans


@pytest.mark.parametrize("W", [0, 1, 2])
def test_banded_equals_band_confined_enumeration(ggo, W):
    sc = SCHEMES[1]
    rng = np.random.default_rng(7 + W)
    for trial in range(25):
        R, C = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        q, s = rand_text(rng, R, "ACG"), rand_text(rng, C, "ACG")
        dmin = int(rng.integers(-3, 4))
        dmax = dmin + int(rng.integers(0, 4))
        d0 = (dmin + dmax) // 2  # Python floor division
        # the box starts at query 0 and database 0, so cell (i, j) sits on diagonal j - i
        in_band = lambda i, j: abs(j - i - d0) <= W
        best, spans = enumerate_local(q, s, in_band=in_band, **sc)
        prm = ggo.params(0, band=W, **sc)
        hit, cells = ggo.bsw(codes(q), codes(s), box_of(0, R, 0, C, dmin, dmax), prm)
        assert cells == sum(in_band(i, j) for i in range(R) for j in range(C))
        assert hit["score"] == best, (q, s, dmin, dmax)
        if best > 0:
            assert (hit["q_start"], hit["q_end"], hit["d_start"], hit["d_end"]) in spans


def kadane_best(vals):
    best = cur = 0
    for v in vals:
        cur = max(0, cur + v)
        best = max(best, cur)
    return best


@pytest.mark.parametrize("trial", range(8))
def test_no_gap_limit_is_best_diagonal_segment(ggo, trial):
    """With gaps costing more than any alignment can gain, banded SW is the best
    maximum-sum segment over the band's diagonals (Kadane's algorithm)."""
    rng = np.random.default_rng(trial)
    R, C = int(rng.integers(30, 200)), int(rng.integers(30, 200))
    q, s = rand_text(rng, R), rand_text(rng, C)
    # plant a similar stretch so the best is not tiny
    a = int(rng.integers(0, R // 2)); b = int(rng.integers(0, C // 2)); ln = min(R - a, C - b, 25)
    s = s[:b] + q[a:a + ln] + s[b + ln:]
    W = 32
    prm = ggo.params(0, band=W, gap_open=10 ** 6, gap_extend=10 ** 6)
    ds = int(rng.integers(0, 20))
    dmin = dmax = ds + int(rng.integers(-10, 10))
    hit, _ = ggo.bsw(codes(q), codes("A" * ds + s), box_of(0, R, ds, ds + C, dmin, dmax), prm)
    qa, sa = codes(q), codes("A" * ds + s)
    best = 0
    for diag in range(dmin - W, dmin + W + 1):
        vals = [1 if qa[i] == sa[i + diag] else -3 for i in range(R) if ds <= i + diag < ds + C]
        best = max(best, kadane_best(vals))
    assert hit["score"] == best
    if best > 0:
        L = hit["q_end"] - hit["q_start"]
        assert hit["d_end"] - hit["d_start"] == L
        seg = [1 if qa[hit["q_start"] + t] == sa[hit["d_start"] + t] else -3 for t in range(L)]
        assert sum(seg) == best


def test_identical_sequences(ggo):
    rng = np.random.default_rng(1)
    prm = ggo.params(0)
    for L in (1, 2, 33, 64, 65, 500, 2000):
        t = rand_text(rng, L)
        hit, cells = ggo.bsw(codes(t), codes(t), box_of(0, L, 0, L), prm)
        assert (hit["score"], hit["q_start"], hit["q_end"], hit["d_start"], hit["d_end"]) == (
            L, 0, L, 0, L)
        assert cells == sum(min(L - 1, i + 32) - max(0, i - 32) + 1 for i in range(L))


def test_one_substitution(ggo):
    rng = np.random.default_rng(2)
    prm = ggo.params(0)
    for a, b in ((4, 4), (10, 50), (200, 7)):
        x = rand_text(rng, a + 1 + b)
        y = list(x)
        y[a] = "ACGT"[("ACGT".index(x[a]) + 1) % 4]
        y = "".join(y)
        hit, _ = ggo.bsw(codes(x), codes(y), box_of(0, len(x), 0, len(y)), prm)
        assert hit["score"] == a + b - 3
        assert (hit["q_start"], hit["q_end"]) == (0, a + 1 + b)


@pytest.mark.parametrize("g", [1, 2, 3, 5, 10])
def test_one_gap_closed_form(ggo, g):
    rng = np.random.default_rng(10 + g)
    prm = ggo.params(0)
    for a, b in ((60, 50), (30, 80), (12, 9)):
        A, B, X = rand_text(rng, a), rand_text(rng, b), rand_text(rng, g)
        q, s = A + B, A + X + B
        hit, _ = ggo.bsw(codes(q), codes(s), box_of(0, len(q), 0, len(s)), prm)
        want = max(a + b - 5 - 2 * g, a, b)
        assert hit["score"] == want
        if a + b - 5 - 2 * g > max(a, b):  # a strict optimum fixes the span
            assert (hit["q_start"], hit["q_end"], hit["d_start"], hit["d_end"]) == (
                0, a + b, 0, a + g + b)
        # and the mirror: the extra bases on the query side
        hit2, _ = ggo.bsw(codes(s), codes(q), box_of(0, len(s), 0, len(q)), prm)
        assert hit2["score"] == want


def test_band_half_width_and_centre(ggo):
    g = json.load(open(os.path.join(GOLD, "bsw_closed_forms.json")))["band_centre"]
    rng = np.random.default_rng(3)
    prm = ggo.params(0)
    W = prm.band
    L = 40
    core = rand_text(rng, L)
    for diag, expect in ((g["inside"], True), (g["outside"], False),
                         (-2 + W, True), (-2 + W + 1, False), (-2 - W - 1, False)):
        # query holds core at 100; database holds it at 100 + diag; the rest mismatches
        n = 400
        q = ["A"] * n
        s = ["C"] * n
        q[100:100 + L] = core
        s[100 + diag:100 + diag + L] = core
        hit, _ = ggo.bsw(codes("".join(q)), codes("".join(s)),
                         box_of(0, n, 0, n, g["dmin"], g["dmax"]), prm)
        assert (hit["score"] == L) == expect, diag
        if expect:
            assert (hit["q_start"], hit["d_start"]) == (100, 100 + diag)


def test_empty_box(ggo):
    prm = ggo.params(0)
    hit, cells = ggo.bsw(codes("ACGT"), codes("ACGT"), box_of(2, 2, 2, 2), prm)
    assert cells == 0 and hit["score"] == 0


TIES = json.load(open(os.path.join(GOLD, "bsw_ties.json")))


@pytest.mark.parametrize("case", TIES["cases"], ids=[c["name"] for c in TIES["cases"]])
def test_tie_rules_hand_worked(ggo, case):
    """Tied optima: the reported span is the one the tie rules pick (hand-worked
    cells in the golden file), and it is one of several optimal spans that the
    brute-force enumeration finds, so the case really turns on the rule."""
    sc = TIES["scheme"]
    q, s, W, d0 = case["q"], case["s"], case["band"], case["d0"]
    prm = ggo.params(0, band=W, **sc)
    hit, cells = ggo.bsw(codes(q), codes(s), box_of(0, len(q), 0, len(s), d0, d0), prm)
    in_band = lambda i, j: abs(j - i - d0) <= W
    assert cells == sum(in_band(i, j) for i in range(len(q)) for j in range(len(s)))
    assert hit["score"] == case["score"]
    assert [hit["q_start"], hit["q_end"], hit["d_start"], hit["d_end"]] == case["span"]
    best, spans = enumerate_local(q, s, in_band=in_band, **sc)
    assert best == case["score"]
    assert tuple(case["span"]) in spans
    assert (len(spans) > 1) == case["tied_optima"]
