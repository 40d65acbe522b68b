"""Pins of the oracle's significance statistics (the e-value and normalized score
reported with each alignment, Section 2.2), computed by Karlin-Altschul statistics
of ungapped scoring on uniform bases:

* +1/-1 scoring has closed forms: lambda = ln(q/p) = ln 3, K = (q - p)^2 / q = 1/3,
  H = lambda (p e^lambda - q e^-lambda) = ln(3) / 2;
* lambda is the positive root of its defining equation, and the only one;
* scaling both scores by c divides lambda by c and leaves K and H unchanged (this
  catches a lattice span left out of K);
* K against a Monte-Carlo sample of the best ungapped local score of random
  sequence pairs, P(S >= x) = 1 - exp(-K m n e^(-lambda x));
* bit score and e-value of a hand-worked case, and E = m n 2^(-bits).
"""
import math

import numpy as np
import pytest


def test_plus_minus_one_closed_forms(ggo):
    lam, K, H = ggo.karlin_altschul(1, 1)
    assert lam == pytest.approx(math.log(3), rel=1e-12)
    assert K == pytest.approx((0.75 - 0.25) ** 2 / 0.75, rel=1e-9)
    assert H == pytest.approx(math.log(3) / 2, rel=1e-12)


@pytest.mark.parametrize("match,mismatch", [(1, 3), (1, 2), (2, 3), (1, 5), (3, 4)])
def test_lambda_is_the_positive_root(ggo, match, mismatch):
    lam, K, H = ggo.karlin_altschul(match, mismatch)
    f = lambda x: 0.25 * math.exp(x * match) + 0.75 * math.exp(-x * mismatch) - 1  # noqa: E731
    assert lam > 0 and abs(f(lam)) < 1e-12
    assert f(lam * 0.999) < 0 < f(lam * 1.001)
    assert 0 < K < 1 and H > 0


@pytest.mark.parametrize("c", [2, 3, 5])
def test_scaling_the_scores(ggo, c):
    lam, K, H = ggo.karlin_altschul(1, 3)
    lc, Kc, Hc = ggo.karlin_altschul(c, 3 * c)
    assert lc == pytest.approx(lam / c, rel=1e-12)
    assert Kc == pytest.approx(K, rel=1e-9)
    assert Hc == pytest.approx(H, rel=1e-12)


def best_ungapped(a: np.ndarray, b: np.ndarray, match: int, mismatch: int) -> int:
    """Best-scoring ungapped local alignment of a and b, over every diagonal."""
    m, n = len(a), len(b)
    s = np.where(a[:, None] == b[None, :], match, -mismatch).astype(np.int64)
    # t[i, d] = s[i, i + d - (m - 1)]: column d holds diagonal d - (m - 1), cells
    # outside the matrix score 0 and so never raise a maximum
    t = np.zeros((m, m + n - 1), np.int64)
    i = np.repeat(np.arange(m), n)
    j = np.tile(np.arange(n), m)
    t[i, j - i + (m - 1)] = s.ravel()
    pre = np.vstack([np.zeros((1, t.shape[1]), np.int64), np.cumsum(t, axis=0)])
    low = np.minimum.accumulate(pre, axis=0)
    return int((pre - low).max())


@pytest.mark.parametrize("match,mismatch", [(1, 3), (1, 1)])
def test_K_against_monte_carlo(ggo, match, mismatch):
    lam, K, H = ggo.karlin_altschul(match, mismatch)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([150702987, 31, match])))
    m = n = 300
    best = np.array([best_ungapped(rng.integers(0, 4, m), rng.integers(0, 4, n), match, mismatch)
                     for _ in range(1500)])
    # effective lengths: an alignment of expected length ln(K m n) / H cannot start
    # within that distance of either end
    ell = math.log(K * m * n) / H
    mn = (m - ell) * (n - ell)
    ests = []
    for x in range(int(best.min()), int(best.max()) + 1):
        tail = float((best >= x).mean())
        if 0.1 <= tail <= 0.9:
            ests.append(-math.log(1 - tail) * math.exp(lam * x) / mn)
    assert len(ests) >= 2
    assert np.median(ests) == pytest.approx(K, rel=0.15)


def test_bit_score_and_evalue_hand_worked(ggo):
    lam, K = math.log(3), 1 / 3
    bits, ev = ggo.significance(10, 100, 100, lam, K)
    # E = (1/3) 100 100 3^-10 = 10^4 / 3^11; bits = (10 ln 3 + ln 3) / ln 2 = 11 log2 3
    assert ev == pytest.approx(1e4 / 3 ** 11, rel=1e-12)
    assert bits == pytest.approx(11 * math.log2(3), rel=1e-12)
    lam, K, _ = ggo.karlin_altschul(1, 3)
    for s, m, n in [(30, 500, 2_000_000), (200, 4000, 3_000_000_000), (1, 11, 11)]:
        bits, ev = ggo.significance(s, m, n, lam, K)
        assert ev == pytest.approx(m * n * 2.0 ** -bits, rel=1e-12)


def test_bad_scores(ggo):
    for m, mm in [(0, 3), (1, 0), (-1, 3)]:
        with pytest.raises(ValueError):
            ggo.karlin_altschul(m, mm)
