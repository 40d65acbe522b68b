"""The library's significance statistics (host code, no GPU needed) against the
oracle's: lambda, K and H for several scoring schemes, and the bit scores and
e-values of hit lists, within double-precision rounding.  The two are written
independently (Newton's method and a convolved score law in the library,
bisection and binomial sums in the oracle)."""
import numpy as np
import pytest

from paper_1507_02987_amd import gg


@pytest.mark.parametrize("match,mismatch", [(1, 3), (1, 1), (1, 2), (2, 3), (2, 6), (1, 5),
                                            (3, 4)])
def test_karlin_altschul_matches_oracle(ggo, match, mismatch):
    got = gg.karlin_altschul(match, mismatch)
    want = ggo.karlin_altschul(match, mismatch)
    for g, w in zip(got, want):
        assert g == pytest.approx(w, rel=1e-10)


def test_significance_matches_oracle(ggo):
    lam, K, _ = gg.karlin_altschul(1, 3)
    hits = np.zeros(6, gg.HIT_DTYPE)
    hits["score"] = [1, 17, 30, 100, 600, 5000]
    for m, n in [(500, 2_180_000), (10_000, 3_000_000_000), (80, 275_000_000)]:
        bits, ev = gg.significance(hits, m, n, lam, K)
        for i, s in enumerate(hits["score"]):
            wb, we = ggo.significance(int(s), m, n, lam, K)
            assert bits[i] == pytest.approx(wb, rel=1e-12)
            assert ev[i] == pytest.approx(we, rel=1e-12, abs=1e-300)


def test_bad_arguments():
    with pytest.raises(gg.GGError):
        gg.karlin_altschul(0, 3)
    with pytest.raises(gg.GGError):
        gg.significance(np.zeros(1, gg.HIT_DTYPE), 10, 10, 0.0, 0.7)
