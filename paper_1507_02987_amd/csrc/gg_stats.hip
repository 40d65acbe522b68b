// Significance of reported alignments: the e-value and normalized (bit) score the
// search returns with each alignment (Section 2.2), by Karlin-Altschul statistics
// of ungapped local alignment (Karlin and Altschul 1990) for +match / -mismatch
// scoring on uniform, independent bases.  Host arithmetic in double precision on
// the few hits a search reports.
#include <cmath>
#include <cstdint>
#include <vector>

#include "gg.h"

namespace {

int32_t gcd_of(int32_t a, int32_t b)
{
    while (b) {
        const int32_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" {

gg_status gg_karlin_altschul(int32_t match, int32_t mismatch, double *lambda, double *K,
                             double *H)
{
    if (match <= 0 || mismatch <= 0 || !lambda || !K || !H) return GG_EINVAL;
    const double p = 0.25, q = 0.75;  // a pair of uniform bases matches with probability 1/4
    const double a = match, b = mismatch;
    // lambda: the positive root of phi(l) = p e^(a l) + q e^(-b l) - 1.  phi is
    // convex, negative just above 0 (the expected score is negative) and positive at
    // ln(1/p)/a, so Newton's method from there decreases monotonically to the root.
    double l = std::log(1.0 / p) / a;
    for (int it = 0; it < 100; ++it) {
        const double ea = std::exp(a * l), eb = std::exp(-b * l);
        const double phi = p * ea + q * eb - 1.0, dphi = p * a * ea - q * b * eb;
        const double next = l - phi / dphi;
        if (!(next < l)) break;  // no further decrease in double precision
        l = next;
    }
    const double h = l * (p * a * std::exp(a * l) - q * b * std::exp(-b * l));
    // sigma = sum over k of (1/k) (E[e^(l S_k); S_k < 0] + P(S_k >= 0)), with the law
    // of S_k (a sum of k pair scores) carried forward by one convolution per step
    // over the scores -k b .. k a
    const int32_t span = match + mismatch;
    std::vector<double> dist(1, 1.0), nxt;  // dist[x] = P(S_k = x - k b)
    double sigma = 0.0;
    for (int32_t k = 1; k <= 20000; ++k) {
        nxt.assign(dist.size() + (size_t)span, 0.0);
        for (size_t x = 0; x < dist.size(); ++x) {
            nxt[x] += q * dist[x];                 // a mismatch: -b
            nxt[x + (size_t)span] += p * dist[x];  // a match: +a (offsets shift by b)
        }
        dist.swap(nxt);
        double term = 0.0;
        const int64_t low = (int64_t)k * mismatch;  // dist[x] holds score x - low
        for (size_t x = 0; x < dist.size(); ++x) {
            const int64_t sc = (int64_t)x - low;
            term += sc < 0 ? dist[x] * std::exp(l * (double)sc) : dist[x];
        }
        sigma += term / k;
        if (term / k < 1e-18) break;
    }
    const double d = gcd_of(match, mismatch);
    *lambda = l;
    *H = h;
    *K = std::exp(-2.0 * sigma) * l * d / (h * -std::expm1(-l * d));
    return GG_OK;
}

gg_status gg_hit_significance(const gg_hit *hits, int64_t n, int64_t query_len, int64_t bank_bases,
                              double lambda, double K, double *bit_score, double *evalue)
{
    if (n < 0 || (n > 0 && (!hits || !bit_score || !evalue)) || query_len < 0 || bank_bases < 0 ||
        !(lambda > 0) || !(K > 0))
        return GG_EINVAL;
    const double lnk = std::log(K), ln2 = std::log(2.0);
    const double space = std::log((double)query_len) + std::log((double)bank_bases);
    for (int64_t i = 0; i < n; ++i) {
        const double s = hits[i].score;
        bit_score[i] = (lambda * s - lnk) / ln2;
        evalue[i] = std::exp(lnk + space - lambda * s);
    }
    return GG_OK;
}

}  // extern "C"
