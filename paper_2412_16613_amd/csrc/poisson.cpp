// Poisson inverse-CDF tables for the event budgets, in IEEE binary128.
//
// The ghost reactions make the total propensity a constant (Eq. (9) of the
// paper), so the waiting times of Eq. (8) form a Poisson process independent
// of the reactions that fire.  With the padded total 2^B, the number of
// events of a replica in a time interval is Poisson with mean
// mu = lambda * dt.  A replica draws it from one 64-bit uniform u by
// inversion against
//     T[j] = floor(2^64 P(K <= k_lo + j)),   K = k_lo + #{j : T[j] <= u}.
// k_lo is the smallest k with T >= 1; the table ends at the first entry
// equal to 2^64 - 1.
//
// Accuracy: log p(mode) is evaluated with the Stirling series in the form
// m log1p(delta) - m delta - log(2 pi m)/2 - S(m), which avoids the
// cancellation of -mu + m log mu - lgamma(m+1) for large m; the other
// probabilities follow by the ratios mu/k and k/mu.  The relative error of
// the CDF stays near 1e-30, so an entry differs from the exact floor only
// when 2^64 F lies within ~1e-10 of an integer.

#include <quadmath.h>
#include <stdint.h>

#include <cmath>
#include <vector>

namespace bwg {

static __float128 log_pmf_at(int64_t m, __float128 mu)
{
    if (m < 1000) return -mu + (__float128)m * logq(mu) - lgammaq((__float128)m + 1);
    const __float128 M = (__float128)m;
    const __float128 delta = (mu - M) / M;
    // lgamma(m+1) = m ln m - m + ln(2 pi m)/2 + S(m),
    // S(m) = 1/(12m) - 1/(360m^3) + 1/(1260m^5) - 1/(1680m^7) + 1/(1188m^9)
    //        - 691/(360360m^11) + 1/(156m^13)
    const __float128 r = 1 / M, r2 = r * r;
    __float128 S = (__float128)1 / 156;
    S = S * r2 - (__float128)691 / 360360;
    S = S * r2 + (__float128)1 / 1188;
    S = S * r2 - (__float128)1 / 1680;
    S = S * r2 + (__float128)1 / 1260;
    S = S * r2 - (__float128)1 / 360;
    S = S * r2 + (__float128)1 / 12;
    S = S * r;
    return M * (log1pq(delta) - delta) - logq(2 * M_PIq * M) / 2 - S;
}

// Returns 0 on success, -1 for an invalid mean.
int poisson_table_q(double mu_d, int64_t *k_lo_out, std::vector<uint64_t> &T)
{
    T.clear();
    if (!(mu_d >= 0) || std::isinf(mu_d)) return -1;
    if (mu_d == 0.0) {
        *k_lo_out = 0;
        T.push_back(~0ull);
        return 0;
    }
    const __float128 mu = (__float128)mu_d;
    const int64_t mode = (int64_t)mu_d;  // floor for mu >= 0
    const __float128 p_mode = expq(log_pmf_at(mode, mu));
    const __float128 tiny = 1e-60Q;
    // pmf below the mode down to a negligible tail
    std::vector<__float128> lower;
    {
        __float128 p = p_mode;
        int64_t k = mode;
        while (k > 0) {
            p = p * (__float128)k / mu;
            --k;
            lower.push_back(p);
            if (p < tiny) break;
        }
    }
    const __float128 two64 = 18446744073709551616.0Q;
    __float128 F = 0;
    bool started = false;
    int64_t k_lo = 0;
    auto push = [&](int64_t k, __float128 p) -> bool {
        F += p;
        __float128 x = floorq(F * two64);
        uint64_t t;
        if (x >= two64 - 1)
            t = ~0ull;
        else
            t = (uint64_t)x;
        if (!started) {
            if (t < 1) return false;
            started = true;
            k_lo = k;
        }
        T.push_back(t);
        return t == ~0ull;
    };
    // lower[idx] holds p(mode - 1 - idx): walk it from the bottom up
    for (int64_t idx = (int64_t)lower.size() - 1; idx >= 0; --idx) {
        if (push(mode - 1 - idx, lower[idx])) {
            *k_lo_out = k_lo;
            return 0;
        }
    }
    __float128 p = p_mode;
    int64_t k = mode;
    for (;;) {
        if (push(k, p)) break;
        ++k;
        p = p * mu / (__float128)k;
        if (k > mode + 100000000) return -1;
    }
    *k_lo_out = k_lo;
    return 0;
}

}  // namespace bwg
