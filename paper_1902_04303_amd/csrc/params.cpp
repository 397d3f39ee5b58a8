// Parameters, RNS prime chain and host number theory of the RNS-CKKS library.
//
// The paper describes CKKS with power-of-two moduli (Methods, "Homomorphic
// Encryption"); this is its residue-number-system form.  Chain rule:
//   q_0 = largest prime < 2^60 with q = 1 mod 2N;  P = p_1 ... p_alpha, the alpha largest primes < 2^41
//   with p = 1 mod 2N that are not in the chain (alpha: the digit-group size of the hybrid key switch);
//   pool = the 4L primes = 1 mod 2N nearest to 2^b (lower candidate first on equal distance);
//   for depth d = 0..L-1: q_{L-d} = unused pool prime nearest to Delta_d^2 / 2^b (smaller on ties),
//   Delta_0 = 2^b, Delta_{d+1} = (Delta_d * Delta_d) / q_{L-d} in FP64.
#include <algorithm>
#include <cmath>
#include <set>

#include "ckks_internal.h"

namespace gck {

u64 mulmod_host(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 powmod_host(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod_host(r, b, q);
        b = mulmod_host(b, b, q);
        e >>= 1;
    }
    return r;
}

u64 invmod_host(u64 a, u64 q) { return powmod_host(a % q, q - 2, q); }

static bool is_prime_u64(u64 n) {
    if (n < 2) return false;
    static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : bases) {
        if (n % p == 0) return n == p;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; ++r; }
    for (u64 a : bases) {
        u64 x = powmod_host(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = mulmod_host(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static u64 largest_prime_below(int bits, u64 m) {
    u64 top = (bits >= 64) ? ~0ULL : ((1ULL << bits) - 1);
    u64 c = top / m * m + 1;
    if (c > top) c -= m;
    while (!is_prime_u64(c)) c -= m;
    return c;
}

u64 find_psi(u64 q, int n) {
    u64 m = 2ULL * (u64)n;
    for (u64 g = 2; g < q; ++g) {
        u64 psi = powmod_host(g, (q - 1) / m, q);
        if (powmod_host(psi, (u64)n, q) == q - 1) return psi;
    }
    throw Error(CKKS_E_INVALID_ARG, "no primitive 2N-th root of unity");
}

i64 round_half_away(double x) {
    if (!(std::fabs(x) < 9.2e18)) throw Error(CKKS_E_INVALID_ARG, "constant out of the int64 range");
    return (i64)std::llround(x);
}

Params make_params(int log_n, int levels, int log2_scale, int alpha) {
    if (alpha == 0) alpha = CKKS_DEFAULT_KS_ALPHA;
    if (log_n < 10 || log_n > 17) throw Error(CKKS_E_INVALID_ARG, "log_n must be in [10, 17]");
    if (alpha < 2 || alpha > kMaxAlpha) throw Error(CKKS_E_INVALID_ARG, "ks_alpha must be 0 or in [2, 8]");
    if (levels < 1 || levels + 1 + alpha > kMaxMods) throw Error(CKKS_E_INVALID_ARG, "levels out of range");
    if (log2_scale < 20 || log2_scale > 50) throw Error(CKKS_E_INVALID_ARG, "log2_scale must be in [20, 50]");
    Params p;
    p.log_n = log_n;
    p.n = 1 << log_n;
    p.levels = levels;
    p.log2_scale = log2_scale;
    p.alpha = alpha;
    const u64 m = 2ULL * (u64)p.n;
    const u64 q0 = largest_prime_below(60, m);
    // pool of 4L primes nearest 2^b
    const u64 center = 1ULL << log2_scale;
    std::vector<u64> pool;
    u64 lo = center / m * m + 1;
    if (lo > center) lo -= m;
    u64 hi = lo + m;
    while ((int)pool.size() < 4 * levels) {
        u64 dl = center - lo, dh = hi - center;
        if (dl <= dh) {
            if (lo > 1 && is_prime_u64(lo)) pool.push_back(lo);
            lo -= m;
        } else {
            if (is_prime_u64(hi)) pool.push_back(hi);
            hi += m;
        }
    }
    std::sort(pool.begin(), pool.end());
    std::vector<bool> used(pool.size(), false);
    p.q.assign(levels + 1, 0);
    p.q[0] = q0;
    p.scales.push_back((double)center);
    for (int d = 0; d < levels; ++d) {
        const double s = p.scales[d];
        const double target = (s * s) / (double)center;
        int best = -1;
        double best_dist = 0;
        for (size_t i = 0; i < pool.size(); ++i) {
            if (used[i]) continue;
            double dist = std::fabs((double)pool[i] - target);   // exact: both near 2^b (Sterbenz)
            if (best < 0 || dist < best_dist) { best = (int)i; best_dist = dist; }
        }
        used[best] = true;
        p.q[levels - d] = pool[best];
        p.scales.push_back((s * s) / (double)pool[best]);
    }
    // special primes: the alpha largest primes below 2^41 that are 1 mod 2N and not in the chain
    for (u64 c = ((1ULL << 41) - 1) / m * m + 1; (int)p.P.size() < alpha; c -= m)
        if (is_prime_u64(c) && std::find(p.q.begin(), p.q.end(), c) == p.q.end()) p.P.push_back(c);
    return p;
}

}  // namespace gck
