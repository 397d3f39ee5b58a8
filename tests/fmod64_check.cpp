// Host check of the device's FP64 modular arithmetic (paper_1902_04303_amd/csrc/fmod64.h) against
// 128-bit integer arithmetic.  TEST INFRASTRUCTURE: built and run by tests/test_fmod64_host.py.
//
// usage: fmod64_check TRIALS q_1 q_2 ...   (each q odd, below 2^41)
// For every modulus, edge inputs and TRIALS seeded random inputs are checked:
//   fmul_mod(a, w): |a| < 2^47, 0 <= w < q  ->  r = a w (mod q), r integer-valued, |r| < 1.1 q
//   fred(x):        |x| < 2^52              ->  r = x (mod q), |r| < 0.6 q
//   fcanon(x):      |x| < 2^52              ->  x mod q in [0, q)
//   d2u(u2d(x)) = x for 0 <= x < 2^52
// Prints "ok <cases>" and exits 0, or prints the first failing case and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1902_04303_amd/csrc/fmod64.h"

using gck::FMod;
typedef __int128 i128;
typedef unsigned long long u64;
typedef long long i64;

static u64 g_state = 0x243F6A8885A308D3ULL;
static u64 next64() {   // SplitMix64 (Steele, Lea, Flood 2014)
    u64 z = (g_state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static i64 rand_signed(int bits) {   // uniform in (-2^bits, 2^bits)
    i64 v = (i64)(next64() >> (64 - bits));
    return (next64() & 1) ? -v : v;
}

static i128 mod_pos(i128 x, i128 q) {
    i128 r = x % q;
    return r < 0 ? r + q : r;
}

static long n_cases = 0;

static bool is_int(double d) { return std::floor(d) == d; }

static void fail(const char *what, u64 q, i64 a, i64 w, double r) {
    std::printf("FAIL %s q=%llu a=%lld w=%lld r=%.17g\n", what, q, a, w, r);
    std::exit(1);
}

static void check_mul(u64 q, const FMod &m, i64 a, i64 w) {
    ++n_cases;
    const double r = gck::fmul_mod((double)a, (double)w, m);
    if (!is_int(r) || std::fabs(r) >= 1.1 * (double)q) fail("fmul_mod bound", q, a, w, r);
    if (mod_pos((i128)a * w - (i128)(i64)r, (i128)q) != 0) fail("fmul_mod residue", q, a, w, r);
}

static void check_red(u64 q, const FMod &m, i64 x) {
    ++n_cases;
    const double r = gck::fred((double)x, m);
    if (!is_int(r) || std::fabs(r) >= 0.6 * (double)q) fail("fred bound", q, x, 0, r);
    if (mod_pos((i128)x - (i128)(i64)r, (i128)q) != 0) fail("fred residue", q, x, 0, r);
    ++n_cases;
    const u64 c = gck::fcanon((double)x, m);
    if ((i128)c != mod_pos((i128)x, (i128)q)) fail("fcanon", q, x, 0, (double)c);
}

int main(int argc, char **argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s TRIALS q...\n", argv[0]);
        return 2;
    }
    const long trials = std::atol(argv[1]);
    const i64 A_MAX = (1LL << 47) - 1, X_MAX = (1LL << 52) - 1;
    for (u64 x : {0ULL, 1ULL, 12345ULL, (1ULL << 41) - 1, (1ULL << 52) - 1}) {
        ++n_cases;
        if (gck::d2u(gck::u2d(x)) != x || gck::u2d(x) != (double)x) fail("u2d/d2u", 0, (i64)x, 0, gck::u2d(x));
    }
    for (int i = 2; i < argc; ++i) {
        const u64 q = std::strtoull(argv[i], nullptr, 10);
        if (q < 3 || q % 2 == 0 || q >= (1ULL << 41)) {
            std::fprintf(stderr, "bad modulus %llu\n", q);
            return 2;
        }
        const FMod m{(double)q, 1.0 / (double)q};
        const i64 qs = (i64)q;
        // edge operands: 0, +-1, +-(q-1), +-q, near +-2^47, multiples of q and half of q
        std::vector<i64> as = {0, 1, -1, qs - 1, -(qs - 1), qs, -qs, qs + 1, A_MAX, -A_MAX, A_MAX - 1, -(A_MAX - 1),
                               (A_MAX / qs) * qs, -(A_MAX / qs) * qs, (A_MAX / qs) * qs - 1, qs / 2, -(qs / 2)};
        std::vector<i64> ws = {0, 1, 2, qs - 1, qs - 2, qs / 2, qs / 2 + 1, qs / 3};
        for (i64 a : as)
            for (i64 w : ws) check_mul(q, m, a, w);
        std::vector<i64> xs = {0, 1, -1, qs - 1, -(qs - 1), qs, -qs, qs / 2, -(qs / 2), qs / 2 + 1, -(qs / 2 + 1),
                               X_MAX, -X_MAX, (X_MAX / qs) * qs, -(X_MAX / qs) * qs, (X_MAX / qs) * qs + qs / 2,
                               -((X_MAX / qs) * qs + qs / 2), (X_MAX / qs) * qs - 1};
        for (i64 x : xs) check_red(q, m, x);
        for (long t = 0; t < trials; ++t) {
            check_mul(q, m, rand_signed(47), (i64)(next64() % q));
            check_red(q, m, rand_signed(52));
            // products of two residues as the NTT and key switch form them (|a| < q, w < q)
            check_mul(q, m, (i64)(next64() % (2 * q)) - qs, (i64)(next64() % q));
        }
    }
    std::printf("ok %ld\n", n_cases);
    return 0;
}
