// Exact modular arithmetic on integer-valued doubles for moduli below 2^41, shared by every kernel file
// and compiled for the host as well, where a CPU test checks it against 128-bit integer arithmetic.
//
// A residue is held as a double whose value is an integer.  The product a w of two such integers is
// split exactly into its rounded value h and the FMA error l (a w = h + l); the quotient by q is rounded
// from a multiply by RN(1/q), and the remainder h - qt q is then an integer of magnitude below q, which
// the FMA computes exactly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gck {

#define GCK_HD __host__ __device__ __forceinline__

// exact conversions between integers below 2^52 and doubles through the bias 2^52 (the integer fills the
// mantissa of 2^52 + x): one integer OR or AND and one FP64 add, where a general 64-bit conversion takes
// several instructions
GCK_HD double u2d(uint64_t x) {
#pragma clang fp contract(off)
    return __builtin_bit_cast(double, x | 0x4330000000000000ULL) - 4503599627370496.0;
}
GCK_HD uint64_t d2u(double x) {   // x integer-valued in [0, 2^52)
#pragma clang fp contract(off)
    return __builtin_bit_cast(uint64_t, x + 4503599627370496.0) & 0xFFFFFFFFFFFFFULL;
}

struct FMod {
    double q, qinv;   // q < 2^41 and RN(1 / q)
};

// a w mod q as a signed representative in (-1.1q, 1.1q), exact; a, w integers, |a| < 2^47, 0 <= w < q
GCK_HD double fmul_mod(double a, double w, FMod m) {
#pragma clang fp contract(off)
    const double h = a * w;
    const double l = __builtin_fma(a, w, -h);         // a w = h + l exactly
    const double qt = __builtin_rint(h * m.qinv);
    const double r = __builtin_fma(-qt, m.q, h);      // integer of magnitude < q: exact
    return r + l;
}

// signed reduction of an integer |x| < 2^52 to (-0.6q, 0.6q)
GCK_HD double fred(double x, FMod m) {
#pragma clang fp contract(off)
    const double qt = __builtin_rint(x * m.qinv);
    return __builtin_fma(-qt, m.q, x);
}

// canonical residue in [0, q) of an integer |x| < 2^52, as a 64-bit word
GCK_HD uint64_t fcanon(double x, FMod m) {
#pragma clang fp contract(off)
    const double qt = __builtin_floor(x * m.qinv);
    double r = __builtin_fma(-qt, m.q, x);
    r = r < 0.0 ? r + m.q : r;
    r = r >= m.q ? r - m.q : r;
    return d2u(r);
}

#undef GCK_HD

}  // namespace gck
