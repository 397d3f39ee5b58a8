// Device-side modular arithmetic and helpers shared by the HIP kernel files.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ckks_internal.h"
// u2d / d2u and the FP64 arithmetic for moduli below 2^41 (host and device: a host build of the same
// source is checked against 128-bit integers on the CPU)
#include "fmod64.h"

namespace gck {

// ---------------------------------------------------------------- device arithmetic

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// a * w mod q for fixed w with companion wsh = floor(w 2^64 / q); any a < 2^64
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 wsh, u64 q) {
    u64 hi = __umul64hi(a, wsh);
    u64 r = a * w - hi * q;
    return r >= q ? r - q : r;
}

// (hi, lo) * 2^-64 mod q, for hi < q
__device__ __forceinline__ u64 redc(u64 hi, u64 lo, const ModInfo &M) {
    u64 m = lo * M.mont_inv;
    u64 mh = __umul64hi(m, M.q);
    u64 r = hi + mh + (lo != 0 ? 1 : 0);
    return r >= M.q ? r - M.q : r;
}

// a * b mod q for a, b < q
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const ModInfo &M) {
    u64 t = redc(__umul64hi(a, b), a * b, M);
    return mul_shoup(t, M.r_mod, M.r_mod_sh, M.q);
}

// x mod q for any 64-bit x
__device__ __forceinline__ u64 reduce64(u64 x, const ModInfo &M) {
    u64 qh = __umul64hi(x, M.barrett);
    u64 r = x - qh * M.q;
    return r >= M.q ? r - M.q : r;
}

// chain index of limb lam: t = lam mod period is q_t below nq, else special prime p_idx + (t - nq)
__device__ __forceinline__ int chain_of(int lam, ModMap m) {
    int t = lam % m.period;
    return t < m.nq ? m.q_off + t : m.p_idx + (t - m.nq);
}

// NTT-domain automorphism X -> X^g: word k of the result is word k2 of the input, where the evaluation
// point of k2 is that of k raised to g, psi^(2 brev(k2) + 1) = (psi^(2 brev(k) + 1))^g.  The 64 words of
// an aligned group of 64 map into one aligned group of 64 (only the top bits of brev(k) vary).
// The exponents live modulo 2N: 32-bit arithmetic keeps their low bits exactly for log_n <= 30.
__device__ __forceinline__ size_t automorph_src(size_t k, int log_n, u64 g) {
    const unsigned mask2n = (2u << log_n) - 1;
    const unsigned e = 2 * (__brev((unsigned)k) >> (32 - log_n)) + 1;
    const unsigned e2 = (e * (unsigned)g) & mask2n;
    return __brev((e2 - 1) >> 1) >> (32 - log_n);
}

// ---------------------------------------------------------------- SplitMix64 (test-only randomness)

__device__ __forceinline__ u64 sm_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ u64 sm_out(u64 x, u64 i) { return sm_mix(x + (i + 1) * 0x9E3779B97F4A7C15ULL); }

// (w1 2^64 + w2) mod q
__device__ __forceinline__ u64 mod_u128(u64 w1, u64 w2, u64 q) {
    u64 r = w1 % q;
    for (int b = 63; b >= 0; --b) {
        r = (r << 1) | ((w2 >> b) & 1ULL);
        if (r >= q) r -= q;
    }
    return r;
}


// a * w mod q in [0, 2q) (Shoup, no final correction); any a < 2^64
__device__ __forceinline__ u64 mul_shoup_lazy(u64 a, u64 w, u64 wsh, u64 q) {
    return a * w - __umul64hi(a, wsh) * q;
}

// Kernel launch: plain, or with the events of the pending timing record (see KTimer) when a TScope is open.
extern thread_local KTimer::Rec *tl_timed_launch;
template <typename... KArgs, typename... Args>
inline void gck_launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, unsigned shmem, hipStream_t st, Args... args) {
    if (KTimer::Rec *r = tl_timed_launch) {
        tl_timed_launch = nullptr;
        r->launched = true;
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, r->a, r->b, 0u, static_cast<KArgs>(args)...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, static_cast<KArgs>(args)...);
    }
}

// RAII timing scope around one kernel launch (records its events when timing is on)
struct TScope {
    KTimer *t;
    int idx = -1;
    hipStream_t st;
    // bytes: algorithmic HBM bytes of the launch; flops: its algorithmic FP64 operations when the kernel is
    // bound by arithmetic rather than memory (0 otherwise)
    // pass_bytes: the bytes of the launch when each word it touches is read and written once (default: bytes)
    TScope(const DevTables &tab, const char *name, double bytes, hipStream_t s, double flops = 0,
           double pass_bytes = -1)
        : t(tab.timer), st(s) {
        if (t && t->on) idx = t->begin(name, bytes, flops, st, pass_bytes);
    }
    ~TScope() {
        if (idx >= 0) t->end(idx, st);
    }
};

inline void check_launch() { GCK_HIP(hipGetLastError()); }

}  // namespace gck
