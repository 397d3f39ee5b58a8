// Negacyclic NTT over Z_q[X]/(X^N + 1) for gfx950.
//
// Forward: coefficients -> evaluations at psi^(2 brev(k) + 1) stored at index k (bit-reversed
// order), psi a primitive 2N-th root of unity; merged Cooley-Tukey butterflies with the table
// psi_rev[k] = psi^brev(k).  Inverse: Gentleman-Sande butterflies with psi^-brev(k), then N^-1.
//
// N = N1 * N2 in two passes over HBM.  The first log2(N1) stages pair words of the same column
// (index mod N2): pass "cols" runs N1-point sub-transforms down columns; the last log2(N2) stages
// pair words of the same row of N2 contiguous words: pass "rows".  Each block stages a tile of
// 4096 words in LDS; each thread holds 16 words in registers and runs up to four radix-2 stages on
// them before one LDS exchange (a 256-point sub-transform is two register phases).
//
// Two arithmetics, chosen per limb by its modulus:
// * q < 2^41 (the rescale primes): FP64.  Words are integer-valued doubles with signed
//   representatives; a product a w is split exactly into a rounded high part and its FMA error,
//   and the quotient by q is rounded from a multiply by RN(1/q), so the remainder is exact and
//   lies in (-1.1q, 1.1q).  Forward butterflies grow values by at most 1.1q per stage, inverse
//   sums double per stage and are reduced once per register phase; every bound stays below 2^46
//   so all sums and remainders are exact.  Between the two passes a limb holds the doubles' bit
//   patterns; the last pass writes canonical residues in [0, q).
// * otherwise (q_0, P; q < 2^62): 64-bit integers with Shoup multiplications and lazy (Harvey)
//   butterflies: values stay in [0, 4q) (forward) or [0, 2q) (inverse) between stages and are
//   fully reduced on the way out.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "modarith.h"

namespace gck {

namespace {

enum { kGmPlain = 0, kGmConv = 1, kGmEpi = 2 };   // ntt_pass instantiations (see ntt_pass)
constexpr int kLogTileRows = 12;   // rows pass: 16 rows of 256 words per block
constexpr int kLogTileCols = 12;   // cols pass: 16 columns of 256 words per block (32 columns measured slower)
constexpr int kPer = 16;   // words per thread

struct Geom {
    int log_n, n2, log_n1, log_n2;
    int log_g_cols;   // sub-transforms (columns) per cols tile
    int log_g_rows;   // sub-transforms (rows) per rows tile
    int log_tile_cols, log_tile_rows;   // tile sizes of the two passes (log2 words)
    int xcd_group;    // 1: place consecutive logical blocks on one XCD (see block_id)
    const ConvEntry *conv;     // basis-conversion launches: chain of limb lam is conv[lam % conv_period]
    int conv_period;
    const LimbScale *scale;    // inverse: output limb lam scaled by scale[lam % scale_period] (else N^-1)
    int scale_period;
    ModDownEpi epi;
};

__device__ __forceinline__ size_t gathered(const Gather &g, int lam) {
    return (size_t)((lam / g.div) * g.mul + g.add + (lam % g.div) * g.inner);
}

// Logical block of a launch.  Workgroups are handed to the 8 XCDs round-robin (workgroup i to XCD
// i mod 8), each with its own L2.  When several output limbs read the same source limb (ModUp,
// rescale), xcd_group renumbers so that XCD x runs logical blocks [x nb / 8, (x + 1) nb / 8) in order:
// the readers of one source tile then share an L2.  Needs nb divisible by 8.
__device__ __forceinline__ int block_id(const Geom &g) {
    const int b = blockIdx.x;
    if (!g.xcd_group) return b;
    return (b & 7) * (int)(gridDim.x >> 3) + (b >> 3);
}

Geom make_geom(int log_n) {
    Geom g;
    g.log_n = log_n;
    g.log_n1 = (log_n + 1) / 2;   // 256 x 256 at N = 2^16 (128 x 512 measured slower overall)
    g.log_n2 = log_n - g.log_n1;
    g.n2 = 1 << g.log_n2;
    g.log_tile_cols = log_n < kLogTileCols ? log_n : kLogTileCols;
    g.log_tile_rows = log_n < kLogTileRows ? log_n : kLogTileRows;
    g.log_g_cols = g.log_tile_cols - g.log_n1;
    g.log_g_rows = g.log_tile_rows - g.log_n2;
    g.xcd_group = 0;
    g.conv = nullptr;
    g.conv_period = 1;
    g.scale = nullptr;
    g.scale_period = 1;
    g.epi = ModDownEpi{};
    return g;
}

// LDS address of word idx of sub-transform gi, padded by one word per 16 so that the 4 rows of a
// wave access (16 words apart within a row, or 16 column rows apart) fall in different banks.
template <bool ROWS>
__device__ __forceinline__ int lds_addr(int gi, int idx, int log_m, int log_g) {
    if (ROWS) {
        const int m = 1 << log_m;
        return gi * (m + (m >> 4)) + idx + (idx >> 4);
    }
    return (idx << log_g) + gi + (idx >> 4);
}

// One register phase of a sub-transform of size M = 2^LOGM: stages S0 .. S0 + R - 1.
// The thread owns groups gam = q + j * T (T = M / 16 threads per sub-transform), each of 2^R words
// index(k) = hi * (M >> S0) + k * tmin + lo, tmin = M >> (S0 + R), gam = hi * tmin + lo.
// Twiddle of a butterfly at stage s, block i: table[(1 << s) * base_off + i].
template <int LOGM, int S0, int R>
__device__ __forceinline__ int slot_index(int e, int q) {
    constexpr int LOG_TMIN = LOGM - S0 - R;
    const int jg = e >> R, k = e & ((1 << R) - 1);
    const int gam = q + (jg << (LOGM - 4));
    const int hi = gam >> LOG_TMIN, lo = gam & ((1 << LOG_TMIN) - 1);
    return (hi << (LOGM - S0)) + (k << LOG_TMIN) + lo;
}

template <bool INV, int LOGM, int S0, int R>
__device__ __forceinline__ void phase(u64 (&v)[kPer], int q, int base_off, const u64 *__restrict__ W,
                                      const u64 *__restrict__ Ws, u64 qm) {
    constexpr int LOG_TMIN = LOGM - S0 - R;
    constexpr int GPT = kPer >> R;
    const u64 q2 = 2 * qm;
#pragma unroll
    for (int jg = 0; jg < GPT; ++jg) {
        const int gam = q + (jg << (LOGM - 4));
        const int hi = gam >> LOG_TMIN, lo = gam & ((1 << LOG_TMIN) - 1);
        const int base_idx = (hi << (LOGM - S0)) + lo;
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int u = INV ? R - 1 - uu : uu;
            const int s = S0 + u;
            const int half = 1 << (R - 1 - u);
            const int log_t = LOGM - s - 1;
#pragma unroll
            for (int k = 0; k < (1 << R); ++k) {
                if (k & half) continue;
                const int e0 = jg * (1 << R) + k, e1 = e0 + half;
                const int idx = base_idx + (k << LOG_TMIN);
                const int widx = (base_off << s) + (idx >> (log_t + 1));
                const u64 w = W[widx], wsh = Ws[widx];
                if (!INV) {
                    u64 a = v[e0];
                    a = a >= q2 ? a - q2 : a;
                    const u64 t = mul_shoup_lazy(v[e1], w, wsh, qm);
                    v[e0] = a + t;
                    v[e1] = a - t + q2;
                } else {
                    const u64 a = v[e0], b = v[e1];
                    u64 sum = a + b;
                    v[e0] = sum >= q2 ? sum - q2 : sum;
                    v[e1] = mul_shoup_lazy(a - b + q2, w, wsh, qm);
                }
            }
        }
    }
}

template <bool INV, int LOGM, int S0, int R>
__device__ __forceinline__ void fphase(double (&v)[kPer], int q, int base_off, const double *__restrict__ W, FMod m) {
#pragma clang fp contract(off)
    constexpr int LOG_TMIN = LOGM - S0 - R;
    constexpr int GPT = kPer >> R;
#pragma unroll
    for (int jg = 0; jg < GPT; ++jg) {
        const int gam = q + (jg << (LOGM - 4));
        const int hi = gam >> LOG_TMIN, lo = gam & ((1 << LOG_TMIN) - 1);
        const int base_idx = (hi << (LOGM - S0)) + lo;
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int u = INV ? R - 1 - uu : uu;
            const int s = S0 + u;
            const int half = 1 << (R - 1 - u);
            const int log_t = LOGM - s - 1;
#pragma unroll
            for (int k = 0; k < (1 << R); ++k) {
                if (k & half) continue;
                const int e0 = jg * (1 << R) + k, e1 = e0 + half;
                const int idx = base_idx + (k << LOG_TMIN);
                const double w = W[(base_off << s) + (idx >> (log_t + 1))];
                const double a = v[e0], b = v[e1];
                if (!INV) {
                    const double t = fmul_mod(b, w, m);
                    v[e0] = a + t;
                    v[e1] = a - t;
                } else {
                    v[e0] = a + b;
                    v[e1] = fmul_mod(a - b, w, m);
                }
            }
        }
    }
}

template <int LOGM, int PH>
struct Ph {
    static constexpr int S0 = PH * 4;
    static constexpr int R = (LOGM - S0) < 4 ? (LOGM - S0) : 4;
};

// LDS exchange: registers laid out for phase FROM -> LDS -> registers laid out for phase TO
template <bool ROWS, int LOGM, int FROM, int TO, typename T>
__device__ __forceinline__ void exchange(T (&v)[kPer], T *sh, int gi, int q, int log_g) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e)
        sh[lds_addr<ROWS>(gi, slot_index<LOGM, Ph<LOGM, FROM>::S0, Ph<LOGM, FROM>::R>(e, q), LOGM, log_g)] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e)
        v[e] = sh[lds_addr<ROWS>(gi, slot_index<LOGM, Ph<LOGM, TO>::S0, Ph<LOGM, TO>::R>(e, q), LOGM, log_g)];
}

// The register phases of one pass over a tile, with the LDS exchanges between them: FP64 words (the
// inverse reduces the doubled sums before each later phase) and 64-bit integer words (lazy reduction).
template <bool INV, bool ROWS, int LOGM>
__device__ __forceinline__ void fp_phases(double (&f)[kPer], double *shf, int gi, int q, int log_g, int base_off,
                                          const double *__restrict__ Wf, FMod fm) {
    constexpr int NPH = (LOGM + 3) / 4;
    constexpr int FIRST = INV ? NPH - 1 : 0;
    fphase<INV, LOGM, Ph<LOGM, FIRST>::S0, Ph<LOGM, FIRST>::R>(f, q, base_off, Wf, fm);
    if constexpr (NPH > 1) {
        constexpr int P1 = INV ? NPH - 2 : 1;
        exchange<ROWS, LOGM, FIRST, P1>(f, shf, gi, q, log_g);
        if (INV) {
#pragma unroll
            for (int e = 0; e < kPer; ++e) f[e] = fred(f[e], fm);
        }
        fphase<INV, LOGM, Ph<LOGM, P1>::S0, Ph<LOGM, P1>::R>(f, q, base_off, Wf, fm);
        if constexpr (NPH > 2) {
            constexpr int P2 = INV ? NPH - 3 : 2;
            exchange<ROWS, LOGM, P1, P2>(f, shf, gi, q, log_g);
            if (INV) {
#pragma unroll
                for (int e = 0; e < kPer; ++e) f[e] = fred(f[e], fm);
            }
            fphase<INV, LOGM, Ph<LOGM, P2>::S0, Ph<LOGM, P2>::R>(f, q, base_off, Wf, fm);
        }
    }
}

template <bool INV, bool ROWS, int LOGM>
__device__ __forceinline__ void int_phases(u64 (&v)[kPer], u64 *sh, int gi, int q, int log_g, int base_off,
                                           const u64 *__restrict__ W, const u64 *__restrict__ Ws, u64 qm) {
    constexpr int NPH = (LOGM + 3) / 4;
    constexpr int FIRST = INV ? NPH - 1 : 0;
    phase<INV, LOGM, Ph<LOGM, FIRST>::S0, Ph<LOGM, FIRST>::R>(v, q, base_off, W, Ws, qm);
    if constexpr (NPH > 1) {
        constexpr int P1 = INV ? NPH - 2 : 1;
        exchange<ROWS, LOGM, FIRST, P1>(v, sh, gi, q, log_g);
        phase<INV, LOGM, Ph<LOGM, P1>::S0, Ph<LOGM, P1>::R>(v, q, base_off, W, Ws, qm);
        if constexpr (NPH > 2) {
            constexpr int P2 = INV ? NPH - 3 : 2;
            exchange<ROWS, LOGM, P1, P2>(v, sh, gi, q, log_g);
            phase<INV, LOGM, Ph<LOGM, P2>::S0, Ph<LOGM, P2>::R>(v, q, base_off, W, Ws, qm);
        }
    }
}

// One pass.  ROWS selects the rows pass (sub-transforms of N2 contiguous words) or the cols pass
// (N1-point sub-transforms down columns).  `in` (first pass only) gathers the input from another buffer;
// GM selects a separate instantiation for the work only some launches do, so that the other passes do
// not carry its registers: kGmConv (forward cols pass) is the basis-conversion gather, kGmEpi (forward
// rows pass) the ModDown epilogue.  At least 3 waves per SIMD (up to 168 VGPRs): the passes
// then run without spills, faster than at 4 waves with spills.
template <bool INV, bool ROWS, int LOGM, int GM>
__global__ void __launch_bounds__((1 << (ROWS ? kLogTileRows : kLogTileCols)) / kPer, 3) ntt_pass(u64 *__restrict__ buf, Gather in, ModMap mm,
                                                     const ModInfo *__restrict__ mods, const u64 *__restrict__ tw,
                                                     const u64 *__restrict__ tw_sh,
                                                     const double *__restrict__ tw_f, Geom g) {
    constexpr int LT = ROWS ? kLogTileRows : kLogTileCols;
    constexpr bool CONV = GM == kGmConv;
    __shared__ u64 sh[(1 << LT) + ((1 << LT) >> 4)];
    constexpr int NPH = (LOGM + 3) / 4;
    constexpr int FIRST = INV ? NPH - 1 : 0;
    constexpr int LAST = INV ? 0 : NPH - 1;
    const int log_tile = ROWS ? g.log_tile_rows : g.log_tile_cols;
    const int bid = block_id(g);
    const int limb = bid >> (g.log_n - log_tile);
    const int tile = bid & ((1 << (g.log_n - log_tile)) - 1);
    // a basis-conversion NTT takes every output limb's modulus from its conversion entry, in both passes
    const ConvEntry *ce = g.conv ? g.conv + limb % g.conv_period : nullptr;
    const int chain = ce ? ce->chain : chain_of(limb, mm);
    const ModInfo M = mods[chain];
    const u64 qm = M.q;
    const size_t n = (size_t)1 << g.log_n;
    const u64 *W = tw + (size_t)chain * n, *Ws = tw_sh + (size_t)chain * n;
    const int log_g = ROWS ? g.log_g_rows : g.log_g_cols;
    constexpr int LOG_T = LOGM - 4;
    const int tid = threadIdx.x;
    int gi, q;
    if (ROWS) {
        q = tid & ((1 << LOG_T) - 1);
        gi = tid >> LOG_T;
    } else {
        gi = tid & ((1 << log_g) - 1);
        q = tid >> log_g;
    }
    u64 *a = buf + (size_t)limb * n;
    const u64 *ain = a;
    int mode = kPlain;
    u64 src_q = 0, src_half = 0, src_q_red = 0;
    if (CONV) {
        mode = kConv;
        ain = in.ptr + ((size_t)(limb / g.conv_period) * in.src_stride + ce->src) * n;
    } else if (in.ptr) {
        const int sl = (limb / in.div) * in.mul + in.add + (limb % in.div) * in.inner;
        ain = in.ptr + (size_t)sl * n;
        mode = in.mode;
        if (mode == kCentred) {
            src_q = mods[in.src_chain].q;
            src_half = src_q >> 1;
            src_q_red = reduce64(src_q, M);
        }
    }
    size_t base;
    int stride, base_off;
    if (ROWS) {
        const int row = (tile << log_g) + gi;
        base = (size_t)row << g.log_n2;
        stride = 1;
        base_off = (1 << g.log_n1) + row;
    } else {
        base = (size_t)(tile << log_g) + gi;
        stride = g.n2;
        base_off = 1;
    }
    const bool last_pass = INV ? !ROWS : ROWS;
    // global loads in the layout of the first phase; stores of the rows pass go through LDS so that a
    // wave instruction covers 16 consecutive words of each of 4 rows (an LDS transposition in the cols
    // passes, loads or stores, measured slower than the strided access it replaces)
    u64 v[kPer];
    if constexpr (CONV) {
        // basis conversion while loading: sum_m y_m c_m mod q over the source limbs, 8 words at a time with
        // the next 8 words' loads issued before the current 8 are converted (double buffer); FP64 moduli
        // keep the sum as a double (|sum| < 1.1 q per source, below 2^45 for up to kMaxSpecial sources)
        // and store its bits
        const int ns = ce->nsrc, big = ce->big, centre = ce->centre;
        const FMod fm{M.qd, M.qinv};
        if (M.fp) {
            constexpr int H = kPer / 2;
            double x[kPer];
#pragma unroll
            for (int e = 0; e < kPer; ++e) x[e] = 0.0;
            // buffer 0 holds words 0..H-1 of a source, buffer 1 words H..2H-1
            u64 y0[H], y1[H];
            auto load = [&](u64 (&yb)[H], int m, int h) {
                const u64 *src = ain + (size_t)m * n + base;
#pragma unroll
                for (int e = 0; e < H; ++e)
                    yb[e] = src[(size_t)slot_index<LOGM, Ph<LOGM, FIRST>::S0, Ph<LOGM, FIRST>::R>(h + e, q) * stride];
            };
            auto convert = [&](const u64 (&yb)[H], double *xh, int m) {
                const double w = ce->cd[m];
                const bool split = (big >> m) & 1;
                // centred sources (never split): y - s when y > s / 2, |y - s| < 2^41
                const u64 half = centre ? ce->half[m] : ~0ULL;
                const double sqd = ce->sqd[m];
#pragma unroll
                for (int e = 0; e < H; ++e) {
                    const u64 y = yb[e];
                    double a = split ? fred(fmul_mod((double)(unsigned)(y >> 32), M.c32_d, fm) +
                                                (double)(unsigned)(y & 0xFFFFFFFFULL), fm)
                                     : u2d(y);
                    a = y > half ? a - sqd : a;
                    xh[e] += fmul_mod(a, w, fm);
                }
            };
            load(y0, 0, 0);
            for (int m = 0; m < ns; ++m) {
                load(y1, m, H);
                convert(y0, x, m);
                if (m + 1 < ns) load(y0, m + 1, 0);
                convert(y1, x + H, m);
            }
#pragma unroll
            for (int e = 0; e < kPer; ++e) v[e] = (u64)__double_as_longlong(fred(x[e], fm));
        } else {
#pragma unroll
            for (int e = 0; e < kPer; ++e) v[e] = 0;
            for (int m = 0; m < ns; ++m) {
                const u64 *src = ain + (size_t)m * n + base;
                const u64 w = ce->c[m], wsh = ce->c_sh[m];
                const u64 half = centre ? ce->half[m] : ~0ULL, negsq = ce->negsq[m];   // y - s = y + negsq
#pragma unroll
                for (int h = 0; h < kPer; h += kPer / 2) {
                    u64 y[kPer / 2];
#pragma unroll
                    for (int e = 0; e < kPer / 2; ++e)
                        y[e] = src[(size_t)slot_index<LOGM, Ph<LOGM, FIRST>::S0, Ph<LOGM, FIRST>::R>(h + e, q) * stride];
#pragma unroll
                    for (int e = 0; e < kPer / 2; ++e) {
                        const u64 yc = y[e] > half ? y[e] + negsq : y[e];
                        v[h + e] = add_mod(v[h + e], mul_shoup(yc, w, wsh, qm), qm);
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = slot_index<LOGM, Ph<LOGM, FIRST>::S0, Ph<LOGM, FIRST>::R>(e, q);
            v[e] = ain[base + (size_t)idx * stride];
        }
        if (mode == kCentred && in.cmul) {   // a rescale of k a: the source residue times k, then centred
#pragma unroll
            for (int e = 0; e < kPer; ++e) v[e] = mul_shoup(v[e], in.cmul, in.cmul_sh, src_q);
        }
    }
    if (M.fp) {
        // FP64 butterflies; the first pass reads residues, the second the first pass's doubles
        const FMod fm{M.qd, M.qinv};
        const double *Wf = tw_f + (size_t)chain * n;
        double f[kPer];
        if (last_pass || CONV) {
#pragma unroll
            for (int e = 0; e < kPer; ++e) f[e] = __longlong_as_double((long long)v[e]);
        } else if (mode == kPlain) {
#pragma unroll
            for (int e = 0; e < kPer; ++e) f[e] = u2d(v[e]);
        } else {
            // any word x < 2^64 taken mod q as (x >> 32) (2^32 mod q) + (x mod 2^32); a centred source
            // residue above half its modulus also subtracts that modulus
            const double sq = (double)src_q_red;
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                const u64 x = v[e];
                double y = fmul_mod((double)(unsigned)(x >> 32), M.c32_d, fm) + (double)(unsigned)(x & 0xFFFFFFFFULL);
                if (mode == kCentred && x > src_half) y -= sq;
                f[e] = fred(y, fm);
            }
        }
        fp_phases<INV, ROWS, LOGM>(f, reinterpret_cast<double *>(sh), gi, q, log_g, base_off, Wf, fm);
        const double sc = (INV && !ROWS && g.scale) ? g.scale[limb % g.scale_period].wd : M.ninv_d;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            double x = f[e];
            if (INV && !ROWS) x = fmul_mod(x, sc, fm);
            v[e] = last_pass ? fcanon(x, fm) : (u64)__double_as_longlong(fred(x, fm));
        }
    } else {
        if (!CONV && !last_pass && mode != kPlain) {
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                u64 x = v[e];
                const bool neg = (mode == kCentred) && x > src_half;
                x = reduce64(x, M);
                if (neg) x = x >= src_q_red ? x - src_q_red : x + qm - src_q_red;   // x - src_q is negative
                v[e] = x;
            }
        }
        int_phases<INV, ROWS, LOGM>(v, sh, gi, q, log_g, base_off, W, Ws, qm);
        // final scaling (inverse cols pass: N^-1) and reduction ([0, q) at the end of a transform)
        const u64 q2 = 2 * qm;
        u64 sw = M.ninv, sw_sh = M.ninv_sh;
        if (INV && !ROWS && g.scale) {
            sw = g.scale[limb % g.scale_period].w;
            sw_sh = g.scale[limb % g.scale_period].w_sh;
        }
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            u64 x = v[e];
            if (INV && !ROWS) x = mul_shoup_lazy(x, sw, sw_sh, qm);
            x = x >= q2 ? x - q2 : x;
            if (last_pass) x = x >= qm ? x - qm : x;
            v[e] = x;
        }
    }
    if (ROWS && LAST != 0) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kPer; ++e)
            sh[lds_addr<ROWS>(gi, slot_index<LOGM, Ph<LOGM, LAST>::S0, Ph<LOGM, LAST>::R>(e, q), LOGM, log_g)] = v[e];
        __syncthreads();
        if constexpr (!INV && GM == kGmEpi) {
            // ModDown epilogue: (acc - t) P^-1 (+ add) (+ automorphism term), t the transform just computed
            const ModDownEpi &E = g.epi;
            const u64 *xa = E.acc.ptr + gathered(E.acc, limb) * n;
            const bool even = ((limb / E.rowlen) & 1) == 0;
            const bool with_add = E.add.ptr && (!E.add_even || even);
            const int arow = limb / E.rowlen;
            const u64 *xd = !with_add ? nullptr
                            : E.add_ct ? E.add.ptr + ((size_t)(arow >> 1) * E.add_ct + (size_t)(arow & 1) * E.add_poly +
                                                      (size_t)(limb % E.rowlen)) * n
                                       : E.add.ptr + gathered(E.add, limb) * n;
            const u64 *xs = E.aut ? E.aut + (size_t)limb * n : nullptr;
            const int n_aut = (xs && even) ? E.n_g : 0;
            // aut_self 1: the ciphertext itself on every row; 2: on odd rows only (the even rows' term comes
            // summed in add)
            const bool aut_self = xs && (E.aut_self == 1 || (E.aut_self == 2 && !even));
            if (M.fp) {
                // FP64: |acc - t| < q, the product's remainder below 1.1 q, each added residue below q: the
                // sum stays below 20 q for up to 16 automorphism terms, well inside the exact range (the
                // sums of two residues below 2^42 are exact as well)
                const FMod fm{M.qd, M.qinv};
                const double pd = E.pinv_d[chain];
                // every load of a group of EG words is issued before the group's stores (the stores could
                // otherwise alias later loads for the compiler)
                constexpr int EG = 4, AU = 3;   // words per group, automorphism terms loaded ahead
#pragma unroll
                for (int e0 = 0; e0 < kPer; e0 += EG) {
                    u64 va[EG], vt[EG], vd[EG], vs[EG], vp[AU][EG];
#pragma unroll
                    for (int j = 0; j < EG; ++j) {
                        const size_t w = base + slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e0 + j, q);
                        vt[j] = sh[lds_addr<ROWS>(gi, slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e0 + j, q), LOGM, log_g)];
                        va[j] = __builtin_nontemporal_load(xa + w);   // read once: kept out of the caches
                        vd[j] = with_add ? __builtin_nontemporal_load(xd + w) : 0;
                        vs[j] = aut_self ? xs[w] : 0;
#pragma unroll
                        for (int i = 0; i < AU; ++i) vp[i][j] = i < n_aut ? xs[automorph_src(w, g.log_n, E.g[i])] : 0;
                    }
                    double r[EG];
                    const double kmul = E.acc_mul ? u2d(E.km[chain]) : 0.0;
                    const double amul = E.addmul_d ? E.addmul_d[chain] : 0.0;
#pragma unroll
                    for (int j = 0; j < EG; ++j) {
                        const double av = E.acc_mul ? fmul_mod(u2d(va[j]), kmul, fm) : u2d(va[j]);
                        r[j] = fmul_mod(av - u2d(vt[j]), pd, fm);
                        r[j] += (E.addmul_d ? fmul_mod(u2d(vd[j]), amul, fm) : u2d(vd[j])) + u2d(vs[j]);
#pragma unroll
                        for (int i = 0; i < AU; ++i) r[j] += u2d(vp[i][j]);
                    }
                    // further automorphism terms AU at a time, the loads of a batch issued together
                    for (int i0 = AU; i0 < n_aut; i0 += AU) {
#pragma unroll
                        for (int j = 0; j < EG; ++j) {
                            const size_t w = base + slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e0 + j, q);
#pragma unroll
                            for (int i = 0; i < AU; ++i)
                                vp[i][j] = i0 + i < n_aut ? xs[automorph_src(w, g.log_n, E.g[i0 + i])] : 0;
                        }
#pragma unroll
                        for (int j = 0; j < EG; ++j)
#pragma unroll
                            for (int i = 0; i < AU; ++i) r[j] += u2d(vp[i][j]);
                    }
#pragma unroll
                    for (int j = 0; j < EG; ++j) {
                        const size_t w = base + slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e0 + j, q);
                        __builtin_nontemporal_store(fcanon(r[j], fm), a + w);
                    }
                }
            } else {
                const u64 pv = E.pinv[chain], ps = E.pinv_sh[chain];
#pragma unroll
                for (int e = 0; e < kPer; ++e) {
                    const int idx = slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e, q);
                    const u64 t = sh[lds_addr<ROWS>(gi, idx, LOGM, log_g)];
                    const u64 av = E.acc_mul ? mul_mod(xa[base + idx], E.km[chain], M) : xa[base + idx];
                    u64 r = mul_shoup(sub_mod(av, t, qm), pv, ps, qm);
                    if (with_add)
                        r = add_mod(r, E.addmul ? mul_shoup(xd[base + idx], E.addmul[chain], E.addmul_sh[chain], qm)
                                                : xd[base + idx], qm);
                    if (aut_self) r = add_mod(r, xs[base + idx], qm);
                    for (int i = 0; i < n_aut; ++i) r = add_mod(r, xs[automorph_src(base + idx, g.log_n, E.g[i])], qm);
                    a[base + idx] = r;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                const int idx = slot_index<LOGM, 0, Ph<LOGM, 0>::R>(e, q);
                a[base + idx] = sh[lds_addr<ROWS>(gi, idx, LOGM, log_g)];
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = slot_index<LOGM, Ph<LOGM, LAST>::S0, Ph<LOGM, LAST>::R>(e, q);
            a[base + (size_t)idx * stride] = v[e];
        }
    }
}

template <bool INV, bool ROWS, int GM = kGmPlain>
void launch_pass(int log_m, dim3 grid, dim3 block, hipStream_t st, u64 *buf, const Gather &in, ModMap m,
                 const ModInfo *mods, const u64 *tw, const u64 *tws, const double *twf, Geom g) {
    switch (log_m) {
#define GCK_NTT_CASE(L)                                                                                   \
    case L:                                                                                               \
        gck_launch((ntt_pass<INV, ROWS, L, GM>), grid, block, 0, st, buf, in, m, mods, tw, tws, twf, g); \
        break;
        GCK_NTT_CASE(5)
        GCK_NTT_CASE(6)
        GCK_NTT_CASE(7)
        GCK_NTT_CASE(8)
        GCK_NTT_CASE(9)
#undef GCK_NTT_CASE
    default:
        throw Error(CKKS_E_INVALID_ARG, "unsupported NTT sub-transform size");
    }
}

}  // namespace

// timing names: the kernel symbols as a profiler lists them
static const char *pass_name(bool inv, bool rows, int log_m, int gm) {
    static const std::vector<std::string> names = [] {   // index ((inv * 2 + rows) * 3 + gm) * 5 + log_m - 5
        std::vector<std::string> v;
        const char *tf[2] = {"false", "true"};
        for (int i = 0; i < 2; ++i)
            for (int r = 0; r < 2; ++r)
                for (int g = 0; g < 3; ++g)
                    for (int lm = 5; lm <= 9; ++lm)
                        v.push_back(std::string("ntt_pass<") + tf[i] + ", " + tf[r] + ", " + std::to_string(lm) + ", " +
                                    std::to_string(g) + ">");
        return v;
    }();
    return names[(((inv ? 1 : 0) * 2 + (rows ? 1 : 0)) * 3 + gm) * 5 + (log_m - 5)].c_str();
}

static void launch(const DevTables &t, u64 *buf, const Gather &in, int n_limbs, ModMap m, bool inv, hipStream_t st,
                   const LimbScale *scale = nullptr, int scale_period = 1, const ModDownEpi *epi = nullptr) {
    if (n_limbs <= 0) return;
    if (t.log_n < 10 || t.log_n > 17) throw Error(CKKS_E_INVALID_ARG, "NTT needs 2^10 <= N <= 2^17");
    Geom g = make_geom(t.log_n);
    if (in.ptr && in.mode == kConv) {
        if (inv || !in.conv || in.conv_period < 1) throw Error(CKKS_E_INVALID_ARG, "basis conversion needs a forward NTT");
        g.conv = in.conv;
        g.conv_period = in.conv_period;
    }
    if (scale) {
        if (!inv || scale_period < 1) throw Error(CKKS_E_INVALID_ARG, "limb scales apply to inverse NTTs");
        g.scale = scale;
        g.scale_period = scale_period;
    }
    Geom g_rows = g;   // the epilogue applies to the forward rows pass only
    if (epi) {
        if (inv) throw Error(CKKS_E_INVALID_ARG, "the ModDown epilogue ends a forward NTT");
        g_rows.epi = *epi;
    }
    const dim3 grid_c((unsigned)((size_t)n_limbs << (t.log_n - g.log_tile_cols)));
    const dim3 block_c((unsigned)((1 << g.log_tile_cols) / kPer));
    const dim3 grid_r((unsigned)((size_t)n_limbs << (t.log_n - g.log_tile_rows)));
    const dim3 block_r((unsigned)((1 << g.log_tile_rows) / kPer));
    // Algorithmic bytes of a transform: each distinct input word read once and each output word written
    // once, 16 N per limb (a gather whose output limbs share a source limb, inner == 0, reads n_limbs / div
    // source limbs; a basis conversion reads its source limbs once).  The first pass is credited with the
    // reads and the second with the writes; the words the first pass writes and the second reads again
    // are the price of the two-pass design and count only in the pass bytes (each pass reading and
    // writing every word once).
    const double bytes = 16.0 * (double)n_limbs * t.n;
    const bool conv = in.ptr && in.mode == kConv;
    const bool shared_src = conv || (in.ptr && in.div > 1 && in.inner == 0);
    const double src_limbs = conv ? (double)(n_limbs / in.conv_period) * in.src_stride : (double)n_limbs / in.div;
    const double bytes1 = shared_src ? 8.0 * t.n * ((double)n_limbs + src_limbs) : bytes;
    const double alg_read = 8.0 * t.n * (shared_src ? src_limbs : (double)n_limbs);
    const double alg_write = 8.0 * t.n * (double)n_limbs;
    const Gather none{nullptr, 1, 1, 0, 0, kPlain, 0};
    auto name = [&](bool i, bool rows, int log_m, int gm = kGmPlain) { return pass_name(i, rows, log_m, gm); };
    Geom g1 = g;   // first pass: group the readers of a shared source limb on one XCD
    g1.xcd_group = (shared_src && (inv ? grid_r.x : grid_c.x) % 8 == 0) ? 1 : 0;
    if (!inv) {
        {
            TScope ts_(t, name(false, false, g.log_n1, conv ? kGmConv : kGmPlain), alg_read, st, 0, bytes1);
            if (conv)
                launch_pass<false, false, kGmConv>(g.log_n1, grid_c, block_c, st, buf, in, m, t.mods, t.psi, t.psi_sh, t.psi_f, g1);
            else
                launch_pass<false, false>(g.log_n1, grid_c, block_c, st, buf, in, m, t.mods, t.psi, t.psi_sh, t.psi_f, g1);
        }
        {
            // epilogue reads: acc, the added term, the automorphism source (each distinct word once)
            const double epi_bytes =
                epi ? 8.0 * t.n * n_limbs *
                          (1.0 + (epi->add.ptr ? (epi->add_even ? 0.5 : 1.0) : 0.0) +
                           (epi->aut ? (epi->aut_self == 1 ? 1.0 : 0.5) : 0.0))
                    : 0.0;
            TScope ts_(t, name(false, true, g.log_n2, epi ? kGmEpi : kGmPlain), alg_write + epi_bytes, st, 0,
                       bytes + epi_bytes);
            if (epi)
                launch_pass<false, true, kGmEpi>(g.log_n2, grid_r, block_r, st, buf, none, m, t.mods, t.psi, t.psi_sh, t.psi_f, g_rows);
            else
                launch_pass<false, true>(g.log_n2, grid_r, block_r, st, buf, none, m, t.mods, t.psi, t.psi_sh, t.psi_f, g_rows);
        }
    } else {
        {
            TScope ts_(t, name(true, true, g.log_n2), alg_read, st, 0, bytes1);
            launch_pass<true, true>(g.log_n2, grid_r, block_r, st, buf, in, m, t.mods, t.ipsi, t.ipsi_sh, t.ipsi_f, g1);
        }
        {
            TScope ts_(t, name(true, false, g.log_n1), alg_write, st, 0, bytes);
            launch_pass<true, false>(g.log_n1, grid_c, block_c, st, buf, none, m, t.mods, t.ipsi, t.ipsi_sh, t.ipsi_f, g);
        }
    }
    check_launch();
}

void k_ntt_forward(const DevTables &t, u64 *buf, int n_limbs, ModMap m, hipStream_t st) {
    launch(t, buf, Gather{nullptr, 1, 1, 0, 0, kPlain, 0}, n_limbs, m, false, st);
}

void k_ntt_inverse(const DevTables &t, u64 *buf, int n_limbs, ModMap m, hipStream_t st) {
    launch(t, buf, Gather{nullptr, 1, 1, 0, 0, kPlain, 0}, n_limbs, m, true, st);
}

void k_ntt_forward_g(const DevTables &t, u64 *buf, const Gather &in, int n_limbs, ModMap m, hipStream_t st,
                     const ModDownEpi *epi) {
    launch(t, buf, in, n_limbs, m, false, st, nullptr, 1, epi);
}

void k_ntt_inverse_g(const DevTables &t, u64 *buf, const Gather &in, int n_limbs, ModMap m, hipStream_t st,
                     const LimbScale *scale, int scale_period) {
    launch(t, buf, in, n_limbs, m, true, st, scale, scale_period);
}


}  // namespace gck
