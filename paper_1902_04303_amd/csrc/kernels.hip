// HIP kernels of the RNS-CKKS evaluator for gfx950 (CDNA4).
//
// All arithmetic is exact modular arithmetic on residues in [0, q), stored as
// 64-bit words, on the vector ALU (no matrix cores: nothing here is a float
// contraction).  Moduli below 2^41 may use the exact FP64 products of
// modarith.h; the others use 64-bit integers:
//   - fixed-operand products (twiddles, constants): Shoup's method with a
//     precomputed companion w' = floor(w 2^64 / q);
//   - variable products: Montgomery reduction (REDC) of the 128-bit product;
//   - arbitrary 64-bit words: Barrett with floor(2^64 / q).
// Data layout: contiguous limbs of N words, limb-major; a ModMap gives the
// chain index of each limb (see ckks_internal.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ckks_internal.h"
#include "modarith.h"

namespace gck {

// ---------------------------------------------------------------- launch timing

hipEvent_t KTimer::take() {
    if (!spare.empty()) {
        hipEvent_t e = spare.back();
        spare.pop_back();
        return e;
    }
    hipEvent_t e;
    GCK_HIP(hipEventCreate(&e));
    return e;
}

int KTimer::id_of(const char *name) {
    auto it = ids.find(name);
    if (it != ids.end()) return it->second;
    const int id = (int)names.size();
    ids[name] = id;
    names.push_back(name);
    stats.emplace_back();
    return id;
}

int KTimer::begin(const char *name, double bytes, double flops, hipStream_t st, double pass_bytes) {
    if (!only.empty() && only != name) return -1;
    const int id = id_of(name);
    (void)st;
    recs.push_back(Rec{id, take(), take(), bytes, flops, pass_bytes < 0 ? bytes : pass_bytes, false});
    tl_timed_launch = &recs.back();   // the next launch on this thread fills its events
    return (int)recs.size() - 1;
}

void KTimer::end(int idx, hipStream_t) {
    tl_timed_launch = nullptr;
    if (!recs[idx].launched && idx == (int)recs.size() - 1) {   // nothing was launched in the scope
        spare.push_back(recs[idx].a);
        spare.push_back(recs[idx].b);
        recs.pop_back();
    }
}

int KTimer::region_begin(const char *name, double bytes, hipStream_t st) {
    if (only != name) return -1;
    const int id = id_of(name);
    recs.push_back(Rec{id, take(), take(), bytes, 0.0, bytes, true});
    GCK_HIP(hipEventRecord(recs.back().a, st));
    return (int)recs.size() - 1;
}

void KTimer::region_end(int idx, hipStream_t st) { GCK_HIP(hipEventRecord(recs[idx].b, st)); }

thread_local KTimer::Rec *tl_timed_launch = nullptr;

void KTimer::collect() {
    for (auto &r : recs) {
        GCK_HIP(hipEventSynchronize(r.b));
        float ms = 0;
        GCK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        Stat &s = stats[r.id];
        ++s.count;
        s.ms += ms;
        s.bytes += r.bytes;
        s.flops += r.flops;
        s.pass_bytes += r.pass_bytes;
        spare.push_back(r.a);
        spare.push_back(r.b);
    }
    recs.clear();
}

void KTimer::reset() {
    collect();
    for (auto &s : stats) s = Stat{};
}

KTimer::~KTimer() {
    for (auto &r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : spare) (void)hipEventDestroy(e);
}


// ---------------------------------------------------------------- elementwise

constexpr int kEwThreads = 256;

static dim3 ew_grid(size_t total) {
    size_t blocks = (total + kEwThreads - 1) / kEwThreads;
    if (blocks > 65536 * 8) blocks = 65536 * 8;
    return dim3((unsigned)blocks);
}

template <int OP>
__global__ void ew_binary(u64 *out, const u64 *a, const u64 *b, size_t total, int log_n, ModMap mm,
                          const ModInfo *mods, int na, int nb) {
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);
        size_t k = idx & (n - 1);
        const ModInfo &M = mods[chain_of(lam, mm)];
        u64 x = a[(size_t)(lam % na) * n + k], y = b[(size_t)(lam % nb) * n + k];
        u64 r;
        if (OP == 0) r = add_mod(x, y, M.q);
        else if (OP == 1) r = sub_mod(x, y, M.q);
        else r = mul_mod(x, y, M);
        out[idx] = r;
    }
}

void k_add(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st) {
    TScope ts_(t, "ew_binary<0>", 24.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_binary<0>, ew_grid(total), dim3(kEwThreads), 0, st, out, a, b, total, t.log_n, m, t.mods, na, nb);
    check_launch();
}
void k_sub(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st) {
    TScope ts_(t, "ew_binary<1>", 24.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_binary<1>, ew_grid(total), dim3(kEwThreads), 0, st, out, a, b, total, t.log_n, m, t.mods, na, nb);
    check_launch();
}
void k_mul(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st) {
    TScope ts_(t, "ew_binary<2>", 24.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_binary<2>, ew_grid(total), dim3(kEwThreads), 0, st, out, a, b, total, t.log_n, m, t.mods, na, nb);
    check_launch();
}

__global__ void ew_mul_const(u64 *out, const u64 *a, size_t total, int log_n, ModMap mm, const ModInfo *mods,
                             ChainConst c) {
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);
        int ch = chain_of(lam, mm);
        out[idx] = mul_shoup(a[idx], c.v[ch], c.sh[ch], mods[ch].q);
    }
}
void k_mul_const(const DevTables &t, u64 *out, const u64 *a, int n_limbs, ModMap m, const ChainConst &c,
                 hipStream_t st) {
    TScope ts_(t, "ew_mul_const", 16.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_mul_const, ew_grid(total), dim3(kEwThreads), 0, st, out, a, total, t.log_n, m, t.mods, c);
    check_launch();
}

// a constant polynomial c evaluates to c at every NTT point: out = a + (c, 0), every word written once
__global__ void ew_add_const_c0(u64 *out, const u64 *a, size_t total, int log_n, int l, const ModInfo *mods,
                                ChainConst c) {
    // total = count * 2 * l * N words
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int lam = (int)(idx >> log_n);   // over count * 2 * l
        const int row = lam % (2 * l);
        out[idx] = row < l ? add_mod(a[idx], c.v[row], mods[row].q) : a[idx];
    }
}
void k_add_const_c0(const DevTables &t, u64 *out, const u64 *a, int count, int l, const ChainConst &c, hipStream_t st) {
    TScope ts_(t, "ew_add_const_c0", 16.0 * (double)((size_t)count * 2 * l) * t.n, st);
    size_t total = ((size_t)count * 2 * l) << t.log_n;
    if (!total) return;
    gck_launch(ew_add_const_c0, ew_grid(total), dim3(kEwThreads), 0, st, out, a, total, t.log_n, l, t.mods, c);
    check_launch();
}

__global__ void ew_tensor(u64 *out, const u64 *a, const u64 *b, size_t total, int log_n, int l, const ModInfo *mods,
                          int na, int nb, int accumulate) {
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);       // over count * l
        int ci = lam / l, i = lam % l;
        size_t k = idx & (n - 1);
        const ModInfo &M = mods[i];
        const u64 *pa = a + (size_t)(ci % na) * 2 * l * n, *pb = b + (size_t)(ci % nb) * 2 * l * n;
        u64 a0 = pa[(size_t)i * n + k], a1 = pa[(size_t)(l + i) * n + k];
        u64 b0 = pb[(size_t)i * n + k], b1 = pb[(size_t)(l + i) * n + k];
        if (M.fp) {
            // moduli below 2^41: exact FP64 products (see ew_tensor_sum), made canonical once
            const FMod fm{M.qd, M.qinv};
            const double x0 = u2d(a0), x1 = u2d(a1), y0 = u2d(b0), y1 = u2d(b1);
            double f0 = fmul_mod(x0, y0, fm), f1 = fmul_mod(x0, y1, fm) + fmul_mod(x1, y0, fm), f2 = fmul_mod(x1, y1, fm);
            u64 *po = out + (size_t)ci * 3 * l * n;
            size_t o0 = (size_t)i * n + k, o1 = (size_t)(l + i) * n + k, o2 = (size_t)(2 * l + i) * n + k;
            if (accumulate) {
                f0 += u2d(po[o0]);
                f1 += u2d(po[o1]);
                f2 += u2d(po[o2]);
            }
            po[o0] = fcanon(f0, fm);
            po[o1] = fcanon(f1, fm);
            po[o2] = fcanon(f2, fm);
            continue;
        }
        u64 d0 = mul_mod(a0, b0, M);
        // a0 b1 + a1 b0 as one 128-bit sum (< 2 q^2 < q 2^64), one reduction
        u64 lo1 = a0 * b1, hi1 = __umul64hi(a0, b1);
        u64 lo2 = a1 * b0, hi2 = __umul64hi(a1, b0);
        u64 lo = lo1 + lo2, hi = hi1 + hi2 + (lo < lo1 ? 1 : 0);
        if (hi >= M.q) hi -= M.q;
        u64 d1 = mul_shoup(redc(hi, lo, M), M.r_mod, M.r_mod_sh, M.q);
        u64 d2 = mul_mod(a1, b1, M);
        u64 *po = out + (size_t)ci * 3 * l * n;
        size_t o0 = (size_t)i * n + k, o1 = (size_t)(l + i) * n + k, o2 = (size_t)(2 * l + i) * n + k;
        if (accumulate) {
            po[o0] = add_mod(po[o0], d0, M.q);
            po[o1] = add_mod(po[o1], d1, M.q);
            po[o2] = add_mod(po[o2], d2, M.q);
        } else {
            po[o0] = d0; po[o1] = d1; po[o2] = d2;
        }
    }
}
void k_tensor(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int count, int l, int na, int nb,
              bool accumulate, hipStream_t st) {
    TScope ts_(t, "ew_tensor", 8.0 * 7.0 * (double)((size_t)count * l) * t.n, st);
    size_t total = ((size_t)count * l) << t.log_n;
    if (!total) return;
    gck_launch(ew_tensor, ew_grid(total), dim3(kEwThreads), 0, st, out, a, b, total, t.log_n, l, t.mods, na, nb,
                       accumulate ? 1 : 0);
    check_launch();
}

// sum over the pairs of ew_tensor's products, each as ew_tensor computes it, summed modulo q and stored once
__global__ void ew_tensor_sum(u64 *out, TensorPairs tp, size_t total, int log_n, int l, const ModInfo *mods,
                              int accumulate) {
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);       // over count * l
        int ci = lam / l, i = lam % l;
        size_t k = idx & (n - 1);
        const ModInfo &M = mods[i];
        u64 *po = out + (size_t)ci * 3 * l * n;
        size_t o0 = (size_t)i * n + k, o1 = (size_t)(l + i) * n + k, o2 = (size_t)(2 * l + i) * n + k;
        if (M.fp) {
            // moduli below 2^41: exact FP64 products, each in (-1.1 q, 1.1 q); the sums over at most 8
            // pairs (and the accumulated word) stay below 2^46, exact, and are made canonical once
            const FMod fm{M.qd, M.qinv};
            double f0 = 0.0, f1 = 0.0, f2 = 0.0;
            for (int p = 0; p < tp.n; ++p) {
                const u64 *pa = tp.a[p] + (size_t)(ci % tp.na[p]) * 2 * l * n, *pb = tp.b[p] + (size_t)(ci % tp.nb[p]) * 2 * l * n;
                const double a0 = u2d(pa[(size_t)i * n + k]), a1 = u2d(pa[(size_t)(l + i) * n + k]);
                const double b0 = u2d(pb[(size_t)i * n + k]), b1 = u2d(pb[(size_t)(l + i) * n + k]);
                f0 += fmul_mod(a0, b0, fm);
                f1 += fmul_mod(a0, b1, fm) + fmul_mod(a1, b0, fm);
                f2 += fmul_mod(a1, b1, fm);
            }
            if (accumulate) {
                f0 += u2d(po[o0]);
                f1 += u2d(po[o1]);
                f2 += u2d(po[o2]);
            }
            po[o0] = fcanon(f0, fm);
            po[o1] = fcanon(f1, fm);
            po[o2] = fcanon(f2, fm);
            continue;
        }
        u64 s0 = 0, s1 = 0, s2 = 0;
        for (int p = 0; p < tp.n; ++p) {
            const u64 *pa = tp.a[p] + (size_t)(ci % tp.na[p]) * 2 * l * n, *pb = tp.b[p] + (size_t)(ci % tp.nb[p]) * 2 * l * n;
            u64 a0 = pa[(size_t)i * n + k], a1 = pa[(size_t)(l + i) * n + k];
            u64 b0 = pb[(size_t)i * n + k], b1 = pb[(size_t)(l + i) * n + k];
            u64 d0 = mul_mod(a0, b0, M);
            u64 lo1 = a0 * b1, hi1 = __umul64hi(a0, b1);
            u64 lo2 = a1 * b0, hi2 = __umul64hi(a1, b0);
            u64 lo = lo1 + lo2, hi = hi1 + hi2 + (lo < lo1 ? 1 : 0);
            if (hi >= M.q) hi -= M.q;
            u64 d1 = mul_shoup(redc(hi, lo, M), M.r_mod, M.r_mod_sh, M.q);
            u64 d2 = mul_mod(a1, b1, M);
            s0 = add_mod(s0, d0, M.q);
            s1 = add_mod(s1, d1, M.q);
            s2 = add_mod(s2, d2, M.q);
        }
        if (accumulate) {
            s0 = add_mod(po[o0], s0, M.q);
            s1 = add_mod(po[o1], s1, M.q);
            s2 = add_mod(po[o2], s2, M.q);
        }
        po[o0] = s0; po[o1] = s1; po[o2] = s2;
    }
}

void k_tensor_sum(const DevTables &t, u64 *out, const TensorPairs &tp, int count, int l, bool accumulate, hipStream_t st) {
    TScope ts_(t, "ew_tensor_sum", 8.0 * (4.0 * tp.n + 3.0) * (double)((size_t)count * l) * t.n, st);
    size_t total = ((size_t)count * l) << t.log_n;
    if (!total || tp.n < 1) return;
    if (tp.n > kMaxTensorPairs) throw Error(CKKS_E_INVALID_ARG, "too many pairs in one tensor sum");
    gck_launch(ew_tensor_sum, ew_grid(total), dim3(kEwThreads), 0, st, out, tp, total, t.log_n, l, t.mods,
               accumulate ? 1 : 0);
    check_launch();
}

__global__ void ew_add_scaled_last(u64 *acc, const u64 *add, size_t total, int log_n, int nt, int l, u64 pm,
                                   u64 pm_sh, u64 q) {
    const size_t nw = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx >> log_n, k = idx & (nw - 1);
        u64 *a = acc + (row * nt + l - 1) * nw + k;
        const u64 dv = add[((row >> 1) * 3 * l + (row & 1) * l + l - 1) * nw + k];
        *a = add_mod(*a, mul_shoup(dv, pm, pm_sh, q), q);
    }
}
void k_add_scaled_last(const DevTables &t, u64 *acc, const u64 *add, int count, int nt, int l, u64 pm, u64 pm_sh,
                       u64 q, hipStream_t st) {
    TScope ts_(t, "ew_add_scaled_last", 24.0 * (double)count * 2 * t.n, st);
    const size_t total = (size_t)count * 2 << t.log_n;
    if (!total) return;
    gck_launch(ew_add_scaled_last, ew_grid(total), dim3(kEwThreads), 0, st, acc, add, total, t.log_n, nt, l, pm,
               pm_sh, q);
    check_launch();
}

// CP-REP product sum of the M-materialised layout: for every batch b of the chunk,
//   d_b = sum_{i < n} a_i (x) b_{b, i}   (tensor: d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1, mod q)
// with a = the n duplicated columns of M ([n][2][l][N]) and b the REP rows ([cnt][n][2][l][N]); out is
// [cnt][3][l][N].  A thread owns one word of one limb for kRepCB batches, so each column word is read once
// per kRepCB batches; the sums are kept reduced (one modular addition per product).
constexpr int kRepCB = 4;
__global__ void ew_tensor_rep_sum(u64 *out, const u64 *a, const u64 *b, int cnt, int n_rows, int l, int log_n,
                                  const ModInfo *mods) {
    const size_t nw = (size_t)1 << log_n;
    const int groups = (cnt + kRepCB - 1) / kRepCB;
    const size_t total = (size_t)groups * l * nw;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t k = idx & (nw - 1);
        const int lam = (int)((idx >> log_n) % l);
        const int g0 = (int)((idx >> log_n) / l) * kRepCB;
        const ModInfo &M = mods[lam];
        u64 d0[kRepCB], d1[kRepCB], d2[kRepCB];
        for (int c = 0; c < kRepCB; ++c) d0[c] = d1[c] = d2[c] = 0;
        const size_t per = (size_t)2 * l * nw;
        for (int i = 0; i < n_rows; ++i) {
            const u64 *pa = a + (size_t)i * per;
            const u64 a0 = pa[(size_t)lam * nw + k], a1 = pa[(size_t)(l + lam) * nw + k];
            for (int c = 0; c < kRepCB; ++c) {
                if (g0 + c >= cnt) break;
                const u64 *pb = b + ((size_t)(g0 + c) * n_rows + i) * per;
                const u64 b0 = pb[(size_t)lam * nw + k], b1 = pb[(size_t)(l + lam) * nw + k];
                d0[c] = add_mod(d0[c], mul_mod(a0, b0, M), M.q);
                u64 lo1 = a0 * b1, hi1 = __umul64hi(a0, b1);
                u64 lo2 = a1 * b0, hi2 = __umul64hi(a1, b0);
                u64 lo = lo1 + lo2, hi = hi1 + hi2 + (lo < lo1 ? 1 : 0);
                if (hi >= M.q) hi -= M.q;
                d1[c] = add_mod(d1[c], mul_shoup(redc(hi, lo, M), M.r_mod, M.r_mod_sh, M.q), M.q);
                d2[c] = add_mod(d2[c], mul_mod(a1, b1, M), M.q);
            }
        }
        for (int c = 0; c < kRepCB; ++c) {
            if (g0 + c >= cnt) break;
            u64 *po = out + (size_t)(g0 + c) * 3 * l * nw;
            po[(size_t)lam * nw + k] = d0[c];
            po[(size_t)(l + lam) * nw + k] = d1[c];
            po[(size_t)(2 * l + lam) * nw + k] = d2[c];
        }
    }
}
void k_tensor_rep_sum(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int cnt, int n_rows, int l,
                      hipStream_t st) {
    // algorithmic bytes: the columns once per kRepCB batches, the REP rows once, the tensor written once
    const double groups = (double)((cnt + kRepCB - 1) / kRepCB);
    TScope ts_(t, "ew_tensor_rep_sum",
               8.0 * (double)t.n * l * (groups * 2.0 * n_rows + (double)cnt * (2.0 * n_rows + 3.0)), st);
    const size_t total = (size_t)((cnt + kRepCB - 1) / kRepCB) * l << t.log_n;
    if (!total) return;
    gck_launch(ew_tensor_rep_sum, ew_grid(total), dim3(kEwThreads), 0, st, out, a, b, cnt, n_rows, l, t.log_n, t.mods);
    check_launch();
}

// c0 of ciphertext i of the batch plus the plaintext pt ([l][N], NTT form) moved by the automorphism of a
// right rotation by i mod R (Galois element 5^-i mod 2N): pt the block-start mask, this adds the exact
// indicator of the slots = i mod R (the identity column i of M, duplicated).  c1 is copied.
__global__ void ew_add_rotated_plain(u64 *out, const u64 *a, const u64 *pt, int count, int l, int log_n, int R,
                                     const ModInfo *mods) {
    const size_t nw = (size_t)1 << log_n;
    const size_t total = (size_t)count * 2 * l * nw;
    const unsigned two_n = 2u << log_n, half = 1u << (log_n - 1);
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx >> log_n;          // over count * 2 * l
        const int ci = (int)(row / (2 * l)), pl = (int)(row % (2 * l));
        u64 v = a[idx];
        if (pl < l) {
            // 5^e mod 2N with e = -(i mod R) mod N/2 (5 has order N/2 modulo 2N)
            unsigned e = (half - (unsigned)(ci % R)) % half, g = 1, base = 5;
            while (e) {
                if (e & 1) g = (unsigned)(((unsigned long long)g * base) % two_n);
                base = (unsigned)(((unsigned long long)base * base) % two_n);
                e >>= 1;
            }
            const u64 w = pt[(size_t)pl * nw + automorph_src(idx & (nw - 1), log_n, g)];
            v = add_mod(v, w, mods[pl].q);
        }
        out[idx] = v;
    }
}
void k_add_rotated_plain(const DevTables &t, u64 *out, const u64 *a, const u64 *pt, int count, int l, int R,
                         hipStream_t st) {
    TScope ts_(t, "ew_add_rotated_plain", 8.0 * (double)t.n * (4.0 * count * l + l), st);
    const size_t total = (size_t)count * 2 * l << t.log_n;
    if (!total) return;
    gck_launch(ew_add_rotated_plain, ew_grid(total), dim3(kEwThreads), 0, st, out, a, pt, count, l, t.log_n, R,
               t.mods);
    check_launch();
}

__global__ void ew_automorph(u64 *out, const u64 *a, size_t total, int log_n, u64 g) {
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        size_t lam = idx >> log_n;
        out[idx] = a[lam * n + automorph_src(idx & (n - 1), log_n, g)];
    }
}
void k_automorph(const DevTables &t, u64 *out, const u64 *a, int n_limbs, u64 g, hipStream_t st) {
    TScope ts_(t, "ew_automorph", 16.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_automorph, ew_grid(total), dim3(kEwThreads), 0, st, out, a, total, t.log_n, g);
    check_launch();
}

__global__ void ew_copy_rows(u64 *out, size_t out_stride, const u64 *in, size_t in_stride, size_t total, size_t words) {
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        size_t r = idx / words, k = idx % words;
        out[r * out_stride + k] = in[r * in_stride + k];
    }
}
void k_copy_rows(u64 *out, size_t out_stride, const u64 *in, size_t in_stride, int rows, size_t words,
                 hipStream_t st) {
    size_t total = (size_t)rows * words;
    if (!total) return;
    gck_launch(ew_copy_rows, ew_grid(total), dim3(kEwThreads), 0, st, out, out_stride, in, in_stride, total, words);
    check_launch();
}

__device__ __forceinline__ size_t gather_limb(const Gather &g, int lam) {
    return (size_t)((lam / g.div) * g.mul + g.add + (lam % g.div) * g.inner);
}
// ---------------------------------------------------------------- key-switch inner product
//
// acc[c][comp][t][k] = sum_i sum_b sigma_i(D_b[c][t])[k] * key_i[comp][b][chain(t)][k] mod the target's
// modulus, over the targets t < l + alpha (q_0..q_{l-1}, then the special primes).  The key words
// carry a factor 2^64 (Montgomery form).  One thread per (group of CB ciphertexts, target t, word k);
// consecutive 256-thread blocks hold the groups of one (t, 256-word chunk), so the key words a chunk
// needs are fetched from HBM once and re-read from cache by the other groups.  Targets below 2^41
// accumulate in FP64 (exact products, signed remainders; the factor 2^64 removed by a multiply with
// 2^-64 mod q), the others in 128-bit integers with the high word kept below q and one REDC.
// Accumulators of one target word for CB ciphertexts: FP64 signed remainders (moduli below 2^41) or
// 128-bit integer sums with the high word kept below q.
template <int CB, bool FP>
struct KsAcc;
template <int CB>
struct KsAcc<CB, true> {
    double a0[CB], a1[CB];
    __device__ void zero() {
#pragma unroll
        for (int b = 0; b < CB; ++b) a0[b] = a1[b] = 0.0;
    }
    __device__ void mac(int b, u64 d, u64 k0, u64 k1, const ModInfo &M, const FMod &fm) {
        const double dd = u2d(d);   // a residue of this target (below 2^41)
        a0[b] += fmul_mod(dd, u2d(k0), fm);
        a1[b] += fmul_mod(dd, u2d(k1), fm);
    }
    __device__ void settle(const FMod &fm) {   // each term is below 0.6 q: reduce the sums to below 0.6 q
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            a0[b] = fred(a0[b], fm);
            a1[b] = fred(a1[b], fm);
        }
    }
    __device__ void store(int b, u64 *o, size_t comp_stride, const ModInfo &M, const FMod &fm) {
        o[0] = fcanon(fmul_mod(a0[b], M.rinv_d, fm), fm);
        o[comp_stride] = fcanon(fmul_mod(a1[b], M.rinv_d, fm), fm);
    }
};
template <int CB>
struct KsAcc<CB, false> {
    u64 h0[CB], l0[CB], h1[CB], l1[CB];
    __device__ void zero() {
#pragma unroll
        for (int b = 0; b < CB; ++b) h0[b] = l0[b] = h1[b] = l1[b] = 0;
    }
    __device__ void mac(int b, u64 d, u64 k0, u64 k1, const ModInfo &M, const FMod &) {
        const u64 p0 = d * k0, q0 = __umul64hi(d, k0);
        const u64 p1 = d * k1, q1 = __umul64hi(d, k1);
        l0[b] += p0;
        h0[b] += q0 + (l0[b] < p0 ? 1 : 0);
        l1[b] += p1;
        h1[b] += q1 + (l1[b] < p1 ? 1 : 0);
        if (h0[b] >= M.q) h0[b] -= M.q;
        if (h1[b] >= M.q) h1[b] -= M.q;
    }
    __device__ void settle(const FMod &) {}
    __device__ void store(int b, u64 *o, size_t comp_stride, const ModInfo &M, const FMod &) {
        o[0] = redc(h0[b], l0[b], M);
        o[comp_stride] = redc(h1[b], l1[b], M);
    }
};

// Loads through the global address space.  A pointer chosen at run time between a kernel argument and a
// pointer read from an argument struct is generic to the compiler, and a generic load is a FLAT access,
// which counts on the LDS counter as well: the wait before the first product of a unit then has to drain
// every load in flight, including the next unit's prefetch.  All buffers here are device memory.
typedef __attribute__((address_space(1))) const u64 gu64;
typedef __attribute__((address_space(1))) const char gchar;
__device__ __forceinline__ u64 ld_g(const u64 *p) { return *(gu64 *)p; }

// word at a 32-bit byte offset from a wave-uniform base: the empty asm statement keeps the optimizer from
// widening the offset to 64 bits, so the load takes the base from scalar registers and the offset from one
// vector register (no 64-bit address arithmetic per lane)
__device__ __forceinline__ u64 ld_off(const u64 *base, unsigned byte_off) {
    asm("" : "+v"(byte_off));
    return *(gu64 *)((gchar *)base + byte_off);
}

// one target word for CB ciphertexts.  MK > 0: exactly MK keys, their loads for one digit group issued
// together (unrolled); MK < 0: keys.m keys in chunks of -MK (the last chunk padded with zero words), the
// loads of one (digit group, chunk) unit issued together; MK == 0: keys.m keys in a loop.  FULL: (MK < 0)
// keys.m a multiple of the chunk, and absent ciphertexts (b >= nb) repeat the last present one (computed,
// not stored), so that no load or product is guarded.
template <int CB, int MK, bool FP, bool FULL>
__device__ __forceinline__ void ks_word(u64 *acc, const u64 *digits, int K, const int *__restrict__ didx,
                                        const u64 *const (&own_row)[CB], const KsKeys &keys, const size_t (&kd)[MK > 0 ? MK : 1],
                                        int gl, int nt, int tt, size_t k, size_t krow, size_t key_grp, size_t key_comp,
                                        int log_n, size_t n, int c0, int nb, const ModInfo &M) {
    const FMod fm{M.qd, M.qinv};
    KsAcc<CB, FP> A;
    A.zero();
    // FP64 sums are reduced every kSettleUnits units (at most 3 terms each, every term below 0.6 q): they stay
    // below 15 q < 2^45, exact, and the final multiply by R^-1 takes them (below 2^47)
    constexpr int kSettleUnits = 8;
    int pend = 0;
    if constexpr (MK < 0) {
        // units u = (digit group gb, key chunk kc), gb-major; the loads of unit u + 1 are issued before the
        // products of unit u (double buffer).  A padded key contributes 0 x 0.
        constexpr int KC = -MK;
        const int m = keys.m, nkc = (m + KC - 1) / KC, nu = gl * nkc;
        u64 kw0[2][KC], kw1[2][KC], dw[2][KC][CB];
        // digit rows of the thread's ciphertexts (digit index e adds e N), and the unit the next load takes,
        // advanced by one per load (no division per unit); past the last unit a load repeats it
        const u64 *dbase[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) dbase[b] = digits + (size_t)(c0 + (FULL && b >= nb ? nb - 1 : b)) * K * n;
        int cur_gb = 0, cur_kc = 0;
        auto load = [&](int s) {
            const bool past = cur_gb >= gl;
            const int gb = past ? gl - 1 : cur_gb, kc = past ? nkc - 1 : cur_kc;
            if (++cur_kc == nkc) {
                cur_kc = 0;
                ++cur_gb;
            }
            const int e = didx[gb * nt + tt];
#pragma unroll
            for (int i = 0; i < KC; ++i) {
                const int ki = kc * KC + i;
                const bool on = FULL || ki < m;
                const u64 *key = keys.key[on ? ki : 0] + (size_t)gb * key_grp + (krow - k);   // wave-uniform
                const u64 g = on ? keys.g[ki] : 0;
                const unsigned kdb = (unsigned)(g ? automorph_src(k, log_n, g) : k) << 3;
                const unsigned kb = (unsigned)k << 3;
                kw0[s][i] = on ? ld_off(key, kb) : 0;
                kw1[s][i] = on ? ld_off(key + key_comp, kb) : 0;
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const int bb = FULL && b >= nb ? nb - 1 : b;
                    const u64 *src = e >= 0 ? dbase[b] + ((size_t)e << log_n) : own_row[bb];
                    dw[s][i][b] = (on && (FULL || b < nb)) ? ld_off(src, kdb) : 0;
                }
            }
        };
        // FULL: the prefetch is unconditional (past the end it re-reads the last unit), so that the wait
        // before a unit's products counts only the loads issued before the other buffer's, and an empty asm
        // statement that clobbers memory keeps the compiler from sinking it down to its own products (the
        // guarded form measures faster with the fence and the clamp left out)
        load(0);
        for (int u = 0; u < nu; u += 2) {
            if constexpr (FULL) {
                load(1);
                asm volatile("" ::: "memory");
            } else if (u + 1 < nu) {
                load(1);
            }
#pragma unroll
            for (int i = 0; i < KC; ++i)
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (FULL || b < nb) A.mac(b, dw[0][i][b], kw0[0][i], kw1[0][i], M, fm);
            if (++pend == kSettleUnits) {
                A.settle(fm);
                pend = 0;
            }
            if (u + 1 >= nu) break;
            if constexpr (FULL) {
                load(0);
                asm volatile("" ::: "memory");
            } else if (u + 2 < nu) {
                load(0);
            }
#pragma unroll
            for (int i = 0; i < KC; ++i)
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (FULL || b < nb) A.mac(b, dw[1][i][b], kw0[1][i], kw1[1][i], M, fm);
            if (++pend == kSettleUnits) {
                A.settle(fm);
                pend = 0;
            }
        }
    } else if constexpr (MK > 0) {
        // the loads of digit group gb + 1 are issued before the products of group gb (double buffer)
        u64 kw0[2][MK], kw1[2][MK], dw[2][MK][CB];
        auto load = [&](int gb, int s) {
            const int e = didx[gb * nt + tt];
#pragma unroll
            for (int i = 0; i < MK; ++i) {
                kw0[s][i] = keys.key[i][(size_t)gb * key_grp + krow];
                kw1[s][i] = keys.key[i][key_comp + (size_t)gb * key_grp + krow];
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const int bb = FULL && b >= nb ? nb - 1 : b;
                    const u64 *src = e >= 0 ? digits + ((size_t)(c0 + bb) * K + e) * n : own_row[bb];
                    dw[s][i][b] = (FULL || b < nb) ? ld_g(src + kd[i]) : 0;
                }
            }
        };
        load(0, 0);
        for (int gb = 0; gb < gl; gb += 2) {
            if (gb + 1 < gl) load(gb + 1, 1);
#pragma unroll
            for (int i = 0; i < MK; ++i)
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (FULL || b < nb) A.mac(b, dw[0][i][b], kw0[0][i], kw1[0][i], M, fm);
            if (++pend == kSettleUnits) {
                A.settle(fm);
                pend = 0;
            }
            if (gb + 1 >= gl) break;
            if (gb + 2 < gl) load(gb + 2, 0);
#pragma unroll
            for (int i = 0; i < MK; ++i)
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (FULL || b < nb) A.mac(b, dw[1][i][b], kw0[1][i], kw1[1][i], M, fm);
            if (++pend == kSettleUnits) {
                A.settle(fm);
                pend = 0;
            }
        }
    } else {
        for (int gb = 0; gb < gl; ++gb) {
            const int e = didx[gb * nt + tt];
            const u64 *src[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int bb = FULL && b >= nb ? nb - 1 : b;
                src[b] = e >= 0 ? digits + ((size_t)(c0 + bb) * K + e) * n : own_row[bb];
            }
            for (int i = 0; i < keys.m; ++i) {
                const size_t kdi = keys.g[i] ? automorph_src(k, log_n, keys.g[i]) : k;
                const u64 k0 = keys.key[i][(size_t)gb * key_grp + krow];
                const u64 k1 = keys.key[i][key_comp + (size_t)gb * key_grp + krow];
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (FULL || b < nb) A.mac(b, ld_g(src[b] + kdi), k0, k1, M, fm);
            }
            A.settle(fm);
        }
    }
#pragma unroll
    for (int b = 0; b < CB; ++b)
        if (b < nb) A.store(b, acc + ((size_t)(c0 + b) * 2 * nt + tt) * n + k, (size_t)nt * n, M, fm);
}

// Rotation lines of the NTT domain.  The words of an aligned group of 64 share the low log_n - 5 bits of
// their evaluation exponent e = 2 brev(k) + 1, and X -> X^g maps the group with exponent class E (odd, mod
// 2^(log_n - 5)) onto the group with class E g.  Every odd class is +-5^t for one sign and one
// t < T = N / 128, and a rotation by r slots (g = 5^r) moves t to t + r: the key words of output group
// (sign, t) pair with the digit groups (sign, t + r_i).  When every r_i is a multiple of s, the groups
// (sign, v + s u), u < T / s, form a line that the key switch never leaves.  KsLines hands each XCD whole
// lines (or, for s < 4, one of P contiguous segments of a line) walked in order of u, so that the digit
// groups read through the automorphisms of nearby output groups are the same and stay in the XCD's L2.
struct KsLines {
    int s = 0;        // shift unit (0: the position-range mapping)
    int P = 1;        // segments per line
    int seglen = 0;   // groups per segment
    int spx = 0;      // segments per XCD
};

// Doubling form of a rotate-and-sum group's automorphism sum (aut_sum_dbl)
struct AutDbl {
    int log_m;   // m = 2^log_m terms: the word itself and m - 1 rotations
    int step;    // group-exponent shift of one rotation (s mod T, a power of 2; 0: within each group)
    int dir;     // +1 or -1: the sign of the rotations
    int U;       // groups per line
    int W;       // output groups per workgroup (W divides U)
    int nb;      // groups in LDS: W + m - 1, or U when the window is the whole line
    int cyc;     // 1: the window is the whole line (indices modulo U)
    int lines;   // 2 signs x step lines, or 2 T single-group lines when step == 0
    u64 gp[4];   // Galois elements of sigma^(2^j), j < log_m
};

// group index (word index >> 6) of the class (sign, t): E = +-5^t mod 2^(log_n - 5), G = brev((E - 1) / 2)
__device__ __forceinline__ unsigned rot_group(int sign, unsigned t, int log_n) {
    const unsigned mask = (1u << (log_n - 5)) - 1;
    unsigned e = 1, p = 5;
    for (unsigned x = t; x; x >>= 1) {
        if (x & 1) e = (e * p) & mask;
        p = (p * p) & mask;
    }
    if (sign) e = (0u - e) & mask;
    return __brev((e - 1) >> 1) >> (32 - (log_n - 6));
}

template <int CB, int MK, bool FULL>
__global__ void __launch_bounds__(kEwThreads, 3) ks_inner(u64 *acc, const u64 *digits, int K, const int *__restrict__ didx, Gather own, KsKeys keys,
                         int ng, size_t total, int log_n, int l, int levels, int alpha, int c_first, int count,
                         const ModInfo *mods, KsLines ln) {
    const size_t n = (size_t)1 << log_n;
    const int nt = l + alpha;                 // targets of this key switch
    const int nt_key = levels + 1 + alpha;    // targets of a key
    const size_t key_comp = (size_t)ng * nt_key * n;
    const size_t key_grp = (size_t)nt_key * n;
    const int gl = ks_groups(l, alpha);
    const int groups = (count + CB - 1) / CB;
    const size_t chunks = n >> 8;   // 256-word chunks per limb
    // Work item: (target, 256-word chunk, group of CB ciphertexts).  Workgroup b runs on XCD b mod 8; XCD x
    // takes the chunks [x p8, (x + 1) p8) of every target, and consecutive workgroups of an XCD (which run
    // together) take the ciphertext groups of one chunk: they share its key words in the XCD's L2.
    // gridDim.x is a multiple of 8 and `total` counts 8 p8 nt groups items.
    const int p8 = chunks >= 8 ? (int)(chunks >> 3) : 1;
    const int x = (int)(blockIdx.x & 7);
    const int pos0 = x * p8;
    const int npos = pos0 >= (int)chunks ? 0 : ((int)chunks - pos0 < p8 ? (int)chunks - pos0 : p8);
    // line mapping: 64-thread workgroups, one group of 64 words each; the slot of a workgroup on its XCD
    // runs over (ciphertext group, position u along the segment, target, segment), fastest first
    const size_t items_x = ln.s ? (size_t)ln.spx * ln.seglen * nt * groups : (size_t)npos * nt * groups;
    for (size_t b = blockIdx.x; b < total; b += gridDim.x) {
        const size_t sl = b >> 3;                          // slot of this workgroup on its XCD
        if (sl >= items_x) break;
        const int grp = (int)(sl % groups);
        size_t rest = sl / groups;
        int tt;
        size_t k;
        if (ln.s) {
            const int ui = (int)(rest % ln.seglen);
            rest /= ln.seglen;
            tt = (int)(rest % nt);
            const int seg = (int)(rest / nt) * 8 + x;
            const int line = seg / ln.P, part = seg % ln.P;
            const unsigned t = (unsigned)(line % ln.s) + (unsigned)ln.s * (unsigned)(part * ln.seglen + ui);
            k = ((size_t)rot_group(line / ln.s, t, log_n) << 6) + threadIdx.x;
        } else {
            const int pos = pos0 + (int)(rest % npos);
            tt = (int)(rest / npos);
            k = ((size_t)pos << 8) + threadIdx.x;
        }
        const int chain = tt < l ? tt : levels + 1 + (tt - l);
        const ModInfo M = mods[chain];
        const size_t krow = (size_t)chain * n + k;   // key word of group b: key[b key_grp + krow]
        const int c0 = c_first + grp * CB;   // ciphertexts [c_first, c_first + count) in this launch
        const int nb = c_first + count - c0 < CB ? c_first + count - c0 : CB;
        // the input limb tt of each ciphertext (the digit of tt's own group), when tt is a q-target
        const u64 *own_row[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int lam = (c0 + b) * l + (tt < l ? tt : 0);
            own_row[b] = own.ptr + (size_t)((lam / own.div) * own.mul + own.add + (lam % own.div) * own.inner) * n;
        }
        size_t kd[MK > 0 ? MK : 1];   // permuted digit word of each key (MK > 0)
#pragma unroll
        for (int i = 0; i < (MK > 0 ? MK : 1); ++i) kd[i] = (MK > 0 && keys.g[i]) ? automorph_src(k, log_n, keys.g[i]) : k;
        if (M.fp)
            ks_word<CB, MK, true, FULL>(acc, digits, K, didx, own_row, keys, kd, gl, nt, tt, k, krow, key_grp, key_comp,
                                        log_n, n, c0, nb, M);
        else
            ks_word<CB, MK, false, FULL>(acc, digits, K, didx, own_row, keys, kd, gl, nt, tt, k, krow, key_grp, key_comp,
                                         log_n, n, c0, nb, M);
    }
}
// The line mapping for a key set of two or more rotations (Galois elements 5^r mod 2N, or none); 0 when a
// key is not a rotation (conjugation) or the ring is too small for 8 segments.
static KsLines ks_lines(const KsKeys &keys, int log_n) {
    KsLines ln;
    if (keys.m < 2 || log_n < 9) return ln;
    const int b = log_n - 5, T = 1 << (b - 2);
    const u64 mask = (1ULL << b) - 1;
    int s = T;
    for (int i = 0; i < keys.m; ++i) {
        if (!keys.g[i]) continue;
        const u64 gb = keys.g[i] & mask;
        int r = -1;
        u64 p = 1;
        for (int j = 0; j < T; ++j, p = (p * 5) & mask)
            if (p == gb) {
                r = j;
                break;
            }
        if (r < 0) return ln;   // -5^r: not a rotation
        if (r) s = std::min(s, r & -r);
    }
    ln.s = s;
    ln.P = 2 * s >= 8 ? 1 : 8 / (2 * s);
    ln.seglen = T / s / ln.P;
    ln.spx = 2 * s * ln.P / 8;
    if (ln.seglen < 1 || ln.spx < 1) return KsLines{};
    return ln;
}

void k_ks_inner(const DevTables &t, u64 *acc, const u64 *digits, int K, const int *didx, const Gather &own,
                const KsKeys &keys, int ng, int count, int l, int levels, int alpha, hipStream_t st) {
    const int nt = l + alpha, gl = ks_groups(l, alpha);
    // algorithmic bytes: every key word and every digit word read once, the accumulators written once
    const int cb = count >= 4 ? 4 : (count >= 2 ? 2 : 1);   // 2 or 8 (fewer waves, or spills) measured slower
    // exactly 1 or 3 keys unrolled; more than 3 in chunks of 3 (a fully unrolled 15-key form spilled or ran
    // slower); 2 in the loop
    const int mk = (keys.m == 1 || keys.m == 3) ? keys.m : (keys.m > 3 ? -3 : 0);
    const int mi = mk == 0 ? 0 : (mk == 1 ? 1 : (mk == 3 ? 2 : 3));
    static const char *const names[2][3][4] = {
        {{"ks_inner<1, 0, false>", "ks_inner<1, 1, false>", "ks_inner<1, 3, false>", "ks_inner<1, -3, false>"},
         {"ks_inner<2, 0, false>", "ks_inner<2, 1, false>", "ks_inner<2, 3, false>", "ks_inner<2, -3, false>"},
         {"ks_inner<4, 0, false>", "ks_inner<4, 1, false>", "ks_inner<4, 3, false>", "ks_inner<4, -3, false>"}},
        {{"ks_inner<1, 0, true>", "ks_inner<1, 1, true>", "ks_inner<1, 3, true>", "ks_inner<1, -3, true>"},
         {"ks_inner<2, 0, true>", "ks_inner<2, 1, true>", "ks_inner<2, 3, true>", "ks_inner<2, -3, true>"},
         {"ks_inner<4, 0, true>", "ks_inner<4, 1, true>", "ks_inner<4, 3, true>", "ks_inner<4, -3, true>"}}};
    if (t.log_n < 8) throw Error(CKKS_E_INVALID_ARG, "key switching needs N >= 256");
    if (!count) return;
    const size_t chunks = (size_t)1 << (t.log_n - 8);
    const size_t p8 = chunks >= 8 ? chunks / 8 : 1;
    const KsLines ln = ks_lines(keys, t.log_n);
    // the guard-free form (a ragged last ciphertext group padded) for one key and for key counts that fill
    // their chunks of 3: 140 to 127 us and 709 to 562 us per launch at the 42-batch chunk; with exactly 3 keys
    // it spills and was not faster, so that form keeps its guards
    const bool keys_fill = mk == 1 || (mk < 0 && keys.m % 3 == 0);
    auto launch = [&](bool full, int c_first, int cnt) {
        // algorithmic FP64 operations: one multiply-accumulate per (ciphertext, FP64 target, word, digit group,
        // key), each two modular products (a product and its FMA error 3, the quotient 2, the remainder 2,
        // their sum 1) and two additions: 18.  The target q_0 (60 bits) accumulates in 128-bit integers and
        // does no FP64 work: nt - 1 targets count.
        TScope ts_(t, names[full ? 1 : 0][cb == 4 ? 2 : cb - 1][mi],
                   8.0 * (double)t.n * (keys.m * 2.0 * gl * nt * cnt / count + (double)cnt * (gl * nt + 2.0 * nt)), st,
                   18.0 * (double)cnt * (nt - 1) * (double)t.n * gl * keys.m);
        const size_t ngrp = (size_t)((cnt + cb - 1) / cb);
        const size_t total = ln.s ? 8 * (size_t)ln.spx * ln.seglen * nt * ngrp   // workgroup items
                                  : 8 * p8 * nt * ngrp;
        const dim3 grid((unsigned)(total < 65536 * 8 ? total : 65536 * 8)), block(ln.s ? 64 : kEwThreads);
#define GCK_KS(CB_, MK_)                                                                                              \
    (full ? gck_launch((ks_inner<CB_, MK_, true>), grid, block, 0, st, acc, digits, K, didx, own, keys, ng, total,     \
                       t.log_n, l, levels, alpha, c_first, cnt, t.mods, ln)                                            \
          : gck_launch((ks_inner<CB_, MK_, false>), grid, block, 0, st, acc, digits, K, didx, own, keys, ng, total,    \
                       t.log_n, l, levels, alpha, c_first, cnt, t.mods, ln))
        switch (cb * 10 + mk) {
        case 37: GCK_KS(4, -3); break;
        case 17: GCK_KS(2, -3); break;
        case 7: GCK_KS(1, -3); break;
        case 41: GCK_KS(4, 1); break;
        case 43: GCK_KS(4, 3); break;
        case 40: GCK_KS(4, 0); break;
        case 21: GCK_KS(2, 1); break;
        case 23: GCK_KS(2, 3); break;
        case 20: GCK_KS(2, 0); break;
        case 11: GCK_KS(1, 1); break;
        case 13: GCK_KS(1, 3); break;
        default: GCK_KS(1, 0); break;
        }
        check_launch();
    };
    launch(keys_fill, 0, count);
#undef GCK_KS
}

// z[c][j] = a[c][0][j] + sum_i sigma_i(a[c][0][j]) mod q_j over the keys' automorphisms (NTT domain), a
// [count][2][l][N].  A 256-thread workgroup takes 4 groups of 64 words of one limb, consecutive along a
// rotation line of the key set (KsLines), so that the permuted reads of neighbouring workgroups share the
// XCD's L2 (the word itself is among them).  Residues below 2^41 are summed as integers (at most 17 terms,
// below 2^46) and reduced once; the 60-bit q_0 adds modulo q_0 term by term.
__global__ void __launch_bounds__(256) aut_sum(u64 *z, const u64 *a, int l, KsKeys keys, int log_n, size_t total,
                                               int n_limbs, KsLines ln, const ModInfo *mods) {
    const size_t n = (size_t)1 << log_n;
    const int x = (int)(blockIdx.x & 7);
    const int groups = (int)(n >> 6), wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int steps = ln.s ? (ln.seglen + 3) / 4 : (groups + 3) / 4;   // workgroups along a segment / limb
    for (size_t b = blockIdx.x; b < total; b += gridDim.x) {
        const size_t sl = b >> 3;
        int lam, ui;
        unsigned grp;
        if (ln.s) {
            ui = (int)(sl % steps) * 4 + wave;
            const size_t rest = sl / steps;
            lam = (int)(rest % n_limbs);
            const int seg = (int)(rest / n_limbs) * 8 + x;
            if (seg >= 8 * ln.spx) break;
            if (ui >= ln.seglen) continue;
            const int line = seg / ln.P, part = seg % ln.P;
            const unsigned t = (unsigned)(line % ln.s) + (unsigned)ln.s * (unsigned)(part * ln.seglen + ui);
            grp = rot_group(line / ln.s, t, log_n);
        } else {
            const size_t item = b;   // (limb, step) in order
            if (item >= (size_t)n_limbs * steps) break;
            lam = (int)(item / steps);
            ui = (int)(item % steps) * 4 + wave;
            if (ui >= groups) continue;
            grp = (unsigned)ui;
        }
        const int c = lam / l, j = lam % l;
        const u64 *src = a + ((size_t)c * 2 * l + j) * n;
        const size_t k = ((size_t)grp << 6) + lane;
        u64 v[kMaxKeys];
#pragma unroll
        for (int i = 0; i < kMaxKeys; ++i) v[i] = i < keys.m ? src[automorph_src(k, log_n, keys.g[i])] : 0;
        const u64 self = src[k];
        const ModInfo M = mods[j];
        if (M.fp) {
            u64 sum = self;
#pragma unroll
            for (int i = 0; i < kMaxKeys; ++i) sum += v[i];
            z[(size_t)lam * n + k] = fcanon(u2d(sum), FMod{M.qd, M.qinv});
        } else {
            u64 r = self;
#pragma unroll
            for (int i = 0; i < kMaxKeys; ++i) r = add_mod(r, v[i], M.q);
            z[(size_t)lam * n + k] = r;
        }
    }
}
void k_aut_sum(const DevTables &t, u64 *z, const u64 *a, int count, int l, const KsKeys &keys, hipStream_t st) {
    const int n_limbs = count * l;
    TScope ts_(t, "aut_sum", 16.0 * (double)n_limbs * t.n, st);
    if (!n_limbs) return;
    const KsLines ln = ks_lines(keys, t.log_n);
    const size_t groups = (size_t)t.n >> 6;
    const size_t total = ln.s ? 8 * (size_t)ln.spx * ((ln.seglen + 3) / 4) * n_limbs
                              : ((size_t)n_limbs * ((groups + 3) / 4) + 7) / 8 * 8;
    const dim3 grid((unsigned)(total < 65536 * 8 ? total : 65536 * 8)), block(256);
    gck_launch(aut_sum, grid, block, 0, st, z, a, l, keys, t.log_n, total, n_limbs, ln, t.mods);
    check_launch();
}

// The same sum for the rotations of one rotate-and-sum group, d s, 2 d s, .., (m - 1) d s with m a power of
// 2: z = (1 + sigma)(1 + sigma^2)..(1 + sigma^(m/2)) c0 with sigma the rotation by d s, so log2 m doubling
// steps A <- A + sigma^p(A), each reading its partner word once, in place of m - 1 gathers per word.  A
// 256-thread workgroup loads a window of W groups of one rotation line (t = v + d s u, u along the line) and
// the m - 1 groups after it, or the whole line when it is short (indices then cyclic), into LDS, and runs
// the steps there; the partner of a word is its automorphism source under sigma^p, a word of the group p
// places further along the line.
__global__ void __launch_bounds__(256) aut_sum_dbl(u64 *z, const u64 *a, int l, int log_n, AutDbl ad, int n_limbs,
                                                   const ModInfo *mods) {
    extern __shared__ u64 buf[];                    // nb groups of 64 words
    int *gid = reinterpret_cast<int *>(buf + (size_t)ad.nb * 64);   // group index of each window slot
    const size_t n = (size_t)1 << log_n;
    const unsigned T = 1u << (log_n - 7);
    const int segs = ad.U / ad.W;
    const int item = blockIdx.x;
    const int seg = item % segs, line = (item / segs) % ad.lines, lam = item / (segs * ad.lines);
    if (lam >= n_limbs) return;
    const int per_sign = ad.lines / 2;
    const int sign = line / per_sign, v = line % per_sign;
    const int u0 = seg * ad.W;
    const int c = lam / l, j = lam % l;
    const u64 *src = a + ((size_t)c * 2 * l + j) * n;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    for (int gx = wave; gx < ad.nb; gx += 4) {
        const int u = (u0 + gx) % ad.U;
        const unsigned t = ad.step ? (unsigned)(v + ad.dir * ad.step * u) & (T - 1) : (unsigned)v;
        const unsigned g = rot_group(sign, t, log_n);
        if (lane == 0) gid[gx] = (int)g;
        buf[(size_t)gx * 64 + lane] = src[((size_t)g << 6) + lane];
    }
    __syncthreads();
    constexpr int kMaxPer = 20;   // words per thread per step: nb 64 / 256 with nb <= 79
    for (int st = 0; st < ad.log_m; ++st) {
        const int p = 1 << st;
        const int valid = ad.cyc ? ad.nb : ad.nb - (2 * p - 1);
        u64 r[kMaxPer];
#pragma unroll
        for (int e = 0; e < kMaxPer; ++e) {
            const int x = (int)threadIdx.x + e * 256;
            r[e] = 0;
            if (x < valid * 64) {
                const int gx = x >> 6, w = x & 63;
                const size_t k = ((size_t)gid[gx] << 6) + w;
                const int gp = ad.cyc ? (gx + p) % ad.nb : gx + p;
                const int wp = (int)(automorph_src(k, log_n, ad.gp[st]) & 63);
                r[e] = buf[x] + buf[(size_t)gp * 64 + wp];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kMaxPer; ++e) {
            const int x = (int)threadIdx.x + e * 256;
            if (x < valid * 64) buf[x] = r[e];
        }
        __syncthreads();
    }
    const ModInfo M = mods[j];
    for (int gx = wave; gx < ad.W; gx += 4) {
        const u64 sum = buf[(size_t)gx * 64 + lane];   // at most 16 terms below q: below 2^64 (2^45 for q < 2^41)
        const size_t k = ((size_t)gid[gx] << 6) + lane;
        z[(size_t)lam * n + k] = M.fp ? fcanon(u2d(sum), FMod{M.qd, M.qinv}) : reduce64(sum, M);
    }
}

bool aut_sum_doubling(const DevTables &t, u64 *z, const u64 *a, int count, int l, i64 r1, int m, u64 g1,
                      hipStream_t st) {
    // r1: the first rotation (d s), m: terms (m - 1 rotations r1, 2 r1, ..); g1 its Galois element
    if (t.log_n < 9 || m < 2 || m > 16 || (m & (m - 1)) || r1 == 0) return false;
    const i64 s_abs = r1 < 0 ? -r1 : r1;
    if (s_abs & (s_abs - 1)) return false;   // a power of 2, so that the shifts walk one line
    const int T = 1 << (t.log_n - 7);
    AutDbl ad{};
    ad.log_m = __builtin_ctz((unsigned)m);
    ad.dir = r1 < 0 ? -1 : 1;
    ad.step = s_abs < T ? (int)s_abs : 0;
    ad.U = ad.step ? T / ad.step : 1;
    ad.W = ad.U < 64 ? ad.U : 64;
    ad.cyc = ad.W == ad.U ? 1 : 0;
    ad.nb = ad.cyc ? ad.U : ad.W + m - 1;
    ad.lines = ad.step ? 2 * ad.step : 2 * T;
    const u64 mask = (2ULL << t.log_n) - 1;
    u64 g = g1 & mask;
    for (int j = 0; j < ad.log_m; ++j) {
        ad.gp[j] = g;
        g = (g * g) & mask;
    }
    if (ad.nb * 64 > 20 * 256) return false;
    const int n_limbs = count * l;
    TScope ts_(t, "aut_sum_dbl", 16.0 * (double)n_limbs * t.n, st);
    if (!n_limbs) return true;
    const size_t items = (size_t)n_limbs * ad.lines * (ad.U / ad.W);
    const size_t lds = (size_t)ad.nb * 64 * sizeof(u64) + (size_t)ad.nb * sizeof(int);
    gck_launch(aut_sum_dbl, dim3((unsigned)items), dim3(256), (unsigned)lds, st, z, a, l, t.log_n, ad, n_limbs, t.mods);
    check_launch();
    return true;
}

// ---------------------------------------------------------------- samplers and conversions

__global__ void sample_uniform(u64 *out, u64 seed, u64 sid, size_t total, int log_n, ModMap mm, const ModInfo *mods) {
    const size_t n = (size_t)1 << log_n;
    const u64 st = sm_out(seed, sid);
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);
        u64 k = idx & (n - 1);
        int ch = chain_of(lam, mm);
        u64 ctr = 2 * ((u64)ch * n + k);
        out[idx] = mod_u128(sm_out(st, ctr), sm_out(st, ctr + 1), mods[ch].q);
    }
}
void k_sample_uniform(const DevTables &t, u64 *out, u64 seed, u64 sid, int n_limbs, ModMap m, int, hipStream_t st) {
    TScope ts_(t, "sample_uniform", 8.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(sample_uniform, ew_grid(total), dim3(kEwThreads), 0, st, out, seed, sid, total, t.log_n, m, t.mods);
    check_launch();
}

__global__ void sample_small(i64 *out, u64 seed, u64 sid, int n, int kind) {
    const u64 st = sm_out(seed, sid);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        u64 w = sm_out(st, (u64)i);
        if (kind == 0) out[i] = (i64)__popcll(w & 0x1FFFFFULL) - (i64)__popcll((w >> 21) & 0x1FFFFFULL);
        else out[i] = (i64)(w % 3) - 1;
    }
}
void k_sample_cbd(i64 *out, u64 seed, u64 sid, int n, hipStream_t st) {
    gck_launch(sample_small, ew_grid(n), dim3(kEwThreads), 0, st, out, seed, sid, n, 0);
    check_launch();
}
void k_sample_ternary(i64 *out, u64 seed, u64 sid, int n, hipStream_t st) {
    gck_launch(sample_small, ew_grid(n), dim3(kEwThreads), 0, st, out, seed, sid, n, 1);
    check_launch();
}

__global__ void ew_signed_to_limbs(u64 *out, const i64 *in, size_t total, int log_n, ModMap mm, const ModInfo *mods) {
    const size_t n = (size_t)1 << log_n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);
        size_t k = idx & (n - 1);
        const ModInfo &M = mods[chain_of(lam, mm)];
        i64 v = in[k];
        u64 r;
        if (v >= 0) r = reduce64((u64)v, M);
        else {
            r = reduce64((u64)(-(v + 1)), M);   // -(v+1) >= 0
            r = M.q - 1 - r;
        }
        out[idx] = r;
    }
}
void k_signed_to_limbs(const DevTables &t, u64 *out, const i64 *in, int n_limbs, ModMap m, hipStream_t st) {
    TScope ts_(t, "ew_signed_to_limbs", 8.0 * (double)(n_limbs + 1) * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_signed_to_limbs, ew_grid(total), dim3(kEwThreads), 0, st, out, in, total, t.log_n, m, t.mods);
    check_launch();
}

__global__ void ew_mont(u64 *x, size_t total, int log_n, ModMap mm, const ModInfo *mods, int to) {
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        int lam = (int)(idx >> log_n);
        const ModInfo &M = mods[chain_of(lam, mm)];
        x[idx] = to ? mul_shoup(x[idx], M.r_mod, M.r_mod_sh, M.q) : redc(0, x[idx], M);
    }
}
void k_to_mont(const DevTables &t, u64 *x, int n_limbs, ModMap m, hipStream_t st) {
    TScope ts_(t, "ew_mont", 16.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_mont, ew_grid(total), dim3(kEwThreads), 0, st, x, total, t.log_n, m, t.mods, 1);
    check_launch();
}
void k_from_mont(const DevTables &t, u64 *x, int n_limbs, ModMap m, hipStream_t st) {
    TScope ts_(t, "ew_mont", 16.0 * (double)n_limbs * t.n, st);
    size_t total = (size_t)n_limbs << t.log_n;
    if (!total) return;
    gck_launch(ew_mont, ew_grid(total), dim3(kEwThreads), 0, st, x, total, t.log_n, m, t.mods, 0);
    check_launch();
}

}  // namespace gck
