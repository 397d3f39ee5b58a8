// Internal declarations of the MI355X RNS-CKKS library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/gwas_ckks.h"

namespace gck {

using u64 = uint64_t;
using i64 = int64_t;
using u128 = unsigned __int128;

constexpr int kMaxMods = 64;     // q_0..q_L and the special primes
constexpr int kMaxAlpha = 8;     // special primes p_1 .. p_alpha of the key-switching modulus P (alpha <= 8)
constexpr int kMaxSpecial = kMaxAlpha + 1;   // sources of one basis conversion (P, or P q_j for a fused rescale)

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};
void hip_check(hipError_t e, const char *what);
#define GCK_HIP(x) ::gck::hip_check((x), #x)

// ---------------------------------------------------------------- per-modulus constants (device copy)
struct ModInfo {
    u64 q;
    u64 mont_inv;      // -q^-1 mod 2^64 (Montgomery)
    u64 barrett;       // floor(2^64 / q)
    u64 r_mod;         // 2^64 mod q
    u64 r_mod_sh;      // Shoup companion of r_mod
    u64 r2_mod;        // 2^128 mod q
    u64 ninv, ninv_sh; // N^-1
    u64 w1ninv, w1ninv_sh;  // psi^-1 (first inverse twiddle) * N^-1
    // moduli below 2^41 also run their NTT butterflies in FP64 (exact products by FMA)
    u64 fp;            // 1 when q < 2^41
    double qd, qinv, ninv_d;   // q, RN(1 / q), N^-1 mod q as doubles
    double rinv_d;             // 2^-64 mod q as a double (leaves the Montgomery form of key products)
    double c32_d;              // 2^32 mod q as a double (reduces 64-bit words in FP64)
};
constexpr int kFpModBits = 41;

// ---------------------------------------------------------------- parameters and prime chain
struct Params {
    int log_n = 0, n = 0, levels = 0, log2_scale = 0;
    int alpha = 0;             // digit-group size of the key switch = number of special primes
    std::vector<u64> q;        // q_0 .. q_L
    std::vector<u64> P;        // special primes p_1 .. p_alpha
    std::vector<double> scales;  // canonical Delta_0 .. Delta_L
    int limbs_at(int depth) const { return levels + 1 - depth; }
    u64 dropped_at(int depth) const { return q[levels - depth]; }  // prime removed by the rescale at depth
    int p_index() const { return levels + 1; }                      // chain index of p_1
    int n_mods() const { return levels + 1 + alpha; }               // chain indices q_0..q_L, p_1..p_alpha
    u64 mod(int idx) const { return idx <= levels ? q[idx] : P[idx - levels - 1]; }
};
// Key-switching digit groups (hybrid decomposition, group size a = alpha): group 0 is {q_0 .. q_{a-2}},
// group b >= 1 is {q_{a b - 1} .. q_{a b + a - 2}}; a ciphertext with l limbs uses the 1 + l / a groups
// with a member below l, cut at l.
__host__ __device__ inline int ks_groups(int l, int a) { return 1 + l / a; }
__host__ __device__ inline int ks_group_first(int b, int a) { return b == 0 ? 0 : a * b - 1; }
__host__ __device__ inline int ks_group_size(int b, int l, int a) {
    const int f = ks_group_first(b, a), e = a * (b + 1) - 1;
    return (e < l ? e : l) - f;
}
Params make_params(int log_n, int levels, int log2_scale, int alpha);
u64 mulmod_host(u64 a, u64 b, u64 q);
u64 powmod_host(u64 b, u64 e, u64 q);
u64 invmod_host(u64 a, u64 q);
u64 find_psi(u64 q, int n);
i64 round_half_away(double x);

// ---------------------------------------------------------------- memory pool (device)
class Pool {
public:
    Pool(const ckks_allocator *alloc, size_t budget);
    // An arena over one fixed device region [base, base + bytes): get() takes the next 256-byte aligned
    // block (CKKS_E_NOMEM past the end), put() gives back only the most recent block; the allocator is
    // never called and nothing is freed when the pool is destroyed.
    static std::unique_ptr<Pool> arena(void *base, size_t bytes);
    ~Pool();
    void *get(size_t bytes);
    void put(void *p, size_t bytes);
    void trim();
    // Graph capture: blocks handed out between capture_begin and capture_end are recorded; capture_end
    // takes those that are free again out of the free lists and returns them (they stay reserved for the
    // captured graph, whose replays write them) until give_back.
    void capture_begin();
    std::vector<std::pair<void *, size_t>> capture_end();
    void give_back(const std::vector<std::pair<void *, size_t>> &blocks);
    std::unique_ptr<Pool> sibling() const;   // an empty pool with the same allocator (no budget)
    size_t in_use = 0, cached = 0, peak = 0, n_alloc = 0, budget = 0;
    hipStream_t stream = nullptr;

private:
    ckks_allocator alloc_{};
    bool have_alloc_ = false;
    bool capturing_ = false;
    std::map<void *, size_t> captured_;
    char *arena_base_ = nullptr;   // arena mode when set
    size_t arena_bytes_ = 0, arena_top_ = 0;
    std::multimap<size_t, void *> free_;
    void *raw_alloc(size_t bytes);
    void raw_free(void *p, size_t bytes);
};

// device buffer with RAII return to the pool
struct DBuf {
    Pool *pool = nullptr;
    u64 *ptr = nullptr;
    size_t words = 0;
    DBuf() = default;
    DBuf(Pool *p, size_t w) : pool(p), ptr(static_cast<u64 *>(p->get(w * 8))), words(w) {}
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept { *this = std::move(o); }
    DBuf &operator=(DBuf &&o) noexcept {
        release();
        pool = o.pool; ptr = o.ptr; words = o.words;
        o.ptr = nullptr; o.words = 0;
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (ptr && pool) pool->put(ptr, words * 8);
        ptr = nullptr; words = 0;
    }
};

// ---------------------------------------------------------------- kernels (kernels.hip)
// Every polynomial buffer is a contiguous array of limbs of N words.  The chain
// index (0..L for q_i, L+1.. for the special primes) of limb lam is given by a ModMap:
//     t = lam % period;  chain = (t < nq) ? t : p_idx + (t - nq)
// and t >= nq is the special prime p_idx + (t - nq); e.g. ciphertext data [count][2][l][N] has
// period = nq = l; key-switch accumulators [count][2][l + alpha][N] have period l + alpha, nq = l.
struct ModMap {
    int period, nq, p_idx;
    int q_off = 0;   // t < nq is q_{q_off + t}
};
inline ModMap map_q(int l) { return ModMap{l, l, 0}; }

// Optional per-kernel timing (off by default).  Each timed launch carries a start and a stop event that
// the runtime sets when the kernel itself starts and ends (hipExtLaunchKernelGGL), so the time excludes
// waiting for workgroup slots behind kernels of another stream.  A region (e.g. "keyswitch": every kernel
// of one key switch) is timed by events recorded on its stream before its first and after its last
// launch; regions are recorded only when `only` names them.
struct KTimer {
    bool on = false;
    std::string only;   // when not empty, only launches (or regions) of this name are recorded
    struct Rec {
        int id;
        hipEvent_t a, b;
        double bytes, flops, pass_bytes;
        bool launched;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    std::vector<std::string> names;
    std::map<std::string, int> ids;
    struct Stat {
        uint64_t count = 0;
        // algorithmic HBM bytes (each word of a transform read and written once over its two passes) and
        // FP64 operations (0: not declared), and the bytes a pass moves when it reads and writes each word
        // once itself
        double ms = 0, bytes = 0, flops = 0, pass_bytes = 0;
    };
    std::vector<Stat> stats;
    hipEvent_t take();
    int id_of(const char *name);
    int begin(const char *name, double bytes, double flops, hipStream_t st, double pass_bytes = -1);
    void end(int idx, hipStream_t st);
    int region_begin(const char *name, double bytes, hipStream_t st);
    void region_end(int idx, hipStream_t st);
    void collect();   // synchronises, folds recorded events into stats
    void reset();
    ~KTimer();
};

// RAII timing of a region of launches on one stream (recorded when the timer is on and `only` names it)
struct KRegion {
    KTimer *t;
    int idx = -1;
    hipStream_t st;
    KRegion(KTimer *timer, const char *name, double bytes, hipStream_t s) : t(timer), st(s) {
        if (t && t->on) idx = t->region_begin(name, bytes, st);
    }
    ~KRegion() {
        if (idx >= 0) t->region_end(idx, st);
    }
    KRegion(const KRegion &) = delete;
    KRegion &operator=(const KRegion &) = delete;
};

struct DevTables {
    KTimer *timer = nullptr;
    ModInfo *mods = nullptr;            // [n_mods]
    u64 *psi = nullptr, *psi_sh = nullptr, *ipsi = nullptr, *ipsi_sh = nullptr;  // [n_mods][N]
    double *psi_f = nullptr, *ipsi_f = nullptr;   // [n_mods][N] the same twiddles as doubles (FP64 moduli)
    int n = 0, log_n = 0, n_mods = 0;
};

struct ChainConst {     // one constant per chain index (value and Shoup companion), passed by value
    u64 v[kMaxMods];
    u64 sh[kMaxMods];
};

void k_ntt_forward(const DevTables &t, u64 *buf, int n_limbs, ModMap m, hipStream_t st);
void k_ntt_inverse(const DevTables &t, u64 *buf, int n_limbs, ModMap m, hipStream_t st);
// Where the first pass of an out-of-place NTT reads output limb lam from:
//   src limb  (lam / div) * mul + add + (lam % div) * inner
// and how the word is brought to output limb lam's modulus: kPlain (already reduced),
// kReduce (any word < 2^64, e.g. a digit of another modulus: ModUp), kCentred (centred lift of a
// residue modulo chain src_chain: rescale and ModDown).
// kConv: basis conversion.  Output limb lam takes entry e = conv[lam % conv_period] and row
// r = lam / conv_period; its modulus is chain e.chain and its word is sum_{m < e.nsrc} y_m c_m mod that
// modulus, y_m = src limb r * src_stride + e.src + m (a residue of another modulus, below 2^47 unless
// bit m of e.big is set), c_m = e.c[m] (with its Shoup companion and FP64 copy).
// basis conversion to the modulus `chain`: sum over nsrc consecutive source limbs from `src` of
// y_m c[m]; big bit m: source m's residues need splitting (modulus >= 2^47); centre: each y_m is first
// taken as its centred representative, y_m - s_m when y_m > s_m / 2 (half[m] = s_m >> 1, s_m the source
// modulus; negsq[m] = -s_m mod the target, sqd[m] = s_m as a double)
struct ConvEntry {
    int src, nsrc, chain, big, centre;
    u64 c[kMaxSpecial], c_sh[kMaxSpecial];
    double cd[kMaxSpecial];
    u64 half[kMaxSpecial], negsq[kMaxSpecial];
    double sqd[kMaxSpecial];
};
struct Gather {
    const u64 *ptr;
    int div, mul, add, inner;
    int mode, src_chain;
    const ConvEntry *conv;   // kConv only
    int conv_period, src_stride;
    u64 cmul, cmul_sh;       // kCentred: when cmul != 0, each source residue is first multiplied by cmul
};                           // modulo the source modulus (Shoup companion cmul_sh)
enum { kPlain = 0, kReduce = 1, kCentred = 2, kConv = 3 };
// per output limb scale of an inverse NTT (replaces N^-1): entry lam % period
struct LimbScale {
    u64 w, w_sh;
    double wd;
};
inline Gather gather_plain(const u64 *p) { return Gather{p, 1, 1, 0, 0, kPlain, 0}; }
// Epilogue of the forward NTT that ends a key switch's ModDown: output limb lam becomes
// (acc - ntt) * P^-1 (+ add) (+ aut) with acc and add gathered (add may be null; add_even: added only on
// rows lam / rowlen that are even, the first polynomial of each ciphertext); pinv[chain], pinv_sh[chain]
// and pinv_d[chain] (device) hold P^-1 modulo each chain modulus, with Shoup companions and as doubles.
// aut (may be null) is a ciphertext batch laid out like the output, [count][2][rowlen][N]: even rows add
// self * aut[lam][k] +
// sum_i aut[lam][k_i] with k_i the source word of the NTT-domain automorphism X -> X^g[i], odd rows add
// self * aut[lam][k] (rotate-and-sum: a + sum_i sigma_i(a c0); a single Galois map: sigma(a c0)); self is
// aut_self on odd rows and (aut_self == 1) on even rows.
constexpr int kMaxKeys = 16;
struct ModDownEpi {
    Gather acc, add;
    int add_even, rowlen;
    const u64 *pinv, *pinv_sh;
    const double *pinv_d;
    const u64 *aut;
    int aut_self, n_g;
    u64 g[kMaxKeys];
    int acc_mul;           // 1: acc is first multiplied by km[chain] (an integer constant modulo each modulus)
    u64 km[kMaxMods];
    // a product's relinearisation fused with its rescale: the added term (d0, d1 of the tensor) is read
    // from [count][3][l][N] (row r = lam / rowlen of the output takes ciphertext r / 2, polynomial r % 2:
    // add.ptr + ((r / 2) add_ct + (r % 2) add_poly + lam % rowlen) N) and multiplied by addmul[chain]
    // (q_{l-1}^-1), with pinv = (P q_{l-1})^-1; add_ct == 0: the plain gather of `add`
    const u64 *addmul = nullptr, *addmul_sh = nullptr;
    const double *addmul_d = nullptr;
    int add_ct = 0, add_poly = 0;
};
void k_ntt_forward_g(const DevTables &t, u64 *buf, const Gather &in, int n_limbs, ModMap m, hipStream_t st,
                     const ModDownEpi *epi = nullptr);
// scale (nullable): multiply output limb lam by scale[lam % scale_period].w instead of N^-1
void k_ntt_inverse_g(const DevTables &t, u64 *buf, const Gather &in, int n_limbs, ModMap m, hipStream_t st,
                     const LimbScale *scale = nullptr, int scale_period = 1);
// out = a op b over n_limbs limbs; a is read at limb (lam % na_limbs), b at (lam % nb_limbs)
void k_add(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st);
void k_sub(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st);
// acc[row][l-1] += pm add[row / 2][row % 2][l-1] (NTT domain, modulo q_{l-1}) for the 2 count rows of a
// key switch's accumulators ([count][2][nt][N]) and a tensor add ([count][3][l][N])
void k_add_scaled_last(const DevTables &t, u64 *acc, const u64 *add, int count, int nt, int l, u64 pm, u64 pm_sh,
                       u64 q, hipStream_t st);
void k_tensor_rep_sum(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int cnt, int n_rows, int l,
                      hipStream_t st);
void k_add_rotated_plain(const DevTables &t, u64 *out, const u64 *a, const u64 *pt, int count, int l, int R,
                         hipStream_t st);
void k_mul(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int n_limbs, ModMap m, int na, int nb,
           hipStream_t st);
// out = a * c[chain]
void k_mul_const(const DevTables &t, u64 *out, const u64 *a, int n_limbs, ModMap m, const ChainConst &c,
                 hipStream_t st);
// ct data [count][2][l][N]: out = a with c[chain] added to the limbs of poly 0 (out may be a)
void k_add_const_c0(const DevTables &t, u64 *out, const u64 *a, int count, int l, const ChainConst &c, hipStream_t st);
// tensor of [count][2][l] ciphertexts into [count][3][l]; a / b read at ciphertext (c % na) / (c % nb)
// sum over up to kMaxTensorPairs pairs of the tensors of k_tensor (pair p read at ciphertexts c % na[p] and
// c % nb[p]), stored once into out ([count][3][l][N]; added to out when accumulate)
constexpr int kMaxTensorPairs = 8;
struct TensorPairs {
    const u64 *a[kMaxTensorPairs];
    const u64 *b[kMaxTensorPairs];
    int na[kMaxTensorPairs], nb[kMaxTensorPairs];
    int n;
};
void k_tensor_sum(const DevTables &t, u64 *out, const TensorPairs &tp, int count, int l, bool accumulate, hipStream_t st);
void k_tensor(const DevTables &t, u64 *out, const u64 *a, const u64 *b, int count, int l, int na, int nb,
              bool accumulate, hipStream_t st);
// NTT-domain automorphism X -> X^g on every limb
void k_automorph(const DevTables &t, u64 *out, const u64 *a, int n_limbs, u64 g, hipStream_t st);
// out[r][0:words] = in[r][0:words] with row strides (in words)
void k_copy_rows(u64 *out, size_t out_stride, const u64 *in, size_t in_stride, int rows, size_t words,
                 hipStream_t st);
// Keys of one key-switch inner product: key i is paired with the NTT-domain automorphism X -> X^g[i] of
// the digits (g[i] == 0: none).
struct KsKeys {
    const u64 *key[kMaxKeys];
    u64 g[kMaxKeys];
    int m;
};
// key-switch inner product over the targets t < l + alpha (q_0..q_{l-1}, p_1..p_alpha):
//   acc[c][comp][t] = sum_i sum_b sigma_i(D_b[c][t]) * key_i[comp][b][chain(t)],
// D_b[c][t] = digits[c][didx[b (l + alpha) + t]] when that index is >= 0, else limb t of ciphertext c
// gathered by `own` (the digit's residue at its own group's primes equals the input residue).  Keys are
// [2][ng][L + 1 + alpha][N] in NTT and Montgomery form (times 2^64); digits hold K limbs per ciphertext.
void k_ks_inner(const DevTables &t, u64 *acc, const u64 *digits, int K, const int *didx, const Gather &own,
                const KsKeys &keys, int ng, int count, int l, int levels, int alpha, hipStream_t st);
// z[c][j] = a[c][0][j] + sum_i sigma_i(a[c][0][j]) mod q_j (NTT domain) for the keys' automorphisms (any
// Galois maps, up to kMaxKeys), a [count][2][l][N] and z [count][l][N]
void k_aut_sum(const DevTables &t, u64 *z, const u64 *a, int count, int l, const KsKeys &keys, hipStream_t st);
// the same for the rotations r1, 2 r1, .., (m - 1) r1 (m a power of 2 up to 16, |r1| a power of 2; g1 the
// Galois element of r1) by log2 m doubling steps in LDS; false (nothing launched) for other rotation sets
bool aut_sum_doubling(const DevTables &t, u64 *z, const u64 *a, int count, int l, i64 r1, int m, u64 g1,
                      hipStream_t st);
// samplers of the test-only SplitMix64 streams
void k_sample_uniform(const DevTables &t, u64 *out, u64 seed, u64 sid, int n_limbs, ModMap m, int mi_of_p,
                      hipStream_t st);
void k_sample_cbd(i64 *out, u64 seed, u64 sid, int n, hipStream_t st);
void k_sample_ternary(i64 *out, u64 seed, u64 sid, int n, hipStream_t st);
// signed small coefficients -> residues for every limb of a ModMap'd buffer
void k_signed_to_limbs(const DevTables &t, u64 *out, const i64 *in, int n_limbs, ModMap m, hipStream_t st);
// Montgomery form conversion (x * 2^64 mod q and back)
void k_to_mont(const DevTables &t, u64 *x, int n_limbs, ModMap m, hipStream_t st);
void k_from_mont(const DevTables &t, u64 *x, int n_limbs, ModMap m, hipStream_t st);

}  // namespace gck
