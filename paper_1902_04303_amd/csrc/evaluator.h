// Context, ciphertext batches and the evaluation operations (host driver over the HIP kernels).
#pragma once

#include <map>
#include <mutex>
#include <tuple>

#include "ckks_internal.h"

struct ckks_ct;

struct ckks_ctx {
    gck::Params p;
    gck::DevTables tab;
    std::vector<gck::ModInfo> h_mods;
    hipStream_t stream = nullptr;
    std::unique_ptr<gck::Pool> pool;
    void *table_mem = nullptr;     // device tables (hipMalloc, outside the pool)
    void *ks_mem = nullptr;        // key-switch tables below (hipMalloc, outside the pool)
    // key-switch tables, per level l (index l = 1..L+1): ModUp basis conversion of every digit group to
    // the other targets (K entries per ciphertext), digit index of (group, target), inverse-NTT scales
    struct KsLevel {
        int K = 0;
        gck::ConvEntry *up = nullptr;
        int *didx = nullptr;
        gck::LimbScale *up_scale = nullptr;
    };
    std::vector<KsLevel> ks_levels;
    gck::ConvEntry *down_conv = nullptr;     // ModDown: target q_i from the special primes, i <= L
    gck::LimbScale *down_scale = nullptr;    // ModDown inverse-NTT scales of the special primes
    gck::ChainConst p_inv{};                 // P^-1 mod every chain modulus
    gck::u64 *p_inv_dev = nullptr, *p_inv_sh_dev = nullptr;   // the same on the device
    double *p_inv_d_dev = nullptr;                             // and as doubles (FP64 moduli)
    // rescale by q_j (j = 1..L): q_j^-1 mod every chain modulus, with Shoup companions and as doubles
    struct QInv {
        gck::u64 *v = nullptr, *sh = nullptr;
        double *d = nullptr;
    };
    std::vector<QInv> q_inv;
    // a product's relinearisation fused with its rescale by q_j (j = 1..L): the division by B = P q_j, its
    // moduli ordered q_j, p_1..p_alpha: conversion to each q_i, i < j (j entries), the inverse-NTT scales
    // N^-1 (B/b)^-1 mod b (alpha + 1 entries) and (P q_j)^-1 mod every chain modulus (value, Shoup
    // companion, double)
    struct RsLevel {
        gck::ConvEntry *conv = nullptr;
        gck::LimbScale *scale = nullptr;
        gck::u64 *binv = nullptr, *binv_sh = nullptr;
        double *binv_d = nullptr;
    };
    std::vector<RsLevel> rs_levels;
    int ng = 0;                              // digit groups of a key (at L + 1 limbs)
    // keys: a context made by keygen holds the secret (the client's side); an evaluating context may hold
    // only imported switching keys (and a public key), never the secret
    bool have_secret = false;      // sk and sk_ntt are set (keygen)
    bool have_pk = false;          // pk is set (keygen or import)
    std::vector<int64_t> sk;       // secret, signed coefficients
    gck::DBuf sk_ntt;              // [L+1+alpha][N]: s mod q_0..q_L, p_1..p_alpha in NTT form
    gck::DBuf pk;                  // [2][L+1][N] NTT form
    std::map<uint64_t, gck::DBuf> ksk;   // key id (0 = relinearisation, else Galois element) -> [2][ng][L+1+alpha][N]
    // counters and optional per-kernel timing
    uint64_t n_keyswitch = 0, n_limb_ntt = 0, n_launch = 0;
    uint64_t n_keyswitch_ct = 0;   // key switches counted per ciphertext (a call over count ciphertexts adds count)
    gck::KTimer timer;
    // serialises use of the context between host threads (client calls and a server's worker)
    std::recursive_mutex mu;
    hipStream_t copy_stream = nullptr;   // second stream for host-to-device prefetch (default priority)
    // second compute stream (default priority) with its own pool: work independent of the main stream's
    // runs there concurrently (see OnStream); buffers move between the two only across event waits
    hipStream_t aux_stream = nullptr;
    std::unique_ptr<gck::Pool> aux_pool;
    int n_streams = 2;   // 1: the circuit runs in order on `stream` only
    // the per-batch part stacks the k covariates' products of a chunk into one batch while it holds at most
    // this many ciphertexts (0: one covariate at a time); results are identical either way.  Off by default:
    // on one stream the stack saves about 1 ms per step at the dataset shape, but on two streams its larger
    // launches leave the logistic-regression part fewer gaps to fill (61.5 against 62.7 ms)
    int stack_cts = 0;
    bool capturing = false;   // a HIP graph capture of the circuit is in progress on `stream`
    // schedules chosen by the tuner per input shape (R, k, kappa, SNP batches): chunk, stream count, stack
    struct Schedule {
        int chunk = 0, streams = 2, stack = 0;
        double ms = 0;
    };
    std::map<std::tuple<int, int, int, int>, Schedule> tuned;
    bool use_tuned = false;
    bool keep_s_proj = true;   // the circuit's outputs include S' of every SNP batch
    // slot-class masks in NTT form by (period, first class, end class, limbs, scale bits), made once and
    // then only read
    std::map<std::tuple<int, int, int, int, uint64_t>, gck::DBuf> mask_cache;
    // the plaintexts a + b X^(N/2) in NTT form by (limbs, a, b), made once and then only read
    std::map<std::tuple<int, int64_t, int64_t>, gck::DBuf> mono_cache;
    ~ckks_ctx();
};

// A batch of `count` ciphertexts at the same depth and tracked scale, data [count][2][limbs][N] in
// NTT form (this library's evaluation order).
struct ckks_ct {
    ckks_ctx *ctx = nullptr;
    int count = 0, depth = 0, limbs = 0;
    double scale = 0;
    gck::DBuf data;
};

namespace gck {

using Ct = std::unique_ptr<ckks_ct>;

Ct new_ct(ckks_ctx &c, int count, int depth, double scale);
Ct clone(ckks_ctx &c, const ckks_ct &a);
// ciphertexts [first, first + n) of batch a, sharing its memory (valid while a lives; never freed)
Ct view(const ckks_ct &a, int first, int n);
// one batch holding the ciphertexts of every part in order (same depth and scale)
Ct stack(ckks_ctx &c, const std::vector<const ckks_ct *> &parts);

void ntt_fwd(ckks_ctx &c, u64 *buf, int n_limbs, ModMap m);
void ntt_inv(ckks_ctx &c, u64 *buf, int n_limbs, ModMap m);

// ---- scheme operations (count-batched; an operand with fewer ciphertexts, a divisor of the other's
//      count, is read cyclically: ciphertext i pairs with ciphertext i mod count)
Ct add(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b);
Ct sub(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b);
Ct neg(ckks_ctx &c, const ckks_ct &a);
Ct mul_int(ckks_ctx &c, const ckks_ct &a, i64 k);
Ct add_const(ckks_ctx &c, const ckks_ct &a, double v);
Ct rescale(ckks_ctx &c, const ckks_ct &a);
Ct mod_drop(ckks_ctx &c, const ckks_ct &a, int depth);
Ct mul_const(ckks_ctx &c, const ckks_ct &a, double v);
Ct mul_mask(ckks_ctx &c, const ckks_ct &a, int R);
// sum_i a_i * m_i, m_i the exact mask of 1 at the slots s = j mod P_i for j0_i <= j < j1_i encoded at the
// operands' common scale s, then one rescale; the result scale is (s * s) / q (as mul_mask)
struct MaskTerm {
    const ckks_ct *a;
    int P, j0, j1;
};
Ct mask_sum(ckks_ctx &c, const std::vector<MaskTerm> &terms);
// a times re + im X^(N/2): every slot times the Gaussian integer re + im i, exact, same depth and scale
Ct mul_gauss(ckks_ctx &c, const ckks_ct &a, i64 re, i64 im);
// a times X^(N/2) (neg: -X^(N/2)): every slot times i (or -i)
Ct mul_i(ckks_ctx &c, const ckks_ct &a, bool neg);
Ct align(ckks_ctx &c, const ckks_ct &a, int depth, double scale, double factor);
Ct set_scale(ckks_ctx &c, Ct a, double factor);
// sum_i a_i * b_i: one tensor per pair accumulated, one relinearisation, one rescale
Ct mul_sum(ckks_ctx &c, const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &pairs);
// the products of several pairs as consecutive ciphertexts of one batch (one key switch for all of them)
Ct mul_stack(ckks_ctx &c, const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &pairs);
Ct mul(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b);
// relinearise and rescale a batch of tensors d ([count][3][l][N] at `depth`, operand scales sa, sb)
Ct relin_rescale(ckks_ctx &c, DBuf d, int count, int depth, int l, double sa, double sb);
// M-materialised layout: sum_i cols_i (x) rep_{b, i} for every batch b (rep: [cnt][n] ciphertexts)
Ct mul_sum_rep(ckks_ctx &c, const ckks_ct &cols, const ckks_ct &rep);
// c0 of ciphertext i plus the exact indicator of the slots = i mod R (at a's scale)
Ct add_slot_indicators(ckks_ctx &c, const ckks_ct &a, int R);
Ct apply_galois(ckks_ctx &c, const ckks_ct &a, u64 g);
Ct rotate(ckks_ctx &c, const ckks_ct &a, i64 r);
// Rot(a, r) for every r of rots as separate ciphertexts, with one ModUp of a's second polynomial shared by
// all of them (bit-identical to one rotate per r)
std::vector<Ct> rotate_many(ckks_ctx &c, const ckks_ct &a, const std::vector<i64> &rots);
// a + sum_i Rot(a, rots[i]) with one key switch shared by the rotations (at most 16)
Ct rotate_sum(ckks_ctx &c, const ckks_ct &a, const std::vector<i64> &rots);
Ct conjugate(ckks_ctx &c, const ckks_ct &a);
u64 galois_rotate(const ckks_ctx &c, i64 r);
u64 galois_rotate_n(int n, i64 r);   // the same for ring degree n
u64 galois_conj(const ckks_ctx &c);
bool has_key(const ckks_ctx &c, u64 id);

// ---- keys / encryption
void keygen(ckks_ctx &c, u64 seed, const std::vector<u64> &galois);
// canonical coefficient-form keys (as exported) into the context's device form
void import_public_key(ckks_ctx &c, const u64 *buf);
void import_switching_key(ckks_ctx &c, u64 key_id, const u64 *buf);
Ct encrypt(ckks_ctx &c, const i64 *m, int depth, double scale, u64 seed);
// c0 + c1 s in coefficient form, centred over q_0 (q_0 q_1 when limbs >= 2), as long doubles
std::vector<long double> decrypt_poly(ckks_ctx &c, const ckks_ct &a, int index);
void export_ct(ckks_ctx &c, const ckks_ct &a, int index, u64 *out);
Ct import_ct(ckks_ctx &c, const u64 *in, int depth, double scale);

// ---- host math (encode.cpp)
void encode_poly(int n, const double *re, const double *im, size_t n_slots, double scale, i64 *out);
void decode_poly(int n, const double *coeffs, double *re, double *im);
void mask_poly(int n, int R, double scale, i64 *out);

// ---- the product without device allocation (noalloc.hip)
void noalloc_init();                     // takes the current device's scratch address (once per device)
size_t noalloc_max_bytes();
size_t mul_noalloc_bytes(const ckks_ctx &c, int count, int l);
void mul_noalloc(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b, ckks_ct &out);

void sync(ckks_ctx &c);
// While alive, the context's operations run on its auxiliary stream and allocate from its auxiliary pool
// (both made on first use).  The caller orders the two streams with events (fork_to_aux, join_from_aux).
struct OnStream {
    ckks_ctx &c;
    explicit OnStream(ckks_ctx &ctx);
    ~OnStream();
    OnStream(const OnStream &) = delete;
    OnStream &operator=(const OnStream &) = delete;
};
void ensure_aux(ckks_ctx &c);
// make stream `to` wait for the work enqueued so far on stream `from`
void stream_wait(hipStream_t to, hipStream_t from);

}  // namespace gck
