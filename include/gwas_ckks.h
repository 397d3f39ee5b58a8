/*
 * gwas_ckks.h — C ABI of the MI355X RNS-CKKS evaluator and the encrypted
 * modified semi-parallel GWAS of Sim, Chan, Chen, Tan and Aung, "Achieving
 * GWAS with Homomorphic Encryption" (arXiv 1902.04303).
 *
 * Conventions
 *   - Every function returns 0 (CKKS_OK) or a negative CKKS_E_* code; no
 *     exception or abort crosses this boundary.  ckks_last_error() returns a
 *     thread-local message for the last failure of the calling thread.
 *   - Handles are opaque.  A context owns its tables, its device memory pool and
 *     every key, plaintext and ciphertext created from it; destroying the
 *     context frees all of them.  A context is not thread-safe: use one per host
 *     thread or stream.
 *   - Device work is enqueued on the HIP stream given to ckks_ctx_create (NULL:
 *     the null stream).  Functions that hand data to the host synchronise that
 *     stream; the others return with work still queued.
 *   - Host buffers are owned by the caller.  Device memory comes from the
 *     context's pool, which takes slabs from the allocator callbacks given at
 *     creation (NULL: hipMalloc / hipFree).
 *   - Polynomial data crosses the boundary in the canonical form: coefficient
 *     domain, standard representatives in [0, q_i), laid out [poly][limb][coeff]
 *     (a ciphertext is [2][limbs][N] uint64).
 *   - "Depth" d counts rescales from a fresh top-level ciphertext; a ciphertext
 *     at depth d has L + 1 - d limbs q_0 .. q_{L-d}.
 */
#ifndef GWAS_CKKS_H
#define GWAS_CKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CKKS_OK = 0,
    CKKS_E_INVALID_ARG = -1,    /* bad pointer, size or value */
    CKKS_E_PARAM_MISMATCH = -2, /* operands differ in context, depth or scale */
    CKKS_E_LEVEL = -3,          /* not enough levels left for the operation or circuit */
    CKKS_E_KEY_MISSING = -4,    /* a needed relinearisation / Galois key was not generated */
    CKKS_E_NOMEM = -5,          /* device memory (or the pool budget) exhausted */
    CKKS_E_HIP = -6,            /* a HIP runtime call failed */
    CKKS_E_CANCELLED = -7,      /* a job was cancelled before it completed */
    CKKS_E_NOT_READY = -8       /* a submitted job has not finished yet */
};

typedef struct ckks_ctx ckks_ctx;
typedef struct ckks_ct ckks_ct;
typedef struct gwas_enc_input gwas_enc_input;
typedef struct gwas_enc_output gwas_enc_output;
typedef struct gwas_server gwas_server;

/* Parameters (the RNS reading of the scheme parameters of the paper's Methods,
 * "Homomorphic Encryption": ring dimension N, levels L, scale).  The prime
 * chain is derived from them by a fixed rule: q_0 is the largest prime below
 * 2^60 that is 1 mod 2N; the L rescale primes are chosen greedily from the 4L
 * primes 1 mod 2N nearest 2^log2_scale so that the canonical scales
 * Delta_{d+1} = Delta_d^2 / q_{L-d} stay near 2^log2_scale; the key-switching
 * modulus P = p_1 ... p_alpha is the product of the alpha largest primes below
 * 2^41 that are 1 mod 2N and not in the chain, alpha the digit-group size of the
 * hybrid key switch (see ckks_keygen). */
#define CKKS_DEFAULT_KS_ALPHA 3
typedef struct {
    int log_n;          /* log2 N, 10 <= log_n <= 17 */
    int levels;         /* L >= 1: number of rescale primes */
    int log2_scale;     /* base scale Delta_0 = 2^log2_scale, 20 <= . <= 50 */
    int ks_alpha;       /* digit-group size alpha of key switching, 2 <= . <= 8; 0: CKKS_DEFAULT_KS_ALPHA */
} ckks_params;

/* Device allocator callbacks (e.g. torch's caching allocator).  alloc returns
 * NULL on failure; user is passed back unchanged. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, size_t bytes, void *user);
    void *user;
} ckks_allocator;

const char *ckks_last_error(void);

/* Host only: the digit-group size alpha the parameters select (ks_alpha, or the default for 0),
 * or CKKS_E_INVALID_ARG when it is out of range. */
int ckks_params_ks_alpha(const ckks_params *params);
/* Host only (no device work): the moduli q_0..q_L, p_1..p_alpha (moduli: L + 1 + alpha entries)
 * and the canonical scales Delta_0..Delta_L (scales: L + 1 entries). */
int ckks_chain(const ckks_params *params, uint64_t *moduli, double *scales);

/* ---------------------------------------------------------------- context */

/* Build the prime chain and NTT tables and upload them.  allocator and
 * hip_stream may be NULL.  pool_budget_bytes caps the device memory the pool
 * may hold (0: no cap). */
int ckks_ctx_create(const ckks_params *params, const ckks_allocator *allocator, void *hip_stream,
                    size_t pool_budget_bytes, ckks_ctx **out);
void ckks_ctx_destroy(ckks_ctx *ctx);

/* Chain moduli: q[0..L] then p_1..p_alpha (caller array of L + 1 + alpha entries). */
int ckks_ctx_moduli(const ckks_ctx *ctx, uint64_t *moduli, int cap);
/* Canonical scales Delta_0..Delta_L (caller array of L + 1 entries). */
int ckks_ctx_scales(const ckks_ctx *ctx, double *scales, int cap);
/* Pool statistics: bytes in use, bytes cached, peak bytes, allocator calls (summed over the main pool and
 * the pool of the context's second compute stream, which the GWAS circuit uses when no budget is set). */
int ckks_ctx_pool_stats(const ckks_ctx *ctx, size_t *in_use, size_t *cached, size_t *peak, size_t *n_alloc);
/* Release cached pool slabs back to the allocator. */
int ckks_ctx_pool_trim(ckks_ctx *ctx);

/* ---------------------------------------------------------------- keys */

/* KeyGen (paper: Methods, "Homomorphic Encryption", KeyGen), RNS form with the
 * special modulus P = p_1 ... p_alpha and a hybrid decomposition into digit
 * groups of alpha primes: G_0 = {q_0 .. q_{alpha-2}},
 * G_b = {q_{alpha b - 1} .. q_{alpha b + alpha - 2}} (b = 1 .. floor((L+1)/alpha)).
 * s has h = min(64, N/2) coefficients in {-1, 1} (HWT(h)), pk = (-a s + e, a) mod Q_L,
 * and a switching key for s' has one part per group b:
 * (-a_b s + e_b + [q_t in G_b] P s', a_b) mod q_t (t = 0..L) and p_1..p_alpha.
 * A relinearisation key (s' = s^2) is always made; one Galois key is made per
 * element of galois[] (s' = s(X^g), g odd in [3, 2N)).  seed != 0 selects the
 * test-only deterministic generator (counter-based SplitMix64); seed == 0 draws
 * the seed from the OS.  Keys stay resident on the device. */
int ckks_keygen(ckks_ctx *ctx, uint64_t seed, const uint64_t *galois, int n_galois);
/* Galois element of a left rotation by r slots (slot j <- slot j + r), 5^r mod 2N; r may be negative. */
uint64_t ckks_galois_rotate(const ckks_ctx *ctx, int64_t r);
/* Galois element of complex conjugation, 2N - 1. */
uint64_t ckks_galois_conj(const ckks_ctx *ctx);
/* Copy out a key in canonical coefficient form.  key_id 0 is the relinearisation
 * key, otherwise a Galois element; buf holds [2][G][L+1+alpha][N] words,
 * G = 1 + floor((L+1)/alpha) groups, targets q_0..q_L then p_1..p_alpha.
 * Secret: [N] int64; public key: [2][L+1][N]. */
int ckks_export_switching_key(ckks_ctx *ctx, uint64_t key_id, uint64_t *buf, size_t cap_words);
/* CKKS_E_KEY_MISSING in a context that holds no secret (one that only imported keys). */
int ckks_export_secret(ckks_ctx *ctx, int64_t *buf, size_t cap);
int ckks_export_public_key(ckks_ctx *ctx, uint64_t *buf, size_t cap_words);

/* Client and server (paper: Introduction and Methods: the data owner encrypts and decrypts, the server
 * computes on ciphertexts only).  An evaluating context is created with ckks_ctx_create and never runs
 * ckks_keygen: it imports the public key and the switching keys the client exported (canonical
 * coefficient form, the layouts of the exports above: words = 2 (L+1) N for the public key and
 * 2 G (L+1+alpha) N for a switching key; every residue below its modulus, else CKKS_E_INVALID_ARG).  It
 * holds no secret: ckks_decrypt, ckks_decrypt_poly, gwas_finalize and ckks_export_secret return
 * CKKS_E_KEY_MISSING there, and encryption needs an imported public key.  Importing a key id that is
 * present replaces it.  The buffers stay the caller's. */
int ckks_import_public_key(ckks_ctx *ctx, const uint64_t *buf, size_t words);
int ckks_import_switching_key(ckks_ctx *ctx, uint64_t key_id, const uint64_t *buf, size_t words);
/* 1 when the context holds the secret (it ran ckks_keygen), else 0 (also for NULL). */
int ckks_ctx_has_secret(const ckks_ctx *ctx);

/* ---------------------------------------------------------------- encode / encrypt / decrypt */

/* Encode (paper: Methods, Encode): integer polynomial round(scale * sigma^-1(z)),
 * slot j <-> evaluation at zeta^(5^j mod 2N), zeta = exp(i pi / N).  re/im hold
 * n <= N/2 slots (the rest are 0; im may be NULL).  FP64 on the host. */
int ckks_encode(ckks_ctx *ctx, const double *re, const double *im, size_t n, double scale, int64_t *coeffs_out);
/* Decode of a real polynomial given as doubles (m_i / scale already applied). */
int ckks_decode(ckks_ctx *ctx, const double *coeffs, double *re, double *im);

/* Encrypt (paper: Encrypt): ct = v pk + (m + e0, e1) at depth `depth` with tracked
 * scale `scale`; m is an integer polynomial (N int64 coefficients).  v is
 * ternary, e0, e1 centred binomial (eta = 21); seed as for keygen. */
int ckks_encrypt(ckks_ctx *ctx, const int64_t *m, int depth, double scale, uint64_t seed, ckks_ct **out);
/* Decrypt (paper: Decrypt) ciphertext `index` of a batch: c0 + c1 s, centred over
 * q_0 q_1 (over q_0 when one limb is left), divided by the tracked scale and
 * decoded into N/2 slots (re, im: caller arrays of N/2 doubles; im may be NULL). */
int ckks_decrypt(ckks_ctx *ctx, const ckks_ct *ct, int index, double *re, double *im);
/* Decrypt to the centred integer polynomial c0 + c1 s (N doubles, not scaled). */
int ckks_decrypt_poly(ckks_ctx *ctx, const ckks_ct *ct, int index, double *coeffs);

/* ---------------------------------------------------------------- ciphertexts
 * A ckks_ct handle is a batch of `count` ciphertexts at one depth and scale,
 * stored [count][2][limbs][N] on the device; operations on two batches pair them
 * element-wise, and a smaller batch whose count divides the larger one's is read
 * cyclically (ciphertext i pairs with ciphertext i mod count; a batch of one
 * broadcasts); other count mismatches fail with CKKS_E_PARAM_MISMATCH. */

int ckks_ct_info(const ckks_ct *ct, int *count, int *depth, int *limbs, double *scale);
/* Canonical export of ciphertext `index` of the batch: [2][limbs][N] words. */
int ckks_ct_export(ckks_ctx *ctx, const ckks_ct *ct, int index, uint64_t *buf, size_t cap_words);
/* Import of a canonical ciphertext at `depth` (limbs = L + 1 - depth). */
int ckks_ct_import(ckks_ctx *ctx, const uint64_t *buf, int depth, double scale, ckks_ct **out);
void ckks_ct_free(ckks_ct *ct);

/* ---------------------------------------------------------------- evaluation (each a device operation) */

/* Add / Sub (paper: Add): operands at equal depth and tracked scale. */
int ckks_add(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);
int ckks_sub(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);
/* Multiply by a signed integer (no level consumed). */
int ckks_mul_int(ckks_ctx *ctx, const ckks_ct *a, int64_t k, ckks_ct **out);
/* Add the real constant c (the integer round_half_away(c * scale) in the constant coefficient). */
int ckks_add_const(ckks_ctx *ctx, const ckks_ct *a, double c, ckks_ct **out);
/* Mult (paper: Mult then Rescale): tensor (d0, d1, d2), relinearise d2 with the s^2
 * key and rescale by the last prime q = q_{l-1}, the two divisions (ModDown's by P,
 * the rescale's by q) taken as one division by P q: with x the key switch's inner
 * product over q_0..q_{l-1}, p_1..p_alpha and x' = x + P (d0, d1),
 *   out = (x' - C) / (P q) mod q_0..q_{l-2},  C = sum_b [x' (P q / b)^-1]_b (P q / b)
 * over b in {q, p_1..p_alpha} (the fast basis conversion: C is x' mod P q plus
 * e P q with 0 <= e <= alpha, so each coefficient of the result differs from
 * round(x' / (P q)) by an integer in [0, alpha + 1]).  Result scale (s_a * s_b) / q. */
int ckks_mul(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);
/* ckks_mul without any device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The product (the same kernels and the same bits as ckks_mul) is
 * written into `out`, a ciphertext batch of this context made earlier by the caller
 * (e.g. by ckks_ct_import) holding max(count_a, count_b) ciphertexts at depth
 * depth_a + 1; its data are overwritten and it takes the product's scale.  out may
 * not overlap a or b.  Every intermediate buffer comes from one static device
 * array of CKKS_NOALLOC_SCRATCH_BYTES per GPU, held from library load until the
 * process ends: a product whose buffers need more (about 2N (3l + K + ...) words
 * at l limbs) returns CKKS_E_INVALID_ARG before any work is enqueued.  Calls that
 * overlap on one GPU (other host threads, other contexts or streams) share that
 * array and race: the caller serialises them.  Nothing of the array needs to start
 * at zero.  Errors as ckks_mul, plus CKKS_E_PARAM_MISMATCH when out has another
 * count or depth. */
#define CKKS_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int ckks_mul_noalloc(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out);
/* Multiply by the real c encoded at a's scale s (integer round_half_away(c s)), then
 * rescale by q; result scale (s * s) / q. */
int ckks_mul_const(ckks_ctx *ctx, const ckks_ct *a, double c, ckks_ct **out);
/* Rescale (paper: Rescale): round(c / q_last) on the centred integer. */
int ckks_rescale(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
/* Align to a deeper depth and a target scale: mod-drop to depth - 1, multiply by
 * round_half_away(((scale * factor) * q) / s_a), rescale, declare `scale`. */
int ckks_align(ckks_ctx *ctx, const ckks_ct *a, int depth, double scale, double factor, ckks_ct **out);
/* Rotate (paper: Rotate) by r slots: slot j of the result holds slot j + r. */
int ckks_rotate(ckks_ctx *ctx, const ckks_ct *a, int64_t r, ckks_ct **out);
/* a + sum_i Rotate(a, rots[i]) for 1 <= n <= 16 rotations sharing one key switch: one decomposition of
 * c1 (each digit permuted by its rotation after the basis extension) and one division by P for the sum
 * (a grouped step of Alg. colSum).  Needs the Galois key of every rotation. */
int ckks_rotate_sum(ckks_ctx *ctx, const ckks_ct *a, const int64_t *rots, int n, ckks_ct **out);
/* Complex conjugation of every slot. */
int ckks_conjugate(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
/* Multiply by the block-start mask (1 at slots = 0 mod R) encoded at a's scale s,
 * then rescale; result scale (s * s) / q. */
int ckks_mul_mask(ckks_ctx *ctx, const ckks_ct *a, int R, ckks_ct **out);
/* Negacyclic NTT of `count` limbs in place on device memory laid out [count][N],
 * limb i modulo chain modulus moduli_index[i] (0..L, then L+1.. = p_1..p_alpha); forward (dir = 1)
 * to this library's evaluation order or inverse (dir = -1).  Host array of indices. */
int ckks_ntt_device(ckks_ctx *ctx, uint64_t *dev_limbs, int count, const int *moduli_index, int dir);

/* ---------------------------------------------------------------- GWAS (paper: Alg. Semi Parallel GWAS) */

/* Layout: R = PO2(n) rows per block, B = N / (2R) blocks, tau = N / R SNPs per
 * SNP-batch ciphertext (two per complex slot), ceil(m / tau) batches.
 * Circuit depth: L must be at least 7 kappa + 5 for kappa >= 2 Newton passes, and 8 for kappa = 1 (then
 * p = sigma7(0) = 1/2, w = 1/4 and w^-1 = inverseSlots(1/4) are public constants, as in the paper's
 * Discussion of the reduced kappa; there is no w or w^-1 ciphertext). */
int gwas_layout(const ckks_ctx *ctx, int n, int k, int m, int kappa, int *R, int *tau, int *n_batches,
                int *levels_needed);

/* Host only: the Galois elements whose keys the circuit needs for block size R at ring degree 2^log_n
 * (the rotations of the grouped rotate-and-sum in both directions, each once: the fixed part groups
 * them by up to 7 per key switch, {s, 2s, .., 7s}, the per-SNP-batch part by up to 15, {s, 2s, .., 15s};
 * then conjugation).  Writes at most cap elements to out and the number needed to *count. */
int gwas_galois_elements(int log_n, int R, uint64_t *out, int cap, int *count);

/* Client side: compute A = (X^T X)^-1 in FP64, encode and encrypt x_j (R-periodic,
 * depth 0), y (depth 0), A_jl for j <= l (replicated, depth 0, scale R Delta_0)
 * and the SNP batches (depth 7 kappa, or 4 for kappa = 1; complex-packed).  X is n x k row-major
 * with X[:,0] = 1; y in {0, 1}; S is n x m row-major uint8 in {0, 1, 2}.
 * Input ciphertext i is encrypted with seed output_i(SplitMix64(enc_seed)). */
int gwas_pack_encrypt(ckks_ctx *ctx, const double *X, const double *y, const uint8_t *S, int n, int k, int m,
                      int kappa, uint64_t enc_seed, gwas_enc_input **out);
/* Assemble an input from imported ciphertexts (x[k], y, A[k(k+1)/2] row-major
 * upper triangle, S[n_batches]); the handles are copied. */
int gwas_input_from_cts(ckks_ctx *ctx, int n, int k, int m, int kappa, ckks_ct *const *x, const ckks_ct *y,
                        ckks_ct *const *A, ckks_ct *const *S, int n_s, gwas_enc_input **out);
void gwas_input_free(gwas_enc_input *in);
/* Input ciphertexts, e.g. for export to a server: which = 0 x_j (index j), 1 y, 2 A (index in row-major
 * upper-triangle order), 3 the SNP batches (one batch handle, index 0; CKKS_E_INVALID_ARG once spilled).
 * The handle stays owned by the input. */
int gwas_input_ct(const gwas_enc_input *in, int which, int index, const ckks_ct **ct);

/* Server side (the hot path): the encrypted circuit.  Fails with CKKS_E_LEVEL or
 * CKKS_E_KEY_MISSING before any launch when the chain or keys do not fit.  The SNP
 * batches are processed `chunk` ciphertexts at a time (gwas_semiparallel: up to 64).
 * The projection S' = S - sum_j x_j E_j (E_j the block sums of r_j S over each block, r_j = (X A)_j)
 * packs the k covariates into one ciphertext when n + K - 1 <= R (K the smallest power of two >= k,
 * at most 16): D = sum_t Rot(Z_t, -t) Rot(S, -t) with the diagonals Z_t of the r_j, a stride-K
 * rotate-and-sum that leaves E_j's sum at slot j of each block, the mask of the first k slots, a
 * stride-K broadcast V and sum_t X_t Rot(V, t) with the diagonals X_t of the x_j; otherwise one
 * colSum, mask and broadcast per covariate.  The stride sums use the rotations of the per-batch
 * rotate-and-sum only (gwas_galois_elements). */
int gwas_semiparallel(ckks_ctx *ctx, const gwas_enc_input *in, gwas_enc_output **out);
int gwas_semiparallel_chunked(ckks_ctx *ctx, const gwas_enc_input *in, int chunk, gwas_enc_output **out);
/* Output ciphertexts: which = 0 num, 1 den_even, 2 den_odd, 3 S' (projected batches):
 * index = chunk number, each a batch of up to `chunk` ciphertexts in SNP-batch order;
 * 4 beta_j (index j), 5 w, 6 w^-1 (CKKS_E_INVALID_ARG for kappa = 1, where both are public), 7 z',
 * 8 u = w z', 9 b' and 10 err' after gwas_divide, 11 the n columns Dup(M_i) of the M-materialised layout
 * (at the SNP depth + 2).  The handle stays owned by out.  The denominators of the even and the odd SNPs
 * are the real parts of den_even and den_odd at the block starts; both come from one rotate-and-sum of
 * W = 4 w (a^2 + i b^2) (S' = a + i b per slot), den_even = sum W / 4 and den_odd = -i den_even (the
 * factor -i as the exact plaintext product with -X^(N/2)), so each carries the other's in its imaginary
 * part. */
int gwas_output_ct(const gwas_enc_output *out, int which, int index, const ckks_ct **ct);

/* ---- Autotuner.  gwas_tune times every candidate schedule of the circuit on `in` itself (SNP-batch chunks
 * of all batches up to 64, 32, 16 and 8, each with the logistic-regression part on a second stream and
 * on one stream, each with the covariates' per-batch products stacked up to 256 ciphertexts and not (see
 * ckks_ctx_set_stack); HIP events around whole calls, best of `reps` after one untimed call) and records
 * the fastest for in's shape (R, k, kappa, number of SNP batches) in the context.  Every candidate computes
 * the same operations on the same ciphertexts: outputs are bit-identical whichever is chosen.  Returns the
 * chosen chunk, stream count and stack size, its time, the default schedule's time (all batches, two
 * streams, no stack) and the number of candidates (any output pointer may be NULL).  With
 * ckks_ctx_use_tuned(ctx, 1), gwas_semiparallel runs a recorded schedule for inputs of a tuned shape. */
int gwas_tune(ckks_ctx *ctx, const gwas_enc_input *in, int reps, int *chunk, int *streams, double *ms,
              double *ms_default, int *candidates, int *stack);
int ckks_ctx_use_tuned(ckks_ctx *ctx, int enable);
/* Whether the circuit's outputs keep S' of every SNP batch (default 1).  With 0 the projected batches are
 * dropped once their numerator and denominators are formed (gwas_output_ct(.., 3, ..) then fails), which
 * saves their HBM (3 limbs per batch at kappa = 3) in large batched runs; nothing else changes. */
int gwas_keep_projected(ckks_ctx *ctx, int keep);

/* ---- HIP graph of the circuit (the batched form's replay path).  gwas_graph_create runs the circuit once
 * on a private copy of `in` (which also creates the second stream and fills the pools), then captures a
 * second call on the context's stream (which must not be the null stream) as a HIP graph and instantiates
 * it.  Every device buffer the call takes stays reserved for the graph until gwas_graph_destroy, so a
 * replay rewrites the same output while other work of the context goes on.  gwas_graph_set_input copies a
 * job of the same shape (n, k, m, kappa; device-resident) into the graph's input, on the context's stream;
 * gwas_graph_launch replays the graph on that stream (asynchronous: the output is complete once the stream
 * reaches that point); gwas_graph_output returns the output (owned by the graph, rewritten by every
 * replay, usable with gwas_output_ct and gwas_finalize).  chunk <= 0: as gwas_semiparallel.  Not with a
 * pool budget, kernel timing or a spilled input (CKKS_E_INVALID_ARG). */
typedef struct gwas_graph gwas_graph;
int gwas_graph_create(ckks_ctx *ctx, const gwas_enc_input *in, int chunk, gwas_graph **out);
int gwas_graph_set_input(gwas_graph *g, const gwas_enc_input *in);
int gwas_graph_launch(gwas_graph *g);
int gwas_graph_output(const gwas_graph *g, const gwas_enc_output **out);
void gwas_graph_destroy(gwas_graph *g);

/* ---- homomorphic division: b' and err' as ciphertexts (an extension; the paper decrypts num and den
 * separately and divides on the client, Methods, walk-through of Alg. Semi Parallel GWAS).  The chain must
 * hold gwas_div_levels() levels after the denominators' depth L_c (7 kappa + 5, or 8 for kappa = 1):
 * create the context with levels >= L_c + gwas_div_levels(); the circuit itself runs unchanged on the
 * longer chain. */
/* ---- M-materialised layout (paper: Alg. CP-REP-MatMult and the walk-through of Alg. Semi Parallel GWAS:
 * M = I - X (X^T X)^-1 X^T as a CP matrix, S' = M S_i by CP-REP-MatMult with S_i in REP form).  An input
 * with these REP parts attached runs the per-SNP-batch projection as
 *   S'_b = sum_{i < n} Dup(M_i) (.) S_rep(b, i)      (one lazy tensor sum, one relinearisation)
 * where Dup(M_i) = Dup(e_i) - sum_j r_j X_ij is column i of M duplicated over the ciphertext (r_j the
 * columns of X A brought to the REP X^T's depth, X_ij from the REP X^T, Dup(e_i) the exact indicator of the
 * slots = i mod R; the columns come out at the REP rows' depth), instead of
 * the rotation-based factorised projection; everything after S' is unchanged, and S' lands at the same
 * depth and scale.  One job at a time (gwas_semiparallel); n REP rows per SNP batch. */
/* Attach REP inputs made elsewhere: xrep[n k] sample-major (X_ij replicated over every slot, at the SNP
 * depth + 1 = 7 kappa + 1, or 5 for kappa = 1, and that depth's scale), srep[n_batches n] batch-major (row i of batch b, each complex-packed entry
 * S[i, b tau + 2c] + i S[i, b tau + 2c + 1] over its block of R slots, depth snp_depth + 2 = 7 kappa + 2,
 * or 6 for kappa = 1, scale Delta of that depth).  Handles are copied. */
int gwas_input_attach_m(ckks_ctx *ctx, gwas_enc_input *in, const ckks_ct *const *xrep, int n_xrep,
                        const ckks_ct *const *srep, int n_srep);
/* Client side: encode and encrypt those REP inputs from X (n x k row-major) and S (n x m row-major uint8)
 * and attach them; REP ciphertext i (X first, then S) is encrypted with seed
 * output_{2^21 + i}(SplitMix64(enc_seed)). */
int gwas_pack_encrypt_m(ckks_ctx *ctx, gwas_enc_input *in, const double *X, const uint8_t *S, uint64_t enc_seed);

/* Levels the division takes after the denominators: 3 + 2 (5 - 1) = 11 (5 Newton steps from guess 1). */
int gwas_div_levels(void);
/* Client side: the normalisers, 1 / d_j at the block start of SNP j with d_j = ||S_j - mean(S_j)||^2 / 4
 * (an upper bound of den_j since w <= 1/4 and S' = M S is the shortest residual of S_j after projecting
 * out X, whose first column is the intercept; 0 for a constant SNP), one ciphertext per SNP batch and
 * parity: a batch of 2 n_batches ciphertexts, the even SNPs of every batch, then the odd, at depth L_c and
 * scale Delta_{L_c} / (2 f), f = 4 (or 16 for kappa = 1) the factor of the denominators' tracked scale.
 * Ciphertext i is encrypted with seed output_{2^20 + i}(SplitMix64(enc_seed)).  S as in gwas_pack_encrypt. */
int gwas_pack_normalisers(ckks_ctx *ctx, const uint8_t *S, int n, int m, int kappa, uint64_t enc_seed,
                          ckks_ct **out);
/* Server side: x = Re(den) v (the real part (den + conj(den)) / 2, since a denominator carries the other
 * parity's denominator in its imaginary part), g_1 = 2 - x, then g <- g (2 - x g) four times (the pattern of
 * Alg. inverseSlots), err' = g v and b' = num err', per chunk of SNP batches, stored in `out` (which = 9
 * b', 10 err' of gwas_output_ct, index = chunk: 2 cnt ciphertexts, the even SNPs' then the odd SNPs'; b'
 * of an even SNP is the real part, of an odd SNP the imaginary part).  Needs the conjugation key.  The
 * relative error of the reciprocal is (1 - x)^32 with x = den_j / d_j in (0, 1]. */
int gwas_divide(ckks_ctx *ctx, gwas_enc_output *out, const ckks_ct *v);
/* Client side: decrypt the divided outputs: b', err' and se = sqrt(err') per SNP (no division). */
int gwas_finalize_divided(ckks_ctx *ctx, const gwas_enc_output *out, int m, double *b, double *err, double *se);
/* One batch holding the ciphertexts of parts[0..n) in order (equal depth and scale); handles are copied. */
int ckks_ct_stack(ckks_ctx *ctx, const ckks_ct *const *parts, int n, ckks_ct **out);
/* Client side: an output assembled from the server's num, den_even and den_odd ciphertexts (one per SNP
 * batch, n_batches of each, e.g. imported with ckks_ct_import), for gwas_finalize; the handles are copied. */
int gwas_output_from_cts(ckks_ctx *ctx, int n, int k, int m, ckks_ct *const *num, ckks_ct *const *den_even,
                         ckks_ct *const *den_odd, int n_batches, gwas_enc_output **out);
int gwas_output_batches(const gwas_enc_output *out, int *n_batches);
void gwas_output_free(gwas_enc_output *out);

/* Client side: decrypt num / den separately and divide (b' = num / den,
 * err' = 1 / den, se = sqrt(err')), m entries each; num and den may be NULL. */
int gwas_finalize(ckks_ctx *ctx, const gwas_enc_output *out, int m, double *b, double *err, double *se,
                  double *num, double *den);

/* Per-kernel timing with HIP events set by the runtime at the start and the end of
 * every launch of the instrumented kernels (hipExtLaunchKernelGGL), on the stream
 * each kernel is launched on.  enable = 1 clears the counters and starts
 * recording; 0 stops.  The report is text, one line per kernel:
 * "name launches total_ms algorithmic_bytes algorithmic_fp64_ops pass_bytes" (the name, a kernel symbol
 * such as "ntt_pass<false, true, 8, 0>", may contain spaces; the last five fields are numbers).
 * algorithmic_bytes count each distinct word a launch must read and each word it must write once; an NTT
 * is 16 N bytes per limb transform, its first pass credited with the reads and its second with the writes
 * (plus operands of a fused epilogue).  pass_bytes count what a pass moves when it reads and writes every
 * word once itself (the two-pass NTT's intermediate round trip included).  The FP64 operation count is 0
 * for kernels bound by memory rather than arithmetic.
 * While two streams run at once a kernel's interval includes waiting for workgroup
 * slots held by the other stream's kernels (see ckks_ctx_set_streams). */
int ckks_ctx_kernel_timing(ckks_ctx *ctx, int enable);
/* Restrict recording to launches of one kernel name (as it appears in the report), so that timing a
 * single kernel adds two event records per launch of that kernel only; NULL or "" records all kernels.
 * The name "keyswitch" records whole key switches instead (events on the stream before the first and
 * after the last kernel of each key switch; algorithmic bytes 8 N [count l (input) + keys 2 G (l + alpha)
 * (key words of the G digit groups below l, read once per call) + count 4 l (two outputs read and
 * written)]); it is meaningful with one compute stream (ckks_ctx_set_streams(ctx, 1)). */
int ckks_ctx_kernel_timing_only(ckks_ctx *ctx, const char *name);
int ckks_ctx_kernel_report(ckks_ctx *ctx, char *buf, size_t cap);
/* Number of compute streams the GWAS circuit may use: 2 (the default) runs the
 * logistic-regression part on a second stream concurrently with the per-batch work
 * that does not depend on it; 1 runs everything in order on the context's stream.
 * Results are identical either way. */
int ckks_ctx_set_streams(ckks_ctx *ctx, int n);
/* The per-batch part of the GWAS circuit stacks the products r_j S of its k
 * covariates into one batch (one set of launches for all of them) while the
 * stack holds at most n ciphertexts (0, the default: one covariate at a time).
 * Results are identical either way. */
int ckks_ctx_set_stack(ckks_ctx *ctx, int n);

/* ---------------------------------------------------------------- batched and serving forms
 * (additions of this library around the paper's algorithm; the arithmetic of each job is unchanged) */

/* Several jobs in one call.  Jobs with the same block size R, covariate count k and kappa share every
 * launch of the fixed part (one batch ciphertext per job) and their SNP batches run through the
 * per-batch part together, `chunk` ciphertexts per launch, each with its own job's values.  A job with
 * at least chunk / 2 SNP batches, or with the M-materialised layout, runs alone, max(chunk, 256) SNP
 * batches per pass when resident and no pool budget is set (every job's outputs stay resident until the
 * call returns, so the passes' transient buffers are bounded), else `chunk` at a time.
 * out[i] receives job i's output (bucketed jobs: one batch per output kind, index 0).  Results are
 * bit-identical to running each job alone. */
int gwas_semiparallel_multi(ckks_ctx *ctx, const gwas_enc_input *const *in, int n_jobs, int chunk,
                            gwas_enc_output **out);
/* Device bytes a job needs while in flight (inputs, outputs and working values). */
int gwas_input_footprint(const gwas_enc_input *in, size_t *bytes);
/* Move a job's SNP batches to pinned host memory; they are then copied back chunk by chunk, the next
 * chunk's copy overlapping the current chunk's compute (the stand-in for the paper's cache module,
 * Methods: "Smart Cache Module"). */
int gwas_input_spill(ckks_ctx *ctx, gwas_enc_input *in);

/* Serving: a worker thread owns the context's device work.  Submitted jobs are admitted in arrival
 * order while the sum of their footprints fits hbm_budget_bytes (0: no cap) and at most
 * max_jobs_in_flight are active; a job larger than the whole budget has its SNP batches spilled to the
 * host.  Each iteration runs the fixed parts of newly admitted jobs together, then one chunk of SNP
 * batches drawn from all active jobs of one shape (continuous batching).  Calls on the same context
 * from other threads are serialised with the worker. */
int gwas_server_create(ckks_ctx *ctx, size_t hbm_budget_bytes, int max_jobs_in_flight, int chunk,
                       gwas_server **out);
/* Ownership of `in` passes to the server when the call succeeds; when it fails the input is unchanged and
 * still the caller's. */
int gwas_server_submit(gwas_server *s, gwas_enc_input *in, uint64_t *job_id);
/* CKKS_OK with *out set (ownership passes to the caller) when the job is done; CKKS_E_NOT_READY when
 * it is not (wait = 0) ; wait = 1 blocks until it is done; CKKS_E_CANCELLED for a cancelled job. */
int gwas_server_poll(gwas_server *s, uint64_t job_id, int wait, gwas_enc_output **out);
/* Cancel a queued, admitted or running job (a finished job is left as it is).  Its device memory and its
 * share of the budget are released by the worker as soon as no launch in flight reads them; polling it
 * then returns CKKS_E_CANCELLED. */
int gwas_server_cancel(gwas_server *s, uint64_t job_id);
/* Latency percentiles (completion - submission) over completed jobs, completed jobs per second
 * (first submission to last completion), and the largest number of jobs in flight together. */
int gwas_server_stats(gwas_server *s, double *p50_ms, double *p99_ms, double *jobs_per_s, uint64_t *completed,
                      int *peak_jobs_in_flight);
void gwas_server_destroy(gwas_server *s);

/* Number of key switches and NTT limb transforms issued by the context so far. */
int ckks_ctx_counters(const ckks_ctx *ctx, uint64_t *keyswitches, uint64_t *limb_ntts, uint64_t *launches);
/* Key switches counted per ciphertext since creation: a key switch over a batch of count ciphertexts adds
 * count (ckks_ctx_counters counts it once).  Equals the number of single-ciphertext key switches a
 * ciphertext-at-a-time evaluator makes for the same work. */
int ckks_ctx_keyswitch_ciphertexts(const ckks_ctx *ctx, uint64_t *n);

#ifdef __cplusplus
}
#endif
#endif /* GWAS_CKKS_H */
