/*
 * CPU reference RNS-CKKS — TEST INFRASTRUCTURE ONLY.
 *
 * This file is part of the oracle: a plain, slow, obviously correct CPU
 * implementation used only by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark.  The product (the HIP library) never links or calls it,
 * and it shares no code, header or table with the product.
 *
 * Every operation works on polynomials in COEFFICIENT form, residues in
 * [0, q) for each RNS modulus, laid out [poly][limb][coeff].  A negacyclic
 * polynomial product mod (X^N + 1, q) is computed by the textbook route:
 * twist by psi^i (psi a primitive 2N-th root of unity), cyclic NTT of length N
 * with omega = psi^2 (iterative radix-2 with an explicit bit-reversal
 * permutation), pointwise product, inverse cyclic NTT, untwist and scale by
 * N^-1.  That route is only an accelerator for the schoolbook product, and the
 * tests pin it against schoolbook convolution.  Modular products use
 * (unsigned __int128) a * b % q.
 *
 * The CKKS operations follow the scheme description of the paper (Methods,
 * "Homomorphic Encryption": KeyGen, Encrypt, Decrypt, Add, Mult, Rescale, and
 * Rotate) in its residue-number-system form with a special modulus
 * P = p_1 ... p_alpha and a hybrid decomposition into digit groups of alpha
 * primes, {q_0 .. q_{alpha-2}}, then {q_{alpha-1} .. q_{2 alpha-2}}, ...:
 *   - key switching of d with a key for s': the digits D_b of d (fast basis
 *     conversion of d modulo the group's primes), x = sum_b D_b * ksk_b and
 *     (x - C) / P, C the fast conversion of x mod P (see ref_keyswitch), where
 *     ksk_b = (-a_b s + e_b + [q_t in group b] P s', a_b) modulo each q_t and p_k;
 *   - rescale by the last prime q_l:  round(c / q_l)  on the centred integer;
 *   - automorphism X -> X^g as the signed coefficient permutation i -> i*g mod 2N.
 *
 * Test-only randomness: a counter-based SplitMix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).  The i-th
 * output (i >= 0) of the generator seeded with state x is mix(x + (i+1)*gamma).
 * A stream `sid` of master seed `seed` is the generator seeded with output
 * number `sid` of the generator seeded with `seed`.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* modular arithmetic                                                   */
/* ------------------------------------------------------------------ */

static inline u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static inline u64 addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static inline u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

static u64 powmod(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime q by Fermat */
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }

/* signed integer -> residue in [0, q) */
static inline u64 from_signed(i64 v, u64 q) {
    if (v >= 0) return (u64)v % q;
    u64 m = (u64)(-(v + 1)) % q; /* -(v+1) >= 0, avoids overflow at INT64_MIN */
    return q - 1 - m;
}

/* ------------------------------------------------------------------ */
/* SplitMix64, counter based                                            */
/* ------------------------------------------------------------------ */

static const u64 SM_GAMMA = 0x9E3779B97F4A7C15ULL;

static inline u64 sm_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* i-th output of SplitMix64 seeded with state x */
u64 ref_splitmix_out(u64 x, u64 i) { return sm_mix(x + (i + 1) * SM_GAMMA); }

u64 ref_word(u64 seed, u64 sid, u64 ctr) {
    return ref_splitmix_out(ref_splitmix_out(seed, sid), ctr);
}

/* uniform ternary coefficient in {-1, 0, 1} */
void ref_sample_ternary(u64 seed, u64 sid, int n, i64 *out) {
    u64 st = ref_splitmix_out(seed, sid);
    for (int i = 0; i < n; ++i) out[i] = (i64)(ref_splitmix_out(st, (u64)i) % 3) - 1;
}

/*
 * Secret with exactly h nonzero coefficients in {-1, 1} (the HWT(h) distribution of KeyGen):
 * draw words w_c for c = 0, 1, 2, ...; position w_c mod N, sign -1 when the top bit of w_c is set;
 * a position already taken is skipped; stop after h positions.
 */
void ref_sample_hwt(u64 seed, u64 sid, int n, int h, i64 *out) {
    u64 st = ref_splitmix_out(seed, sid);
    for (int i = 0; i < n; ++i) out[i] = 0;
    if (h > n) h = n;
    int got = 0;
    for (u64 c = 0; got < h; ++c) {
        u64 w = ref_splitmix_out(st, c);
        int pos = (int)(w % (u64)n);
        if (out[pos] != 0) continue;
        out[pos] = (w >> 63) ? -1 : 1;
        ++got;
    }
}

/* centred binomial with eta = 21: popcount of 21 bits minus popcount of the next 21 */
void ref_sample_cbd(u64 seed, u64 sid, int n, i64 *out) {
    u64 st = ref_splitmix_out(seed, sid);
    for (int i = 0; i < n; ++i) {
        u64 w = ref_splitmix_out(st, (u64)i);
        out[i] = (i64)__builtin_popcountll(w & 0x1FFFFFULL) - (i64)__builtin_popcountll((w >> 21) & 0x1FFFFFULL);
    }
}

/* uniform residue mod q for modulus index mi: (w1 * 2^64 + w2) mod q */
void ref_sample_uniform(u64 seed, u64 sid, int mi, u64 q, int n, u64 *out) {
    u64 st = ref_splitmix_out(seed, sid);
    for (int i = 0; i < n; ++i) {
        u64 c = 2ULL * ((u64)mi * (u64)n + (u64)i);
        u64 w1 = ref_splitmix_out(st, c), w2 = ref_splitmix_out(st, c + 1);
        out[i] = (u64)((((u128)w1) << 64 | w2) % q);
    }
}

/* ------------------------------------------------------------------ */
/* context: moduli and cyclic-NTT tables                                */
/* ------------------------------------------------------------------ */

typedef struct {
    u64 q;
    u64 psi;        /* primitive 2N-th root of unity mod q */
    u64 n_inv;      /* N^-1 mod q */
    u64 *psi_pow;   /* psi^i, i < N */
    u64 *psi_ipow;  /* psi^-i, i < N */
    u64 *w_pow;     /* omega^i, i < N/2, omega = psi^2 */
    u64 *w_ipow;    /* omega^-i, i < N/2 */
} ref_mod;

typedef struct {
    int n, logn, nmod;  /* nmod = number of moduli in the table (q_0..q_L, P) */
    int *brev;
    ref_mod *mods;
} ref_ctx;

static int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

ref_ctx *ref_ctx_new(int n, int nmod, const u64 *qs, const u64 *psis) {
    ref_ctx *c = (ref_ctx *)calloc(1, sizeof(ref_ctx));
    c->n = n;
    c->logn = ilog2(n);
    c->nmod = nmod;
    c->brev = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) {
        int r = 0;
        for (int b = 0; b < c->logn; ++b) if (i & (1 << b)) r |= 1 << (c->logn - 1 - b);
        c->brev[i] = r;
    }
    c->mods = (ref_mod *)calloc(nmod, sizeof(ref_mod));
    for (int m = 0; m < nmod; ++m) {
        ref_mod *M = &c->mods[m];
        M->q = qs[m];
        M->psi = psis[m];
        M->n_inv = invmod((u64)n % M->q, M->q);
        M->psi_pow = (u64 *)malloc(sizeof(u64) * n);
        M->psi_ipow = (u64 *)malloc(sizeof(u64) * n);
        M->w_pow = (u64 *)malloc(sizeof(u64) * n);
        M->w_ipow = (u64 *)malloc(sizeof(u64) * n);
        u64 psi_inv = invmod(M->psi, M->q);
        u64 w = mulmod(M->psi, M->psi, M->q), wi = mulmod(psi_inv, psi_inv, M->q);
        u64 a = 1, b = 1, x = 1, y = 1;
        for (int i = 0; i < n; ++i) {
            M->psi_pow[i] = a; M->psi_ipow[i] = b;
            M->w_pow[i] = x; M->w_ipow[i] = y;
            a = mulmod(a, M->psi, M->q); b = mulmod(b, psi_inv, M->q);
            x = mulmod(x, w, M->q); y = mulmod(y, wi, M->q);
        }
    }
    return c;
}

void ref_ctx_free(ref_ctx *c) {
    if (!c) return;
    for (int m = 0; m < c->nmod; ++m) {
        free(c->mods[m].psi_pow); free(c->mods[m].psi_ipow);
        free(c->mods[m].w_pow); free(c->mods[m].w_ipow);
    }
    free(c->mods); free(c->brev); free(c);
}

/* cyclic NTT of length N in natural order: A_k = sum_i a_i w^(ik) (inverse: w^-1, no scaling) */
static void cyclic_ntt(const ref_ctx *c, const ref_mod *M, u64 *a, int inverse) {
    int n = c->n;
    for (int i = 0; i < n; ++i) {
        int r = c->brev[i];
        if (i < r) { u64 t = a[i]; a[i] = a[r]; a[r] = t; }
    }
    const u64 *tw = inverse ? M->w_ipow : M->w_pow;
    u64 q = M->q;
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1, step = n / len;
        for (int s = 0; s < n; s += len) {
            for (int j = 0; j < half; ++j) {
                u64 u = a[s + j];
                u64 v = mulmod(a[s + j + half], tw[j * step], q);
                a[s + j] = addmod(u, v, q);
                a[s + j + half] = submod(u, v, q);
            }
        }
    }
}

/* evaluation form used inside the oracle: a_i psi^i then cyclic NTT */
void ref_to_eval(const ref_ctx *c, int mi, const u64 *in, u64 *out) {
    const ref_mod *M = &c->mods[mi];
    for (int i = 0; i < c->n; ++i) out[i] = mulmod(in[i], M->psi_pow[i], M->q);
    cyclic_ntt(c, M, out, 0);
}

void ref_from_eval(const ref_ctx *c, int mi, const u64 *in, u64 *out) {
    const ref_mod *M = &c->mods[mi];
    if (out != in) memcpy(out, in, sizeof(u64) * c->n);
    cyclic_ntt(c, M, out, 1);
    for (int i = 0; i < c->n; ++i)
        out[i] = mulmod(mulmod(out[i], M->n_inv, M->q), M->psi_ipow[i], M->q);
}

/* negacyclic product mod (X^N + 1, q_mi) of coefficient-form polynomials */
void ref_polymul(const ref_ctx *c, int mi, const u64 *a, const u64 *b, u64 *out) {
    int n = c->n;
    u64 q = c->mods[mi].q;
    u64 *fa = (u64 *)malloc(sizeof(u64) * n), *fb = (u64 *)malloc(sizeof(u64) * n);
    ref_to_eval(c, mi, a, fa);
    ref_to_eval(c, mi, b, fb);
    for (int i = 0; i < n; ++i) fa[i] = mulmod(fa[i], fb[i], q);
    ref_from_eval(c, mi, fa, out);
    free(fa); free(fb);
}

/* ------------------------------------------------------------------ */
/* ciphertext-level operations (coefficient form, [2][l][N])            */
/* moduli of limb i are c->mods[i]                                      */
/* ------------------------------------------------------------------ */

/* out = a + b (count polys of l limbs) */
void ref_add(const ref_ctx *c, int npoly, int l, const u64 *a, const u64 *b, u64 *out) {
    int n = c->n;
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            size_t o = ((size_t)p * l + i) * n;
            for (int k = 0; k < n; ++k) out[o + k] = addmod(a[o + k], b[o + k], q);
        }
}

void ref_sub(const ref_ctx *c, int npoly, int l, const u64 *a, const u64 *b, u64 *out) {
    int n = c->n;
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            size_t o = ((size_t)p * l + i) * n;
            for (int k = 0; k < n; ++k) out[o + k] = submod(a[o + k], b[o + k], q);
        }
}

/* out = k * a for a signed integer k */
void ref_mul_int(const ref_ctx *c, int npoly, int l, const u64 *a, i64 k, u64 *out) {
    int n = c->n;
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q, kk = from_signed(k, q);
            size_t o = ((size_t)p * l + i) * n;
            for (int t = 0; t < n; ++t) out[o + t] = mulmod(a[o + t], kk, q);
        }
}

/* add the signed integer v to coefficient 0 of poly 0 (adds a constant message) */
void ref_add_const(const ref_ctx *c, int l, u64 *ct, i64 v) {
    int n = c->n;
    for (int i = 0; i < l; ++i) {
        u64 q = c->mods[i].q;
        ct[(size_t)i * n] = addmod(ct[(size_t)i * n], from_signed(v, q), q);
    }
}

/* out[l][N] = sum over the product a*pt where pt is an integer polynomial (signed coefficients) */
void ref_mul_plain(const ref_ctx *c, int npoly, int l, const u64 *a, const i64 *pt, u64 *out) {
    int n = c->n;
    u64 *tmp = (u64 *)malloc(sizeof(u64) * n);
    for (int i = 0; i < l; ++i) {
        u64 q = c->mods[i].q;
        for (int t = 0; t < n; ++t) tmp[t] = from_signed(pt[t], q);
        for (int p = 0; p < npoly; ++p) {
            size_t o = ((size_t)p * l + i) * n;
            ref_polymul(c, i, a + o, tmp, out + o);
        }
    }
    free(tmp);
}

/*
 * Tensor product of two ciphertexts (Mult, first step):
 *   d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1   mod each q_i.
 * `acc` != 0 adds into out (lazy sums of several products before one relinearisation).
 */
void ref_tensor(const ref_ctx *c, int l, const u64 *a, const u64 *b, u64 *out, int acc) {
    int n = c->n;
#pragma omp parallel
    {
        u64 *fa0 = (u64 *)malloc(sizeof(u64) * n), *fa1 = (u64 *)malloc(sizeof(u64) * n);
        u64 *fb0 = (u64 *)malloc(sizeof(u64) * n), *fb1 = (u64 *)malloc(sizeof(u64) * n);
        u64 *t = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for schedule(dynamic)
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            size_t n0 = (size_t)i * n, n1 = ((size_t)l + i) * n;
            ref_to_eval(c, i, a + n0, fa0); ref_to_eval(c, i, a + n1, fa1);
            ref_to_eval(c, i, b + n0, fb0); ref_to_eval(c, i, b + n1, fb1);
            u64 *d0 = out + (size_t)i * n, *d1 = out + ((size_t)l + i) * n, *d2 = out + ((size_t)2 * l + i) * n;
            for (int k = 0; k < n; ++k) t[k] = mulmod(fa0[k], fb0[k], q);
            ref_from_eval(c, i, t, t);
            for (int k = 0; k < n; ++k) d0[k] = acc ? addmod(d0[k], t[k], q) : t[k];
            for (int k = 0; k < n; ++k) t[k] = addmod(mulmod(fa0[k], fb1[k], q), mulmod(fa1[k], fb0[k], q), q);
            ref_from_eval(c, i, t, t);
            for (int k = 0; k < n; ++k) d1[k] = acc ? addmod(d1[k], t[k], q) : t[k];
            for (int k = 0; k < n; ++k) t[k] = mulmod(fa1[k], fb1[k], q);
            ref_from_eval(c, i, t, t);
            for (int k = 0; k < n; ++k) d2[k] = acc ? addmod(d2[k], t[k], q) : t[k];
        }
        free(fa0); free(fa1); free(fb0); free(fb1); free(t);
    }
}

/* centred representative of x mod q (x in [0, q)), reduced mod q2 */
static inline u64 centred_to(u64 x, u64 q, u64 q2) {
    if (x > q / 2) {
        /* x - q is negative: (x - q) mod q2 */
        u64 a = x % q2, b = q % q2;
        return submod(a, b, q2);
    }
    return x % q2;
}

/*
 * Rescale (drop the last limb q_{l-1}):  c' = round(c / q_{l-1}) on the centred integer.
 * Per limb i < l-1:  (c_i - [c_{l-1}]_centred mod q_i) * q_{l-1}^-1 mod q_i.
 * in: [npoly][l][N], out: [npoly][l-1][N].
 */
void ref_rescale(const ref_ctx *c, int npoly, int l, const u64 *in, u64 *out) {
    int n = c->n;
    u64 ql = c->mods[l - 1].q;
    for (int p = 0; p < npoly; ++p) {
        const u64 *last = in + ((size_t)p * l + (l - 1)) * n;
        for (int i = 0; i < l - 1; ++i) {
            u64 q = c->mods[i].q, inv = invmod(ql % q, q);
            const u64 *ci = in + ((size_t)p * l + i) * n;
            u64 *o = out + ((size_t)p * (l - 1) + i) * n;
            for (int k = 0; k < n; ++k) o[k] = mulmod(submod(ci[k], centred_to(last[k], ql, q), q), inv, q);
        }
    }
}

/*
 * Automorphism X -> X^g (g odd): coefficient i moves to i*g mod 2N, negated when that index is >= N.
 */
void ref_automorph(const ref_ctx *c, int npoly, int l, const u64 *in, u64 g, u64 *out) {
    int n = c->n;
    u64 twon = 2ULL * (u64)n;
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            const u64 *a = in + ((size_t)p * l + i) * n;
            u64 *o = out + ((size_t)p * l + i) * n;
            for (int k = 0; k < n; ++k) {
                u64 e = ((u64)k * g) % twon;
                if (e < (u64)n) o[e] = a[k];
                else o[e - n] = a[k] ? q - a[k] : 0;
            }
        }
}

/*
 * Digit groups of the key switch (hybrid decomposition with group size alpha >= 2): group 0 is
 * {q_0 .. q_{alpha-2}}, group b >= 1 is {q_{alpha b - 1} .. q_{alpha b + alpha - 2}}; a ciphertext with
 * l limbs uses the groups with a member below l, each restricted to its members below l.  Special
 * primes: modulus indices L+1 .. L+alpha, P = p_1 ... p_alpha.
 */
static int grp_first(int b, int a) { return b == 0 ? 0 : a * b - 1; }
static int grp_size(int b, int l, int a) {
    int f = grp_first(b, a), e = a * (b + 1) - 1;   /* members [f, e) */
    if (e > l) e = l;
    return e > f ? e - f : 0;
}
int ref_num_groups(int l, int a) { return 1 + l / a; }   /* groups with a member below l */

/*
 * Key switching of the polynomial d (coefficient form, limbs 0..l-1) with one or
 * several keys, each given in the oracle's evaluation form: kevs[i][comp][b][t][N]
 * for the ng groups b and the nt = L + 1 + alpha targets t (q_0..q_L, p_1..p_alpha).
 *
 * Digits: for group b with members G (below l), Q_G = prod q_i, y_i = [d_i (Q_G/q_i)^-1]_{q_i},
 * and the digit is the integer D_b = sum_{i in G} y_i (Q_G/q_i) (fast basis conversion: D_b = d mod
 * Q_G up to a multiple of Q_G, which the keys' gadget annihilates).  Key i is paired with the
 * automorphism X -> X^galois[i] of the digits (galois[i] == 0: none), applied after the digit has been
 * taken modulo the target; the products of all keys are summed, then divided by P once:
 *   x = sum_i sum_b sigma_i(D_b) ksk_{i,b}  mod (q_0..q_{l-1}, p_1..p_alpha),
 *   out = (x - C) / P mod q_0..q_{l-1},  C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k)  (C = x mod P up to a
 *   multiple of P, so the division is exact).
 */
static void automorph_poly(int n, u64 q, const u64 *a, u64 g, u64 *o) {
    u64 twon = 2ULL * (u64)n;
    for (int k = 0; k < n; ++k) {
        u64 e = ((u64)k * g) % twon;
        if (e < (u64)n) o[e] = a[k];
        else o[e - n] = a[k] ? q - a[k] : 0;
    }
}

/* x = sum_i sum_b sigma_i(D_b) ksk_{i,b} in coefficient form, [2][l + alpha][N] (targets q_0..q_{l-1},
 * p_1..p_alpha); the caller frees it */
static u64 *ks_accumulate(const ref_ctx *c, int L, int alpha, int l, const u64 *d, int n_keys, const u64 *galois,
                          const u64 *const *kevs, int ng) {
    int n = c->n, nt = L + 1 + alpha, gl = ref_num_groups(l, alpha), lt = l + alpha;
    size_t kstride_t = (size_t)n, kstride_b = (size_t)nt * n, kstride_c = (size_t)ng * nt * n;
    /* y_i of every limb: d_i times (Q_G / q_i)^-1 modulo q_i */
    u64 *y = (u64 *)malloc(sizeof(u64) * (size_t)l * n);
    for (int b = 0; b < gl; ++b) {
        int f = grp_first(b, alpha), m = grp_size(b, l, alpha);
        for (int i = f; i < f + m; ++i) {
            u64 qi = c->mods[i].q, hat = 1;
            for (int j = f; j < f + m; ++j) if (j != i) hat = mulmod(hat, c->mods[j].q % qi, qi);
            u64 hinv = invmod(hat, qi);
            for (int k = 0; k < n; ++k) y[(size_t)i * n + k] = mulmod(d[(size_t)i * n + k], hinv, qi);
        }
    }
    /* accumulate, per target modulus, both components in evaluation form */
    u64 *acc = (u64 *)calloc((size_t)2 * lt * n, sizeof(u64));
#pragma omp parallel
    {
        u64 *dig = (u64 *)malloc(sizeof(u64) * n), *sg = (u64 *)malloc(sizeof(u64) * n),
            *fe = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for schedule(dynamic)
        for (int ti = 0; ti < lt; ++ti) {
            int mi = ti < l ? ti : L + 1 + (ti - l);   /* modulus (and key target) of this target */
            u64 q = c->mods[mi].q;
            u64 *a0 = acc + (size_t)ti * n, *a1 = acc + ((size_t)lt + ti) * n;
            for (int b = 0; b < gl; ++b) {
                int f = grp_first(b, alpha), m = grp_size(b, l, alpha);
                /* D_b mod q: sum_i y_i (Q_G / q_i) */
                for (int k = 0; k < n; ++k) dig[k] = 0;
                for (int i = f; i < f + m; ++i) {
                    u64 hat = 1;
                    for (int j = f; j < f + m; ++j) if (j != i) hat = mulmod(hat, c->mods[j].q % q, q);
                    for (int k = 0; k < n; ++k) dig[k] = addmod(dig[k], mulmod(y[(size_t)i * n + k] % q, hat, q), q);
                }
                for (int i = 0; i < n_keys; ++i) {
                    if (galois[i]) {
                        automorph_poly(n, q, dig, galois[i], sg);
                        ref_to_eval(c, mi, sg, fe);
                    } else {
                        ref_to_eval(c, mi, dig, fe);
                    }
                    const u64 *k0 = kevs[i] + 0 * kstride_c + b * kstride_b + mi * kstride_t;
                    const u64 *k1 = kevs[i] + 1 * kstride_c + b * kstride_b + mi * kstride_t;
                    for (int k = 0; k < n; ++k) {
                        a0[k] = addmod(a0[k], mulmod(fe[k], k0[k], q), q);
                        a1[k] = addmod(a1[k], mulmod(fe[k], k1[k], q), q);
                    }
                }
            }
            ref_from_eval(c, mi, a0, a0);
            ref_from_eval(c, mi, a1, a1);
        }
        free(dig); free(sg); free(fe);
    }
    free(y);
    return acc;
}

void ref_keyswitch(const ref_ctx *c, int L, int alpha, int l, const u64 *d, int n_keys, const u64 *galois,
                   const u64 *const *kevs, int ng, u64 *out) {
    int n = c->n, lt = l + alpha;
    u64 *acc = ks_accumulate(c, L, alpha, l, d, n_keys, galois, kevs, ng);
    /* ModDown: (x - C) / P with C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k), each [.]_{p_k} the centred
       representative in (-p_k/2, p_k/2) */
    u64 pk[64], hinv[64];   /* alpha <= 8 */
    for (int k = 0; k < alpha; ++k) pk[k] = c->mods[L + 1 + k].q;
    for (int k = 0; k < alpha; ++k) {   /* (P/p_k)^-1 mod p_k */
        u64 hat = 1;
        for (int j = 0; j < alpha; ++j) if (j != k) hat = mulmod(hat, pk[j] % pk[k], pk[k]);
        hinv[k] = invmod(hat, pk[k]);
    }
    for (int comp = 0; comp < 2; ++comp) {
        const u64 *xs = acc + ((size_t)comp * lt + l) * n;   /* x mod p_1 .. p_alpha */
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q, pm = 1, hq[64];
            for (int k = 0; k < alpha; ++k) {
                pm = mulmod(pm, pk[k] % q, q);
                hq[k] = 1;   /* (P/p_k) mod q */
                for (int j = 0; j < alpha; ++j) if (j != k) hq[k] = mulmod(hq[k], pk[j] % q, q);
            }
            u64 pinv = invmod(pm, q);
            const u64 *xi = acc + ((size_t)comp * lt + i) * n;
            u64 *o = out + ((size_t)comp * l + i) * n;
            for (int k = 0; k < n; ++k) {
                u64 cv = 0;
                for (int j = 0; j < alpha; ++j) {
                    u64 yk = mulmod(xs[(size_t)j * n + k], hinv[j], pk[j]);
                    u64 ykq = yk > pk[j] / 2 ? submod(yk % q, pk[j] % q, q) : yk % q;   /* yk - p_k */
                    cv = addmod(cv, mulmod(ykq, hq[j], q), q);
                }
                o[k] = mulmod(submod(xi[k], cv, q), pinv, q);
            }
        }
    }
    free(acc);
}

/*
 * Key switch of d followed by the rescale of (add + KS(d)) by q_{l-1}, in one division by B = P q_{l-1}:
 *   x' = x + P add   (x as in ref_keyswitch; add = [2][l][N] coefficient form, e.g. d0, d1 of a product)
 *   out = (x' - C) / B mod q_0..q_{l-2},  C = sum_{b in {p_1..p_alpha, q_{l-1}}} [x' (B/b)^-1]_b (B/b),
 * each [.]_b the centred representative in (-b/2, b/2); an exact division since C = x' mod B up to a
 * multiple of B.  out: [2][l-1][N].
 */
void ref_keyswitch_rescale(const ref_ctx *c, int L, int alpha, int l, const u64 *d, int n_keys, const u64 *galois,
                           const u64 *const *kevs, int ng, const u64 *add, u64 *out) {
    int n = c->n, lt = l + alpha, nb = alpha + 1;
    u64 *acc = ks_accumulate(c, L, alpha, l, d, n_keys, galois, kevs, ng);
    u64 bm[16];   /* the moduli of B: p_1 .. p_alpha, q_{l-1} */
    for (int k = 0; k < alpha; ++k) bm[k] = c->mods[L + 1 + k].q;
    bm[alpha] = c->mods[l - 1].q;
    u64 hinv[16];   /* (B/b)^-1 mod b */
    for (int k = 0; k < nb; ++k) {
        u64 hat = 1;
        for (int j = 0; j < nb; ++j) if (j != k) hat = mulmod(hat, bm[j] % bm[k], bm[k]);
        hinv[k] = invmod(hat, bm[k]);
    }
    u64 *yb = (u64 *)malloc(sizeof(u64) * (size_t)nb * n);
    for (int comp = 0; comp < 2; ++comp) {
        /* y_b = [x' (B/b)^-1]_b for the moduli of B: x' = x on the special primes, x + P add on q_{l-1} */
        for (int k = 0; k < nb; ++k) {
            const u64 *xs = k < alpha ? acc + ((size_t)comp * lt + l + k) * n : acc + ((size_t)comp * lt + l - 1) * n;
            u64 qb = bm[k], pm = 1;
            if (k == alpha)
                for (int j = 0; j < alpha; ++j) pm = mulmod(pm, bm[j] % qb, qb);
            const u64 *ad = add + ((size_t)comp * l + l - 1) * n;
            for (int t = 0; t < n; ++t) {
                u64 v = xs[t];
                if (k == alpha) v = addmod(v, mulmod(ad[t], pm, qb), qb);
                yb[(size_t)k * n + t] = mulmod(v, hinv[k], qb);
            }
        }
        for (int i = 0; i < l - 1; ++i) {
            u64 q = c->mods[i].q, pm = 1, bmq = 1, hq[16];
            for (int j = 0; j < alpha; ++j) pm = mulmod(pm, bm[j] % q, q);
            for (int k = 0; k < nb; ++k) {
                bmq = mulmod(bmq, bm[k] % q, q);
                hq[k] = 1;   /* (B/b) mod q */
                for (int j = 0; j < nb; ++j) if (j != k) hq[k] = mulmod(hq[k], bm[j] % q, q);
            }
            u64 binv = invmod(bmq, q);
            const u64 *xi = acc + ((size_t)comp * lt + i) * n, *ai = add + ((size_t)comp * l + i) * n;
            u64 *o = out + ((size_t)comp * (l - 1) + i) * n;
            for (int t = 0; t < n; ++t) {
                u64 cv = 0;
                for (int k = 0; k < nb; ++k) {
                    u64 y = yb[(size_t)k * n + t];
                    u64 yq = y > bm[k] / 2 ? submod(y % q, bm[k] % q, q) : y % q;   /* y - b */
                    cv = addmod(cv, mulmod(yq, hq[k], q), q);
                }
                u64 xp = addmod(xi[t], mulmod(ai[t], pm, q), q);
                o[t] = mulmod(submod(xp, cv, q), binv, q);
            }
        }
    }
    free(yb);
    free(acc);
}

/*
 * Switching key for s' (given as residues sp[t][N], t <= L) in coefficient form,
 * key[2][ng][L+1+alpha][N]: for group b and target t (q_0..q_L, p_1..p_alpha),
 *   key[0][b][t] = -a_b s + e_b + [t in group b] (P mod q_t) s'_t,   key[1][b][t] = a_b,
 * a_b uniform with stream sid_base + 2b (modulus index t), e_b centred binomial with stream
 * sid_base + 2b + 1.  max_l < L + 1: only the groups and targets a ciphertext of at most max_l
 * limbs uses (the entries are those of the full key).
 */
void ref_gen_ksk(const ref_ctx *c, int L, int alpha, const i64 *s, const u64 *sp, u64 seed, u64 sid_base,
                 int max_l, u64 *key) {
    int n = c->n, nt = L + 1 + alpha, ng = ref_num_groups(L + 1, alpha);
    size_t kc = (size_t)ng * nt * n;
#pragma omp parallel
    {
        i64 *e = (i64 *)malloc(sizeof(i64) * n);
        u64 *sres = (u64 *)malloc(sizeof(u64) * n), *as = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for schedule(dynamic)
        for (int bt = 0; bt < ng * nt; ++bt) {
            int b = bt / nt, t = bt % nt;
            if (grp_first(b, alpha) >= max_l || (t >= max_l && t <= L)) continue;
            u64 q = c->mods[t].q;
            u64 *kb = key + (size_t)b * nt * n + (size_t)t * n;
            u64 *ka = key + kc + (size_t)b * nt * n + (size_t)t * n;
            ref_sample_uniform(seed, sid_base + 2ULL * b, t, q, n, ka);
            ref_sample_cbd(seed, sid_base + 2ULL * b + 1, n, e);
            for (int k = 0; k < n; ++k) sres[k] = from_signed(s[k], q);
            ref_polymul(c, t, ka, sres, as);
            for (int k = 0; k < n; ++k) kb[k] = addmod(submod(0, as[k], q), from_signed(e[k], q), q);
            int f = grp_first(b, alpha), m = grp_size(b, L + 1, alpha);
            if (t <= L && t >= f && t < f + m) {
                u64 pm = 1;   /* P mod q_t */
                for (int k = 0; k < alpha; ++k) pm = mulmod(pm, c->mods[L + 1 + k].q % q, q);
                const u64 *spt = sp + (size_t)t * n;
                for (int k = 0; k < n; ++k) kb[k] = addmod(kb[k], mulmod(pm, spt[k], q), q);
            }
        }
        free(e); free(sres); free(as);
    }
}

/* key (coefficient form, [2][ng][nt][N]) -> the oracle's evaluation form, same layout */
void ref_key_to_eval(const ref_ctx *c, int L, int alpha, int max_l, const u64 *key, u64 *kev) {
    int n = c->n, nt = L + 1 + alpha, ng = ref_num_groups(L + 1, alpha);
#pragma omp parallel for schedule(dynamic)
    for (int x = 0; x < 2 * ng * nt; ++x) {
        int t = x % nt, b = (x / nt) % ng;
        if (grp_first(b, alpha) >= max_l || (t >= max_l && t <= L)) continue;
        ref_to_eval(c, t, key + (size_t)x * n, kev + (size_t)x * n);
    }
}

/*
 * Public key pk[2][L+1][N] (coefficient form): pk0 = -a s + e, pk1 = a mod q_t, t <= L.
 * a: stream sid_a (uniform, modulus index t), e: stream sid_e.
 */
void ref_gen_pk(const ref_ctx *c, int L, const i64 *s, u64 seed, u64 sid_a, u64 sid_e, u64 *pk) {
    int n = c->n, l = L + 1;
    i64 *e = (i64 *)malloc(sizeof(i64) * n);
    ref_sample_cbd(seed, sid_e, n, e);
#pragma omp parallel
    {
        u64 *sres = (u64 *)malloc(sizeof(u64) * n), *as = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for
        for (int t = 0; t < l; ++t) {
            u64 q = c->mods[t].q;
            u64 *b = pk + (size_t)t * n, *a = pk + ((size_t)l + t) * n;
            ref_sample_uniform(seed, sid_a, t, q, n, a);
            for (int k = 0; k < n; ++k) sres[k] = from_signed(s[k], q);
            ref_polymul(c, t, a, sres, as);
            for (int k = 0; k < n; ++k) b[k] = addmod(submod(0, as[k], q), from_signed(e[k], q), q);
        }
        free(sres); free(as);
    }
    free(e);
}

/*
 * Encrypt (public key): ct = v * pk + (m + e0, e1) mod q_0..q_{l-1}.
 * v ternary (stream 1), e0, e1 centred binomial (streams 2, 3) of the encryption seed.
 * pk holds L+1 limbs (pk_l = L+1); m is an integer polynomial.
 */
void ref_encrypt(const ref_ctx *c, int pk_l, const u64 *pk, int l, const i64 *m, u64 seed, u64 *ct) {
    int n = c->n;
    i64 *v = (i64 *)malloc(sizeof(i64) * n), *e0 = (i64 *)malloc(sizeof(i64) * n), *e1 = (i64 *)malloc(sizeof(i64) * n);
    ref_sample_ternary(seed, 1, n, v);
    ref_sample_cbd(seed, 2, n, e0);
    ref_sample_cbd(seed, 3, n, e1);
#pragma omp parallel
    {
        u64 *vr = (u64 *)malloc(sizeof(u64) * n), *t = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            for (int k = 0; k < n; ++k) vr[k] = from_signed(v[k], q);
            u64 *c0 = ct + (size_t)i * n, *c1 = ct + ((size_t)l + i) * n;
            ref_polymul(c, i, vr, pk + (size_t)i * n, t);
            for (int k = 0; k < n; ++k)
                c0[k] = addmod(addmod(t[k], from_signed(m[k], q), q), from_signed(e0[k], q), q);
            ref_polymul(c, i, vr, pk + ((size_t)pk_l + i) * n, t);
            for (int k = 0; k < n; ++k) c1[k] = addmod(t[k], from_signed(e1[k], q), q);
        }
        free(vr); free(t);
    }
    free(v); free(e0); free(e1);
}

/* Decrypt: m = c0 + c1 s mod q_i for each limb (coefficient form; CRT is left to the caller). */
void ref_decrypt(const ref_ctx *c, int l, const u64 *ct, const i64 *s, u64 *m) {
    int n = c->n;
#pragma omp parallel
    {
        u64 *sr = (u64 *)malloc(sizeof(u64) * n), *t = (u64 *)malloc(sizeof(u64) * n);
#pragma omp for
        for (int i = 0; i < l; ++i) {
            u64 q = c->mods[i].q;
            for (int k = 0; k < n; ++k) sr[k] = from_signed(s[k], q);
            ref_polymul(c, i, ct + ((size_t)l + i) * n, sr, t);
            for (int k = 0; k < n; ++k) m[(size_t)i * n + k] = addmod(ct[(size_t)i * n + k], t[k], q);
        }
        free(sr); free(t);
    }
}

/* number of OpenMP threads the oracle runs with */
int ref_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

/* set the number of OpenMP threads of later calls (n <= 0: one per processor) */
void ref_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

/* s^2 mod each q_t, t < nl (the relinearisation key's target secret) */
void ref_secret_square(const ref_ctx *c, int nl, const i64 *s, u64 *out) {
    int n = c->n;
    u64 *sr = (u64 *)malloc(sizeof(u64) * n);
    for (int t = 0; t < nl; ++t) {
        u64 q = c->mods[t].q;
        for (int k = 0; k < n; ++k) sr[k] = from_signed(s[k], q);
        ref_polymul(c, t, sr, sr, out + (size_t)t * n);
    }
    free(sr);
}
