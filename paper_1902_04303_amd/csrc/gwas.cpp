// The encrypted modified semi-parallel GWAS (paper: Alg. Semi Parallel GWAS with Alg. Homomorphic
// LogReg and Alg. inverseSlots) on the device evaluator.
//
// Layout (paper: Methods, "Homomorphic Matrix Operations" and "Batching SNPs"):
//   R = PO2(n) rows per block, B = N / (2R) blocks, tau = 2B = N / R SNPs per ciphertext.
//   x_j and y are R-periodic (slot s holds v[s mod R] for s mod R < n, else 0): a CP column duplicated
//   into every block, so the log2(R)-step rotate-and-sum leaves the full dot product in every slot.
//   A_jl = ((X^T X)^-1)_jl are replicated scalars, encrypted at depth 0 with scale R * Delta_0.
//   SNP batch b is complex-packed CCP: slot c R + r holds S[r, b tau + 2c] + i S[r, b tau + 2c + 1].
// The projection M S (eqs. M and Sprime) is applied as S - sum_j x_j (.) bcast(mask (.) colSum(r_j (.) S))
// with r_j = sum_l A_jl x_l, all SNP batches of a chunk in one batched ciphertext.
#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <thread>
#include <type_traits>

#include "gwas.h"

namespace gck {

// kappa >= 2: 7 levels per Newton pass after the first, SNP batches at 7 kappa, denominators at 7 kappa + 5.
// kappa = 1: the weights are public (p = sigma7(0) = 1/2), SNP batches at 4, outputs at 8.
int circuit_levels(int kappa) {
    if (kappa < 1) throw Error(CKKS_E_INVALID_ARG, "kappa must be >= 1");
    return kappa == 1 ? 8 : 7 * kappa + 5;
}
int snp_depth(int kappa) {
    if (kappa < 1) throw Error(CKKS_E_INVALID_ARG, "kappa must be >= 1");
    return kappa == 1 ? 4 : 7 * kappa;
}

// Alg. inverseSlots (guess 3, three Newton steps g <- g (2 - w g)) at the public w of kappa = 1; every
// step is exact in FP64 here: 3.75, 3.984375, 4 - 2^-14
static double inverse_slots_public(double w) {
    double g = 3.0;
    for (int i = 0; i < 3; ++i) g = g * (2.0 - w * g);
    return g;
}
constexpr double kWKappa1 = 0.25;

Layout make_layout(int n_ring, int n, int k, int m) {
    if (n < 2 || k < 1 || m < 1) throw Error(CKKS_E_INVALID_ARG, "need n >= 2, k >= 1, m >= 1");
    Layout L;
    L.N = n_ring;
    L.n = n;
    L.k = k;
    L.m = m;
    L.R = 1;
    while (L.R < n) L.R *= 2;
    if (2 * L.R > n_ring) throw Error(CKKS_E_INVALID_ARG, "n too large for the ring: need PO2(n) <= N/2");
    L.blocks = n_ring / (2 * L.R);
    L.tau = 2 * L.blocks;
    L.n_batches = (m + L.tau - 1) / L.tau;
    return L;
}

std::vector<std::vector<i64>> rotation_groups(int R, int radix) {
    std::vector<std::vector<i64>> out;
    for (i64 s = 1; s < R;) {
        const i64 m = std::min<i64>(radix, R / s);   // this group covers the shifts j s, j < m
        std::vector<i64> grp;
        for (i64 j = 1; j < m; ++j) grp.push_back(j * s);
        out.push_back(grp);
        s *= m;
    }
    return out;
}

int diag_width(const Layout &lay) {
    if (lay.k < 2) return 0;
    int K = 1;
    while (K < lay.k) K *= 2;
    const int m = std::min(kBatchRadix, lay.R);
    if (K > m || m % K || lay.n + K - 1 > lay.R) return 0;
    return K;
}

std::vector<std::vector<i64>> stride_groups(int R, int K, int radix) {
    const auto g = rotation_groups(R, radix);
    std::vector<std::vector<i64>> out;
    if (g.empty()) return out;
    std::vector<i64> head;
    for (i64 r : g[0])
        if (r % K == 0) head.push_back(r);
    if (!head.empty()) out.push_back(head);
    for (size_t i = 1; i < g.size(); ++i) out.push_back(g[i]);
    return out;
}

std::vector<u64> required_galois(int n, int R) {
    std::vector<u64> g;
    auto put = [&](u64 e) {
        if (std::find(g.begin(), g.end(), e) == g.end()) g.push_back(e);
    };
    for (int radix : {kFixedRadix, kBatchRadix})
        for (const auto &grp : rotation_groups(R, radix))
            for (i64 r : grp) {
                put(galois_rotate_n(n, r));
                put(galois_rotate_n(n, -r));
            }
    put(2ULL * (u64)n - 1);   // conjugation
    return g;
}

namespace {

struct Circ {
    ckks_ctx &c;
    const Layout &lay;
    int radix;   // rotate-and-sum groups: up to radix - 1 rotations per key switch
    Circ(ckks_ctx &cc, const Layout &l, int rdx) : c(cc), lay(l), radix(rdx) {}

    // a at depth d and the canonical scale; factor multiplies the value.  Already there: a view of a (no
    // copy; valid while a lives, and only read)
    Ct at(const ckks_ct &a, int d, double factor = 1.0) {
        if (d == a.depth && factor == 1.0) return view(a, 0, a.count);
        return align(c, a, d, c.p.scales[d], factor);
    }
    // sum_{i < R} Rot(a, i) (Alg. colSum / Alg. DotProd): per group {s, 2s, .., (m - 1) s} of
    // rotation_groups, a <- a + sum_j Rot(a, j s) with one shared key switch
    Ct rot_sum(Ct a) {
        for (const auto &grp : rotation_groups(lay.R, radix)) a = rotate_sum(c, *a, grp);
        return a;
    }
    Ct bcast(Ct a) {     // sum_{i < R} Rot(a, -i): the first slot of each block over the block
        for (const auto &grp : rotation_groups(lay.R, radix)) {
            std::vector<i64> neg;
            for (i64 r : grp) neg.push_back(-r);
            a = rotate_sum(c, *a, neg);
        }
        return a;
    }
    Ct msum(const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &p) { return mul_sum(c, p); }

    // sigma7 of u = eta / 8 at the canonical scale (eq. sigma7, signs of the odd terms as a sigmoid)
    Ct sigma7(const ckks_ct &u) {
        const int d = u.depth;
        Ct u2 = mul(c, u, u);
        Ct a1 = add_const(c, *mul_const(c, *u2, -kSigma7C3), kSigma7C1);
        Ct a2 = add_const(c, *mul_const(c, *u2, -kSigma7C7), kSigma7C5);
        Ct u4 = mul(c, *u2, *u2);
        Ct b = mul(c, *u4, *a2);
        Ct cc = add(c, *at(*a1, d + 3), *b);
        Ct pr = mul(c, *at(u, d + 3), *cc);
        return add_const(c, *pr, 0.5);
    }
};

}  // namespace

// ---------------------------------------------------------------- batch helpers

// copy ciphertext si of batch s into slot di of batch d (same depth)
static void copy_ct(ckks_ctx &c, ckks_ct &d, int di, const ckks_ct &s, int si) {
    const size_t per = (size_t)2 * s.limbs * c.p.n;
    GCK_HIP(hipMemcpyAsync(d.data.ptr + (size_t)di * per, s.data.ptr + (size_t)si * per, per * 8,
                           hipMemcpyDeviceToDevice, c.stream));
}

// a batch made of ciphertext items[i].second of batch items[i].first
static Ct gather(ckks_ctx &c, const std::vector<std::pair<const ckks_ct *, int>> &items) {
    const ckks_ct &f = *items[0].first;
    Ct r = new_ct(c, (int)items.size(), f.depth, f.scale);
    for (size_t i = 0; i < items.size(); ++i) {
        if (items[i].first->depth != f.depth || items[i].first->scale != f.scale)
            throw Error(CKKS_E_PARAM_MISMATCH, "gathered ciphertexts differ in depth or scale");
        copy_ct(c, *r, (int)i, *items[i].first, items[i].second);
    }
    return r;
}

// ---------------------------------------------------------------- fixed part (per job, batched over jobs)

namespace {
// The stacked inputs of the fixed part and the batched helpers over them.  The k columns x_j are stacked
// into one batch (x_j of job i at position j J + i), and so is each column of A: the k independent
// products, rotate-and-sums and product sums over j then run as one batched call each.  Every ciphertext
// goes through the same operations as in a per-j loop.
struct StackIn {
    Ct Xs;
    std::vector<Ct> Acol;
};
StackIn stack_inputs(ckks_ctx &c, int k, const std::vector<const ckks_ct *> &x, const std::vector<const ckks_ct *> &Ain) {
    StackIn s;
    s.Xs = stack(c, x);
    s.Acol.resize(k);
    for (int l = 0; l < k; ++l) {
        std::vector<const ckks_ct *> col;
        for (int j = 0; j < k; ++j) col.push_back(Ain[a_index(k, std::min(j, l), std::max(j, l))]);
        s.Acol[l] = stack(c, col);
    }
    return s;
}
struct Stacked {
    ckks_ctx &c;
    Layout lay;
    Circ C;
    int k, J;
    StackIn own;
    const StackIn &in;   // pre: stacked once by the caller and shared (read only); else own
    const ckks_ct &Xs;
    const std::vector<Ct> &Acol;
    Stacked(ckks_ctx &ctx, int R, int k_, const std::vector<const ckks_ct *> &x, const std::vector<const ckks_ct *> &Ain,
            const StackIn *pre)
        : c(ctx), lay(make_lay(R, k_)), C(ctx, lay, kFixedRadix), k(k_), J(x[0]->count),
          own(pre ? StackIn{} : stack_inputs(ctx, k_, x, Ain)), in(pre ? *pre : own), Xs(*in.Xs), Acol(in.Acol) {}
    static Layout make_lay(int R, int k) {
        Layout l;
        l.R = R;
        l.k = k;
        return l;
    }
    std::vector<Ct> parts(const ckks_ct &s) const {
        std::vector<Ct> v(k);
        for (int j = 0; j < k; ++j) v[j] = view(s, j * J, J);
        return v;
    }
    // (A v)_j = sum_l A_jl v_l for every j at once, A at the depth of v
    Ct a_times(const std::vector<Ct> &v) {
        std::vector<Ct> Ad(k);
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> q;
        for (int l = 0; l < k; ++l) {
            Ad[l] = C.at(*Acol[l], v[0]->depth);
            q.push_back({Ad[l].get(), v[l].get()});
        }
        return C.msum(q);
    }
    // sum_j x_j t_j for stacked t, x at the depth of t (times factor)
    Ct x_dot(const ckks_ct &t, double factor) {
        Ct Xd = C.at(Xs, t.depth, factor);
        std::vector<Ct> a = parts(*Xd), b = parts(t);
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> q;
        for (int j = 0; j < k; ++j) q.push_back({a[j].get(), b[j].get()});
        return C.msum(q);
    }
};
}  // namespace

void fixed_front(ckks_ctx &c, int R, int k, const std::vector<const ckks_ct *> &x, const std::vector<const ckks_ct *> &Ain,
                 int ds, FixedOut &fx, int K, const StackIn *pre = nullptr, const ckks_ct *xrep = nullptr,
                 EncOutput *rep = nullptr) {
    Stacked st(c, R, k, x, Ain, pre);
    const int J = st.J;
    // ---- r_j = (X A)_{:, j} from A and x brought to the SNP depth - 2 first (r_j is used no higher than
    // the SNP depth - 1, so the products run on the few limbs left there), and x_j at the depth the
    // per-batch part uses it
    std::vector<Ct> x1(k);
    for (int l = 0; l < k; ++l) x1[l] = st.C.at(*x[l], ds - 2);
    Ct RR = st.a_times(x1);
    if (xrep) {
        // M-materialised layout (Alg. CP-REP-MatMult of X A with the REP X^T, one column of M at a time):
        // Dup(M_i) = Dup(e_i) - sum_j r_j X_ij for every sample i, as one batch of n
        if (J != 1) throw Error(CKKS_E_INVALID_ARG, "the M-materialised layout runs one job at a time");
        const int n = xrep->count / k;
        Ct RRx = st.C.at(*RR, xrep->depth);   // r_j at the REP X^T's depth (SNP depth + 1), all j at once
        std::vector<Ct> rj(k), xj(k);
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pr;
        for (int j = 0; j < k; ++j) {
            rj[j] = view(*RRx, j, 1);
            xj[j] = view(*xrep, j * n, n);
            pr.push_back({rj[j].get(), xj[j].get()});
        }
        Ct G = mul_sum(c, pr);   // at the REP rows' depth, SNP depth + 2
        Ct D = add_slot_indicators(c, *neg(c, *G), R);
        if (D->depth != ds + 2) throw Error(CKKS_E_LEVEL, "REP X^T at the wrong depth");
        fx.m_cols = view(*D, 0, D->count);
        fx.hold.push_back(std::move(D));
        if (rep) rep->m_cols = clone(c, *fx.m_cols);
    }
    if (K) {
        // packed projection: Z_t = sum_j comb_{(j - t) mod K} r_j and X_t = sum_j comb_{(j - t) mod K} x_j
        // (comb_c: the slots s = c mod K), block row r of Z_t holding r_{(r + t) mod K}[r].  The mask products
        // take r_j at the SNP depth - 1 and x_j at the SNP depth + 1, so that Z_t lands at the SNP depth and
        // X_t at the SNP depth + 2 with their canonical scales; Z_t is then rotated right by t.  r_s and x_c
        // stay empty (the packed projection does not read them).
        if (RR->depth > ds - 1 || st.Xs.depth >= ds + 1) throw Error(CKKS_E_LEVEL, "diagonals too deep");
        fx.K = K;
        Ct RRa = st.C.at(*RR, ds - 1), Xa = st.C.at(st.Xs, ds + 1);
        const std::vector<Ct> rj = st.parts(*RRa), xj = st.parts(*Xa);
        for (int t = 0; t < K; ++t) {
            std::vector<MaskTerm> tz, tx;
            for (int j = 0; j < k; ++j) {
                const int cls = ((j - t) % K + K) % K;
                tz.push_back({rj[j].get(), K, cls, cls + 1});
                tx.push_back({xj[j].get(), K, cls, cls + 1});
            }
            Ct z = mask_sum(c, tz);
            fx.z_d.push_back(t ? rotate(c, *z, -t) : std::move(z));
            fx.x_d.push_back(mask_sum(c, tx));
        }
        fx.hold.push_back(std::move(RR));
        return;
    }
    Ct RRs = st.C.at(*RR, ds);
    // x_j at ds + 2 owned here (the stacked x may be the caller's, shared with the other part)
    Ct Xc = st.Xs.depth == ds + 2 ? clone(c, st.Xs) : st.C.at(st.Xs, ds + 2);
    fx.r_s.resize(k);
    fx.x_c.resize(k);
    for (int j = 0; j < k; ++j) {
        fx.r_s[j] = view(*RRs, j * J, J);
        fx.x_c[j] = view(*Xc, j * J, J);
    }
    // RRs may be a view of RR (at() does not copy)
    fx.hold.push_back(std::move(RRs));
    fx.hold.push_back(std::move(Xc));
    fx.hold.push_back(std::move(RR));
}

void fixed_back(ckks_ctx &c, int R, int k, int kappa, const std::vector<const ckks_ct *> &x, const ckks_ct &y,
                const std::vector<const ckks_ct *> &Ain, int ds, FixedOut &fx, EncOutput &rep,
                const StackIn *pre = nullptr, hipEvent_t w_ready = nullptr) {
    Stacked st(c, R, k, x, Ain, pre);
    Circ &C = st.C;
    const int J = st.J;
    const ckks_ct &Xs = st.Xs;
    // ---- Alg. Homomorphic LogReg, first pass: beta = 0, so p = sigma7(0) = 1/2 is public
    Ct r = add_const(c, y, -0.5);
    Ct G = C.rot_sum(mul(c, Xs, *r));                    // g_j = X^T (y - p), stacked over j
    Ct beta = mul_int(c, *st.a_times(st.parts(*G)), 4);  // beta_j = 4 (A g)_j, stacked over j
    if (kappa == 1) {
        // p = 1/2, w = 1/4 and w^-1 = inverseSlots(1/4) are public: z = X beta + w^-1 (y - 1/2) with the
        // constant folded into the alignment of y - 1/2; u = z' / 4 by an alignment to the SNP part's depth
        Ct xbeta = st.x_dot(*beta, 1.0);
        Ct z = add(c, *xbeta, *C.at(*r, xbeta->depth, inverse_slots_public(kWKappa1)));
        Ct H = C.rot_sum(mul(c, *C.at(Xs, z->depth), *z));
        Ct V = st.a_times(st.parts(*H));
        Ct xvs = st.x_dot(*V, 1.0);
        Ct z_proj = sub(c, *C.at(*z, xvs->depth), *xvs);
        Ct u = C.at(*z_proj, ds + 3, kWKappa1);
        for (int j = 0; j < k; ++j) rep.beta.push_back(clone(c, *view(*beta, j * J, J)));
        fx.u_s = C.at(*u, ds + 3);   // a view of u, which rep owns from here on
        fx.w_s.reset();
        rep.z_proj = std::move(z_proj);
        rep.u = std::move(u);
        return;
    }
    Ct pk;
    for (int t = 1; t < kappa; ++t) {
        Ct u = st.x_dot(*beta, 0.125);                   // the 1/8 of sigma7's argument
        pk = C.sigma7(*u);
        const int dp = pk->depth;
        r = sub(c, *C.at(y, dp), *pk);
        G = C.rot_sum(mul(c, *C.at(Xs, dp), *r));
        Ct inc = mul_int(c, *st.a_times(st.parts(*G)), 4);
        beta = add(c, *C.at(*beta, inc->depth), *inc);
    }
    // ---- w = p (1 - p), Alg. inverseSlots: guess 3, the first Newton step is 6 - 9 w
    Ct w = mul(c, *pk, *add_const(c, *neg(c, *pk), 1.0));
    fx.w_s = C.at(*w, ds + 4);   // at the depth of the denominators' product T (may be a view of w)
    if (w_ready) GCK_HIP(hipEventRecord(w_ready, c.stream));
    Ct gi = add_const(c, *mul_int(c, *w, -9), 6.0);
    for (int it = 0; it < 2; ++it) {
        Ct wg = mul(c, *C.at(*w, gi->depth), *gi);
        Ct h = add_const(c, *neg(c, *wg), 2.0);
        gi = mul(c, *C.at(*gi, h->depth), *h);
    }
    Ct w_inv = std::move(gi);
    // ---- z = X beta^(kappa) + w^-1 (y - p^(kappa-1))
    Ct xbeta = st.x_dot(*beta, 1.0);
    Ct tz = mul(c, *C.at(*r, w_inv->depth), *w_inv);
    Ct z = add(c, *C.at(*xbeta, tz->depth), *tz);
    // ---- z' = z - X (A (X^T z))
    Ct H = C.rot_sum(mul(c, *C.at(Xs, z->depth), *z));
    Ct V = st.a_times(st.parts(*H));
    Ct xvs = st.x_dot(*V, 1.0);
    Ct z_proj = sub(c, *C.at(*z, xvs->depth), *xvs);
    Ct u = mul(c, *C.at(*w, z_proj->depth), *z_proj);
    // ---- what the per-batch part needs, at the depths it uses them
    for (int j = 0; j < k; ++j) rep.beta.push_back(clone(c, *view(*beta, j * J, J)));
    fx.u_s = C.at(*u, ds + 3);   // may be a view of u, which rep owns from here on
    rep.w = std::move(w);
    rep.w_inv = std::move(w_inv);
    rep.z_proj = std::move(z_proj);
    rep.u = std::move(u);
}

void run_fixed(ckks_ctx &c, int R, int k, int kappa, const std::vector<const ckks_ct *> &x, const ckks_ct &y,
               const std::vector<const ckks_ct *> &Ain, int ds, FixedOut &fx, EncOutput &rep, int K) {
    fixed_front(c, R, k, x, Ain, ds, fx, K);
    fixed_back(c, R, k, kappa, x, y, Ain, ds, fx, rep);
}

// ---------------------------------------------------------------- per-batch part

// S' = S - sum_j x_j E_j with E_j = bcast_R(mask(colSum(r_j S))): needs only r_j and x_j of the fixed part.
// The products r_j S of several covariates run as one stacked batch through colSum, the mask and bcast while
// the stack holds at most c.stack_cts ciphertexts (every key switch then reads its keys once for all of
// them); the same operations on each ciphertext, so the results are those of one covariate at a time.
Ct batch_front(ckks_ctx &c, int R, int k, const FixedOut &fx, const ckks_ct &S) {
    Layout lay;
    lay.R = R;
    lay.k = k;
    Circ C(c, lay, kBatchRadix);
    if (fx.K) {
        // packed projection: D = sum_t Rot(Z_t, -t) Rot(S, -t) (one lazy product sum); W = sum_{u < R/K}
        // Rot(D, K u) holds C_j = colSum(r_j S) at slot j < k of each block; the mask of the first k slots;
        // V = sum_{u < R/K} Rot(., -K u) holds C_{r mod K} at block row r; x E = sum_t X_t Rot(V, t)
        const int K = fx.K;
        const auto groups = stride_groups(R, K, kBatchRadix);
        std::vector<i64> right, left;
        for (int t = 1; t < K; ++t) {
            right.push_back(-t);
            left.push_back(t);
        }
        std::vector<Ct> rs = rotate_many(c, S, right);   // one ModUp of S for the K - 1 rotations
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pd{{fx.z_d[0].get(), &S}};
        for (int t = 1; t < K; ++t) pd.push_back({fx.z_d[t].get(), rs[t - 1].get()});
        Ct w = mul_sum(c, pd);
        rs.clear();
        for (const auto &grp : groups) w = rotate_sum(c, *w, grp);
        Ct v = mask_sum(c, {{w.get(), R, 0, k}});
        w.reset();
        for (const auto &grp : groups) {
            std::vector<i64> neg;
            for (i64 r : grp) neg.push_back(-r);
            v = rotate_sum(c, *v, neg);
        }
        std::vector<Ct> rv = rotate_many(c, *v, left);
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pe{{fx.x_d[0].get(), v.get()}};
        for (int t = 1; t < K; ++t) pe.push_back({fx.x_d[t].get(), rv[t - 1].get()});
        Ct xe = mul_sum(c, pe);
        return sub(c, *C.at(S, xe->depth), *xe);
    }
    const int cnt = S.count;
    const int per = std::max(1, std::min(k, c.stack_cts / std::max(1, cnt)));   // covariates per stack
    std::vector<Ct> stacks, E(k);
    for (int j0 = 0; j0 < k; j0 += per) {
        const int j1 = std::min(k, j0 + per);
        std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pp;
        for (int j = j0; j < j1; ++j) pp.push_back({fx.r_s[j].get(), &S});
        Ct P = mul_stack(c, pp);
        P = C.rot_sum(std::move(P));          // column sums at block starts (Alg. colSum)
        P = mul_mask(c, *P, R);               // keep the block starts
        P = C.bcast(std::move(P));            // (A X^T S)_{j, c} over block c
        for (int j = j0; j < j1; ++j) E[j] = view(*P, (j - j0) * cnt, cnt);
        stacks.push_back(std::move(P));       // owns the views' memory until the sum below
    }
    std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pe;
    for (int j = 0; j < k; ++j) pe.push_back({fx.x_c[j].get(), E[j].get()});
    Ct xe = C.msum(pe);
    return sub(c, *C.at(S, xe->depth), *xe);
}

// S' = M S of a chunk in the M-materialised layout: sum_i Dup(M_i) (.) S_rep(i) per batch
// (Alg. CP-REP-MatMult), one lazy tensor sum, one relinearisation and one rescale
Ct batch_front_m(ckks_ctx &c, const FixedOut &fx, const ckks_ct &S_rep_chunk) {
    return mul_sum_rep(c, *fx.m_cols, S_rep_chunk);
}

// numerator and denominators from S' (needs u and w of the fixed part)
// the numerator of o.sp (needs u of the fixed part)
void batch_num(ckks_ctx &c, int R, int k, const FixedOut &fx, BatchOut &o) {
    Layout lay;
    lay.R = R;
    lay.k = k;
    Circ C(c, lay, kBatchRadix);
    o.num = C.rot_sum(mul(c, *fx.u_s, *o.sp));
}

// both denominators of o.sp (need w of the fixed part, public for kappa = 1)
void batch_den(ckks_ctx &c, int R, int k, const FixedOut &fx, BatchOut &o) {
    Layout lay;
    lay.R = R;
    lay.k = k;
    Circ C(c, lay, kBatchRadix);
    // with S' = a + i b per slot (even SNP a, odd SNP b) both denominators come from one rotate-and-sum of
    // W = 4 w (a^2 + i b^2) = w T, T = (2 + 2i) S' conj(S') + (1 - i) (S'^2 + conj(S')^2) as one lazy
    // product sum (the Gaussian integer factors exact, as products with re + im X^(N/2)); den_even =
    // sum W / 4 and den_odd = -i sum W / 4 have the two denominators as their real parts
    Ct sc = conjugate(c, *o.sp);
    Ct p22 = mul_gauss(c, *o.sp, 2, 2), p1s = mul_gauss(c, *o.sp, 1, -1), p1c = mul_gauss(c, *sc, 1, -1);
    Ct t = mul_sum(c, {{p22.get(), sc.get()}, {p1s.get(), o.sp.get()}, {p1c.get(), sc.get()}});
    p22.reset();
    p1s.reset();
    p1c.reset();
    double f = 4.0 / kWKappa1;   // kappa = 1: public w = 1/4, in the tracked scale
    if (fx.w_s) {
        t = mul(c, *fx.w_s, *t);
        f = 4.0;
    }
    o.de = C.rot_sum(set_scale(c, std::move(t), f));
    o.dodd = mul_i(c, *o.de, true);
}

BatchOut batch_back(ckks_ctx &c, int R, int k, const FixedOut &fx, Ct sp) {
    BatchOut o;
    o.sp = std::move(sp);
    batch_num(c, R, k, fx, o);
    batch_den(c, R, k, fx, o);
    return o;
}

BatchOut run_batch(ckks_ctx &c, int R, int k, const FixedOut &fx, const ckks_ct &S) {
    return batch_back(c, R, k, fx, batch_front(c, R, k, fx, S));
}

static void check_keys(ckks_ctx &c, int R) {
    for (u64 g : required_galois(c.p.n, R))
        if (!has_key(c, g)) throw Error(CKKS_E_KEY_MISSING, "missing Galois key " + std::to_string(g));
    if (!has_key(c, 0)) throw Error(CKKS_E_KEY_MISSING, "missing relinearisation key");
}

void fetch_snp(ckks_ctx &c, const EncInput &in, int b0, int cnt, ckks_ct &dst, int di, hipStream_t st) {
    const size_t per = (size_t)2 * in.S->limbs * c.p.n;
    if (in.S_host) {
        GCK_HIP(hipMemcpyAsync(dst.data.ptr + (size_t)di * per, in.S_host + (size_t)b0 * per, (size_t)cnt * per * 8,
                               hipMemcpyHostToDevice, st));
    } else {
        GCK_HIP(hipMemcpyAsync(dst.data.ptr + (size_t)di * per, in.S->data.ptr + (size_t)b0 * per, (size_t)cnt * per * 8,
                               hipMemcpyDeviceToDevice, st));
    }
}

void spill_snp(ckks_ctx &c, EncInput &in) {
    if (in.S_host) return;
    const size_t bytes = in.S->data.words * 8;
    GCK_HIP(hipHostMalloc((void **)&in.S_host, bytes, hipHostMallocDefault));
    GCK_HIP(hipMemcpyAsync(in.S_host, in.S->data.ptr, bytes, hipMemcpyDeviceToHost, c.stream));
    sync(c);
    in.S->data.release();
}

static hipStream_t copy_stream(ckks_ctx &c) {
    if (!c.copy_stream) GCK_HIP(hipStreamCreate(&c.copy_stream));   // default priority
    return c.copy_stream;
}

void run_circuit(ckks_ctx &c, const EncInput &in, EncOutput &out, int chunk) {
    const Layout &lay = in.lay;
    const int k = lay.k;
    if (c.p.levels < circuit_levels(in.kappa))
        throw Error(CKKS_E_LEVEL, "the chain has " + std::to_string(c.p.levels) + " levels, the circuit needs " +
                                      std::to_string(circuit_levels(in.kappa)));
    check_keys(c, lay.R);
    std::vector<const ckks_ct *> x, A;
    for (auto &p : in.x) x.push_back(p.get());
    for (auto &p : in.A) A.push_back(p.get());
    FixedOut fx;
    const int ds = in.S->depth;
    const int nb = in.S->count;
    if (!in.S_host && c.pool->budget == 0 && c.n_streams == 2) {
        // The logistic regression (u, w) runs on the auxiliary stream while the main stream computes what
        // needs only r_j and x_j (their fixed-part products, then S' of every SNP batch).  The denominators
        // then wait for w only (public for kappa = 1), which the regression has before its last steps
        // (w^-1, z, z', u); the numerators wait for u.
        ensure_aux(c);
        const StackIn sin = stack_inputs(c, k, x, A);   // shared by both parts, read only
        stream_wait(c.aux_stream, c.stream);   // inputs, their stacking and this call's earlier work
        hipEvent_t w_ready;
        GCK_HIP(hipEventCreateWithFlags(&w_ready, hipEventDisableTiming));
        const std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> w_ready_owner(
            w_ready, hipEventDestroy);
        {
            OnStream on_aux(c);
            fixed_back(c, lay.R, k, in.kappa, x, *in.y, A, ds, fx, out, &sin, w_ready);
        }
        fixed_front(c, lay.R, k, x, A, ds, fx, in.S_rep ? 0 : diag_width(lay), &sin, in.Xrep.get(), &out);
        std::vector<Ct> sps;
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            const int cnt = std::min(chunk, nb - b0);
            // the batches are device-resident here (no spill): the chunk is a view, read only
            if (in.S_rep) {
                Ct Sr = view(*in.S_rep, b0 * lay.n, cnt * lay.n);
                sps.push_back(batch_front_m(c, fx, *Sr));
                continue;
            }
            Ct S = view(*in.S, b0, cnt);
            sps.push_back(batch_front(c, lay.R, k, fx, *S));
        }
        if (in.kappa != 1) GCK_HIP(hipStreamWaitEvent(c.stream, w_ready, 0));   // w
        std::vector<BatchOut> bos(sps.size());
        for (size_t i = 0; i < sps.size(); ++i) {
            bos[i].sp = std::move(sps[i]);
            batch_den(c, lay.R, k, fx, bos[i]);
        }
        stream_wait(c.stream, c.aux_stream);   // u
        for (BatchOut &o : bos) {
            batch_num(c, lay.R, k, fx, o);
            if (c.keep_s_proj) out.S_proj.push_back(std::move(o.sp));
            out.num.push_back(std::move(o.num));
            out.den_even.push_back(std::move(o.de));
            out.den_odd.push_back(std::move(o.dodd));
        }
        // buffers of the auxiliary pool were read on the main stream: later reuse on the auxiliary stream
        // comes after this work (under graph capture every block of the call stays reserved for the graph,
        // and the next call's own first wait orders the streams)
        if (!c.capturing) stream_wait(c.aux_stream, c.stream);
        return;
    }
    if (in.S_rep) {
        // M-materialised layout on one stream (or under a pool budget): device-resident REP rows only
        fixed_front(c, lay.R, k, x, A, ds, fx, 0, nullptr, in.Xrep.get(), &out);
        fixed_back(c, lay.R, k, in.kappa, x, *in.y, A, ds, fx, out);
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            const int cnt = std::min(chunk, nb - b0);
            Ct Sr = view(*in.S_rep, b0 * lay.n, cnt * lay.n);
            BatchOut o = batch_back(c, lay.R, k, fx, batch_front_m(c, fx, *Sr));
            if (c.keep_s_proj) out.S_proj.push_back(std::move(o.sp));
            out.num.push_back(std::move(o.num));
            out.den_even.push_back(std::move(o.de));
            out.den_odd.push_back(std::move(o.dodd));
        }
        return;
    }
    run_fixed(c, lay.R, k, in.kappa, x, *in.y, A, ds, fx, out, diag_width(lay));
    if (!in.S_host) {
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            const int cnt = std::min(chunk, nb - b0);
            Ct S = new_ct(c, cnt, ds, in.S->scale);
            fetch_snp(c, in, b0, cnt, *S, 0, c.stream);
            BatchOut o = run_batch(c, lay.R, k, fx, *S);
            if (c.keep_s_proj) out.S_proj.push_back(std::move(o.sp));
            out.num.push_back(std::move(o.num));
            out.den_even.push_back(std::move(o.de));
            out.den_odd.push_back(std::move(o.dodd));
        }
        return;
    }
    // spilled SNP batches: copy chunk i + 1 from pinned host memory on a second stream while chunk i
    // computes.  Each buffer's copy waits for an event recorded on the compute stream when the buffer was
    // taken from the pool, and chunk i's compute waits for its own copy.
    hipStream_t cs = copy_stream(c);
    auto start = [&](int b0, hipEvent_t &done) {
        const int cnt = std::min(chunk, nb - b0);
        Ct S = new_ct(c, cnt, ds, in.S->scale);
        hipEvent_t taken;
        GCK_HIP(hipEventCreateWithFlags(&taken, hipEventDisableTiming));
        GCK_HIP(hipEventRecord(taken, c.stream));
        GCK_HIP(hipStreamWaitEvent(cs, taken, 0));
        fetch_snp(c, in, b0, cnt, *S, 0, cs);
        GCK_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        GCK_HIP(hipEventRecord(done, cs));
        (void)hipEventDestroy(taken);
        return S;
    };
    hipEvent_t ev_cur, ev_next = nullptr;
    Ct cur = start(0, ev_cur);
    for (int b0 = 0; b0 < nb; b0 += chunk) {
        Ct next;
        if (b0 + chunk < nb) next = start(b0 + chunk, ev_next);
        GCK_HIP(hipStreamWaitEvent(c.stream, ev_cur, 0));
        BatchOut o = run_batch(c, lay.R, k, fx, *cur);
        (void)hipEventDestroy(ev_cur);
        if (c.keep_s_proj) out.S_proj.push_back(std::move(o.sp));
        out.num.push_back(std::move(o.num));
        out.den_even.push_back(std::move(o.de));
        out.den_odd.push_back(std::move(o.dodd));
        cur = std::move(next);
        ev_cur = ev_next;
    }
}

// ---------------------------------------------------------------- homomorphic division

// b' = num / den and err' = 1 / den as ciphertexts (an extension: the paper decrypts num and den and
// divides on the client).  Per chunk, the even and the odd denominators are stacked into one batch; the
// real part of each (its imaginary part holds the other parity's denominator) times the client's
// normaliser 1 / d_j gives x in (0, 1], whose reciprocal is taken by Newton steps from guess 1 (the
// pattern of Alg. inverseSlots: g_1 = 2 - x, then g <- g (2 - x g)); err' = g / d_j and b' = num err'
// (num read cyclically: its real part pairs with the even half, its imaginary part with the odd half).
int div_levels() { return 3 + 2 * (kDivIters - 1); }

void run_divide(ckks_ctx &c, EncOutput &out, const ckks_ct &v) {
    const int nb = v.count / 2;
    if (v.count != 2 * nb || nb < 1) throw Error(CKKS_E_INVALID_ARG, "normalisers: 2 per SNP batch");
    if (out.num.empty()) throw Error(CKKS_E_INVALID_ARG, "output has no SNP batches");
    int total = 0;
    for (auto &ct : out.num) total += ct->count;
    if (total != nb) throw Error(CKKS_E_INVALID_ARG, "normalisers do not match the number of SNP batches");
    const int dd = out.den_even[0]->depth;
    if (v.depth != dd) throw Error(CKKS_E_LEVEL, "normalisers must be at the denominators' depth");
    if (c.p.levels < dd + div_levels())
        throw Error(CKKS_E_LEVEL, "the division needs " + std::to_string(div_levels()) + " levels after depth " +
                                      std::to_string(dd));
    Layout lay;
    Circ C(c, lay, kBatchRadix);
    out.div_b.clear();
    out.div_inv.clear();
    int b0 = 0;
    for (size_t ch = 0; ch < out.num.size(); ++ch) {
        const int cnt = out.num[ch]->count;
        Ct D = stack(c, {out.den_even[ch].get(), out.den_odd[ch].get()});
        Ct Ve = view(v, b0, cnt), Vo = view(v, nb + b0, cnt);
        Ct V = stack(c, {Ve.get(), Vo.get()});
        Ct x = mul(c, *set_scale(c, add(c, *D, *conjugate(c, *D)), 2.0), *V);
        Ct g = add_const(c, *neg(c, *x), 2.0);
        for (int it = 1; it < kDivIters; ++it) {
            Ct h = mul(c, *C.at(*x, g->depth), *g);
            Ct e = add_const(c, *neg(c, *h), 2.0);
            g = mul(c, *C.at(*g, e->depth), *e);
        }
        Ct inv = mul(c, *g, *C.at(*V, g->depth));
        out.div_b.push_back(mul(c, *C.at(*out.num[ch], inv->depth), *inv));
        out.div_inv.push_back(std::move(inv));
        b0 += cnt;
    }
}

// ---------------------------------------------------------------- several jobs

std::tuple<int, int, int, int> bucket_of(const EncInput &in) {
    return std::make_tuple(in.lay.R, in.lay.k, in.kappa, diag_width(in.lay));
}

// Fixed parts of several jobs with one shape (R, k, kappa): one launch sequence over a batch of one
// ciphertext per job; the results are split back into one FixedOut (batches of one) per job.
void fixed_for_jobs(ckks_ctx &c, const std::vector<const EncInput *> &jobs, std::vector<FixedOut> &fxs,
                    std::vector<EncOutput> &reps) {
    const EncInput &j0 = *jobs[0];
    const int R = j0.lay.R, k = j0.lay.k, kappa = j0.kappa, J = (int)jobs.size(), K = diag_width(j0.lay);
    if (c.p.levels < circuit_levels(kappa)) throw Error(CKKS_E_LEVEL, "chain too short for kappa");
    for (auto *in : jobs)
        if (bucket_of(*in) != bucket_of(j0)) throw Error(CKKS_E_PARAM_MISMATCH, "jobs of different shapes");
    check_keys(c, R);
    std::vector<Ct> xs(k), As(k * (k + 1) / 2);
    for (int j = 0; j < k; ++j) {
        std::vector<std::pair<const ckks_ct *, int>> it;
        for (auto *in : jobs) it.push_back({in->x[j].get(), 0});
        xs[j] = gather(c, it);
    }
    for (int a = 0; a < k * (k + 1) / 2; ++a) {
        std::vector<std::pair<const ckks_ct *, int>> it;
        for (auto *in : jobs) it.push_back({in->A[a].get(), 0});
        As[a] = gather(c, it);
    }
    std::vector<std::pair<const ckks_ct *, int>> yit;
    for (auto *in : jobs) yit.push_back({in->y.get(), 0});
    Ct ys = gather(c, yit);
    std::vector<const ckks_ct *> xp, Ap;
    for (auto &p : xs) xp.push_back(p.get());
    for (auto &p : As) Ap.push_back(p.get());
    FixedOut fx;
    EncOutput rep;
    run_fixed(c, R, k, kappa, xp, *ys, Ap, snp_depth(kappa), fx, rep, K);
    fxs.clear();
    fxs.resize(J);
    reps.clear();
    reps.resize(J);
    for (int q = 0; q < J; ++q) {
        FixedOut &f = fxs[q];
        for (auto &r : fx.r_s) f.r_s.push_back(gather(c, {{r.get(), q}}));
        for (auto &xc : fx.x_c) f.x_c.push_back(gather(c, {{xc.get(), q}}));
        f.K = fx.K;
        for (auto &z : fx.z_d) f.z_d.push_back(gather(c, {{z.get(), q}}));
        for (auto &xd : fx.x_d) f.x_d.push_back(gather(c, {{xd.get(), q}}));
        f.u_s = gather(c, {{fx.u_s.get(), q}});
        if (fx.w_s) f.w_s = gather(c, {{fx.w_s.get(), q}});
        EncOutput &o = reps[q];
        for (int j = 0; j < k; ++j) o.beta.push_back(gather(c, {{rep.beta[j].get(), q}}));
        if (rep.w) o.w = gather(c, {{rep.w.get(), q}});
        if (rep.w_inv) o.w_inv = gather(c, {{rep.w_inv.get(), q}});
        o.z_proj = gather(c, {{rep.z_proj.get(), q}});
        o.u = gather(c, {{rep.u.get(), q}});
    }
}

// One chunk of SNP batches drawn from several jobs of one shape: items (job, batch); every batch is
// paired with its own job's fixed-part values; outputs land in slot `batch` of each job's outputs
// (allocated on first use).
void chunk_for_jobs(ckks_ctx &c, const std::vector<WorkItem> &items) {
    const EncInput &j0 = *items[0].in;
    const int R = j0.lay.R, k = j0.lay.k;
    Ct S = new_ct(c, (int)items.size(), j0.S->depth, j0.S->scale);
    for (size_t i = 0; i < items.size(); ++i) {
        if (items[i].in->S->depth != S->depth || items[i].in->S->scale != S->scale)
            throw Error(CKKS_E_PARAM_MISMATCH, "SNP batches of different depth or scale");
        fetch_snp(c, *items[i].in, items[i].batch, 1, *S, (int)i, c.stream);
    }
    auto per_item = [&](auto get) {
        std::vector<std::pair<const ckks_ct *, int>> it;
        for (auto &w : items) it.push_back({get(*w.fx), 0});
        return gather(c, it);
    };
    FixedOut fc;
    fc.K = items[0].fx->K;
    if (!fc.K) {
        for (int j = 0; j < k; ++j) fc.r_s.push_back(per_item([&](const FixedOut &f) { return f.r_s[j].get(); }));
        for (int j = 0; j < k; ++j) fc.x_c.push_back(per_item([&](const FixedOut &f) { return f.x_c[j].get(); }));
    }
    for (const WorkItem &w : items)
        if (w.fx->K != fc.K) throw Error(CKKS_E_PARAM_MISMATCH, "SNP batches of different projection widths");
    for (int t = 0; t < fc.K; ++t) {
        fc.z_d.push_back(per_item([&](const FixedOut &f) { return f.z_d[t].get(); }));
        fc.x_d.push_back(per_item([&](const FixedOut &f) { return f.x_d[t].get(); }));
    }
    fc.u_s = per_item([](const FixedOut &f) { return f.u_s.get(); });
    if (items[0].fx->w_s) fc.w_s = per_item([](const FixedOut &f) { return f.w_s.get(); });
    BatchOut bo = run_batch(c, R, k, fc, *S);
    for (size_t i = 0; i < items.size(); ++i) {
        EncOutput &o = *items[i].out;
        const int nbq = items[i].in->S->count;
        if (o.num.empty()) {
            if (c.keep_s_proj) o.S_proj.push_back(new_ct(c, nbq, bo.sp->depth, bo.sp->scale));
            o.num.push_back(new_ct(c, nbq, bo.num->depth, bo.num->scale));
            o.den_even.push_back(new_ct(c, nbq, bo.de->depth, bo.de->scale));
            o.den_odd.push_back(new_ct(c, nbq, bo.dodd->depth, bo.dodd->scale));
            o.chunk = nbq;
        }
        const int b = items[i].batch;
        if (c.keep_s_proj) copy_ct(c, *o.S_proj[0], b, *bo.sp, (int)i);
        copy_ct(c, *o.num[0], b, *bo.num, (int)i);
        copy_ct(c, *o.den_even[0], b, *bo.de, (int)i);
        copy_ct(c, *o.den_odd[0], b, *bo.dodd, (int)i);
    }
}

// Several jobs at once: jobs with the same (R, k, kappa) share every launch of the fixed part and their
// SNP batches go through the per-batch part together, `chunk` at a time.  Each job's output holds one
// batch per output kind.
void run_multi(ckks_ctx &c, const std::vector<const EncInput *> &jobs, std::vector<EncOutput> &outs, int chunk) {
    outs.clear();
    outs.resize(jobs.size());
    // A job with at least half a chunk of SNP batches fills the device with its own launches: it runs as a
    // single job (its logistic-regression part on the second stream, beside its own SNP batches), in chunks
    // of kMultiChunk batches or `chunk` if larger when it is resident and no pool budget is set (every job's
    // outputs stay resident here, so a chunk's transient buffers are bounded), else `chunk` at a time.  The
    // smaller jobs are bucketed by shape and share the fixed-part launches and the SNP-batch chunks (an
    // input with the M-materialised layout always runs as a single job).
    std::map<std::tuple<int, int, int, int>, std::vector<int>> buckets;
    for (size_t i = 0; i < jobs.size(); ++i) {
        if (2 * jobs[i]->S->count >= chunk || jobs[i]->S_rep) {
            const int own = (!jobs[i]->S_host && c.pool->budget == 0)
                                ? std::min(jobs[i]->S->count, std::max(chunk, kMultiChunk))
                                : chunk;
            outs[i].chunk = own;
            run_circuit(c, *jobs[i], outs[i], own);
            continue;
        }
        buckets[bucket_of(*jobs[i])].push_back((int)i);
    }
    for (auto &kv : buckets) {
        const std::vector<int> &ids = kv.second;
        std::vector<const EncInput *> bj;
        for (int id : ids) bj.push_back(jobs[id]);
        // fixed parts in groups of at most kMaxFixedJobs jobs: each group's launches still cover
        // k kMaxFixedJobs ciphertexts, and the transient key-switch buffers of the 27-limb fixed part
        // (about 0.5 GB per job) stay bounded however many jobs share the shape
        std::vector<FixedOut> fxs;
        for (size_t g0 = 0; g0 < bj.size(); g0 += kMaxFixedJobs) {
            const size_t g1 = std::min(bj.size(), g0 + kMaxFixedJobs);
            std::vector<const EncInput *> grp(bj.begin() + g0, bj.begin() + g1);
            std::vector<FixedOut> f;
            std::vector<EncOutput> reps;
            fixed_for_jobs(c, grp, f, reps);
            for (size_t q = 0; q < grp.size(); ++q) {
                outs[ids[g0 + q]] = std::move(reps[q]);
                fxs.push_back(std::move(f[q]));
            }
        }
        std::vector<WorkItem> work;
        for (size_t q = 0; q < ids.size(); ++q)
            for (int b = 0; b < bj[q]->S->count; ++b) work.push_back(WorkItem{bj[q], &fxs[q], &outs[ids[q]], b});
        for (size_t w0 = 0; w0 < work.size(); w0 += chunk) {
            const size_t cnt = std::min((size_t)chunk, work.size() - w0);
            chunk_for_jobs(c, std::vector<WorkItem>(work.begin() + w0, work.begin() + w0 + cnt));
        }
    }
}

// ---------------------------------------------------------------- client side

static std::vector<double> xtx_inverse(const double *X, int n, int k) {
    std::vector<double> G((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double s = 0;
            for (int i = 0; i < n; ++i) s += X[(size_t)i * k + a] * X[(size_t)i * k + b];
            G[(size_t)a * k + b] = s;
        }
    // Cholesky G = L L^T, then A = L^-T L^-1
    std::vector<double> L((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = G[(size_t)i * k + j];
            for (int t = 0; t < j; ++t) s -= L[(size_t)i * k + t] * L[(size_t)j * k + t];
            if (i == j) {
                if (!(s > 0)) throw Error(CKKS_E_INVALID_ARG, "X^T X is not positive definite");
                L[(size_t)i * k + i] = std::sqrt(s);
            } else {
                L[(size_t)i * k + j] = s / L[(size_t)j * k + j];
            }
        }
    std::vector<double> Li((size_t)k * k, 0.0);
    for (int col = 0; col < k; ++col)
        for (int i = 0; i < k; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int t = 0; t < i; ++t) s -= L[(size_t)i * k + t] * Li[(size_t)t * k + col];
            Li[(size_t)i * k + col] = s / L[(size_t)i * k + i];
        }
    std::vector<double> A((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double s = 0;
            for (int t = 0; t < k; ++t) s += Li[(size_t)t * k + a] * Li[(size_t)t * k + b];
            A[(size_t)a * k + b] = s;
        }
    return A;
}

// f(0) .. f(n - 1) on up to 16 host threads (host-side encoding work of the client)
template <typename F>
static void parallel_for(int n, F f) {
    const int T = std::max(1, std::min({n, 16, (int)std::thread::hardware_concurrency()}));
    if (T <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    std::exception_ptr err;
    std::mutex mu;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            try {
                for (int i = t; i < n; i += T) f(i);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
            }
        });
    for (auto &x : th) x.join();
    if (err) std::rethrow_exception(err);
}

static u64 input_seed(u64 enc_seed, u64 i) {
    auto mix = [](u64 z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    return mix(enc_seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

std::unique_ptr<EncInput> pack_encrypt(ckks_ctx &c, const double *X, const double *y, const uint8_t *S, int n, int k,
                                       int m, int kappa, u64 enc_seed) {
    auto in = std::make_unique<EncInput>();
    in->lay = make_layout(c.p.n, n, k, m);
    in->kappa = kappa;
    const Layout &lay = in->lay;
    const int N = c.p.n, slots = N / 2;
    std::vector<double> re(slots), im(slots);
    std::vector<i64> poly(N);
    u64 idx = 0;
    auto periodic = [&](auto get) {
        for (int s = 0; s < slots; ++s) {
            int r = s % lay.R;
            re[s] = r < n ? get(r) : 0.0;
        }
    };
    for (int j = 0; j < k; ++j) {
        periodic([&](int r) { return X[(size_t)r * k + j]; });
        encode_poly(N, re.data(), nullptr, slots, c.p.scales[0], poly.data());
        in->x.push_back(encrypt(c, poly.data(), 0, c.p.scales[0], input_seed(enc_seed, idx++)));
    }
    periodic([&](int r) { return y[r]; });
    encode_poly(N, re.data(), nullptr, slots, c.p.scales[0], poly.data());
    in->y = encrypt(c, poly.data(), 0, c.p.scales[0], input_seed(enc_seed, idx++));
    const std::vector<double> A = xtx_inverse(X, n, k);
    const double a_scale = c.p.scales[0] * (double)lay.R;
    for (int j = 0; j < k; ++j)
        for (int l = j; l < k; ++l) {
            std::fill(poly.begin(), poly.end(), 0);
            poly[0] = round_half_away(A[(size_t)j * k + l] * a_scale);
            in->A.push_back(encrypt(c, poly.data(), 0, a_scale, input_seed(enc_seed, idx++)));
        }
    const int ds = snp_depth(kappa);
    in->S = new_ct(c, lay.n_batches, ds, c.p.scales[ds]);
    const size_t per = (size_t)2 * in->S->limbs * N;
    // the host encodings of up to 64 batches at a time in parallel, then their encryptions in order
    const int group = 64;
    std::vector<std::vector<i64>> polys(group, std::vector<i64>(N));
    for (int b0 = 0; b0 < lay.n_batches; b0 += group) {
        const int cnt = std::min(group, lay.n_batches - b0);
        parallel_for(cnt, [&](int t) {
            const int b = b0 + t;
            std::vector<double> vr(slots, 0.0), vi(slots, 0.0);
            for (int cb = 0; cb < lay.blocks; ++cb) {
                const int j0 = b * lay.tau + 2 * cb;
                for (int r = 0; r < n; ++r) {
                    if (j0 < m) vr[(size_t)cb * lay.R + r] = (double)S[(size_t)r * m + j0];
                    if (j0 + 1 < m) vi[(size_t)cb * lay.R + r] = (double)S[(size_t)r * m + j0 + 1];
                }
            }
            encode_poly(N, vr.data(), vi.data(), slots, c.p.scales[ds], polys[t].data());
        });
        for (int t = 0; t < cnt; ++t) {
            Ct one = encrypt(c, polys[t].data(), ds, c.p.scales[ds], input_seed(enc_seed, idx++));
            GCK_HIP(hipMemcpyAsync(in->S->data.ptr + (size_t)(b0 + t) * per, one->data.ptr, per * 8,
                                   hipMemcpyDeviceToDevice, c.stream));
        }
    }
    sync(c);
    return in;
}

// Client side: the normalisers of the division, 1 / d_j with d_j = ||S_j - mean(S_j)||^2 / 4 (an upper
// bound of den_j: w <= 1/4 and S' = M S is the shortest residual of S_j after projecting out X, whose
// first column is the intercept) at the block start of SNP j, 0 elsewhere and for SNPs with d_j = 0.
// One ciphertext per SNP batch and parity (even SNPs of all batches, then odd), at the denominators'
// depth and at scale Delta / (2 f), f the factor of the denominators' tracked scale (4, or 16 for
// kappa = 1), so that Re(den) v lands on the canonical scale.
Ct pack_normalisers(ckks_ctx &c, const uint8_t *S, int n, int m, int kappa, u64 enc_seed) {
    const Layout lay = make_layout(c.p.n, n, 1, m);
    const int dd = circuit_levels(kappa);
    if (c.p.levels < dd) throw Error(CKKS_E_LEVEL, "chain shorter than the circuit");
    const double f = kappa == 1 ? 4.0 / kWKappa1 : 4.0;
    const double sc = c.p.scales[dd] / (2.0 * f);
    std::vector<double> inv_d(m, 0.0);
    for (int j = 0; j < m; ++j) {
        double mean = 0;
        for (int r = 0; r < n; ++r) mean += (double)S[(size_t)r * m + j];
        mean /= n;
        double ss = 0;
        for (int r = 0; r < n; ++r) {
            const double t = (double)S[(size_t)r * m + j] - mean;
            ss += t * t;
        }
        const double d = 0.25 * ss;
        inv_d[j] = d > 0 ? 1.0 / d : 0.0;
    }
    const int N = c.p.n, slots = N / 2, nb = lay.n_batches;
    Ct v = new_ct(c, 2 * nb, dd, sc);
    const size_t per = (size_t)2 * v->limbs * N;
    std::vector<double> re(slots);
    std::vector<i64> poly(N);
    for (int par = 0; par < 2; ++par)
        for (int b = 0; b < nb; ++b) {
            std::fill(re.begin(), re.end(), 0.0);
            for (int cb = 0; cb < lay.blocks; ++cb) {
                const int j = b * lay.tau + 2 * cb + par;
                if (j < m) re[(size_t)cb * lay.R] = inv_d[j];
            }
            encode_poly(N, re.data(), nullptr, slots, sc, poly.data());
            const int i = par * nb + b;
            Ct one = encrypt(c, poly.data(), dd, sc, input_seed(enc_seed, (1ULL << 20) + (u64)i));
            GCK_HIP(hipMemcpyAsync(v->data.ptr + (size_t)i * per, one->data.ptr, per * 8, hipMemcpyDeviceToDevice,
                                   c.stream));
        }
    sync(c);
    return v;
}

// ---------------------------------------------------------------- HIP graph of one input shape

static void same_shape(const EncInput &a, const EncInput &b) {
    const Layout &x = a.lay, &y = b.lay;
    if (x.n != y.n || x.k != y.k || x.m != y.m || x.R != y.R || a.kappa != b.kappa || !a.S || !b.S ||
        a.S->count != b.S->count || a.S->depth != b.S->depth || a.S->scale != b.S->scale || !!a.S_rep != !!b.S_rep)
        throw Error(CKKS_E_PARAM_MISMATCH, "input of another shape than the captured one");
}

static void copy_into(ckks_ctx &c, ckks_ct &dst, const ckks_ct &src) {
    if (dst.count != src.count || dst.depth != src.depth || dst.scale != src.scale)
        throw Error(CKKS_E_PARAM_MISMATCH, "input ciphertext of another shape, depth or scale");
    GCK_HIP(hipMemcpyAsync(dst.data.ptr, src.data.ptr, src.data.words * 8, hipMemcpyDeviceToDevice, c.stream));
}

std::unique_ptr<gwas_graph> capture_circuit(ckks_ctx &c, const EncInput &in, int chunk) {
    if (in.S_host) throw Error(CKKS_E_INVALID_ARG, "a spilled input cannot be captured");
    if (c.pool->budget) throw Error(CKKS_E_INVALID_ARG, "graph capture needs a context without a pool budget");
    if (c.timer.on) throw Error(CKKS_E_INVALID_ARG, "kernel timing is on");
    if (!c.stream) throw Error(CKKS_E_INVALID_ARG, "graph capture needs a context on its own stream");
    auto g = std::make_unique<gwas_graph>();
    g->ctx = &c;
    g->chunk = chunk;
    g->slot = std::make_unique<EncInput>();
    EncInput &sl = *g->slot;
    sl.lay = in.lay;
    sl.kappa = in.kappa;
    for (auto &x : in.x) sl.x.push_back(clone(c, *x));
    sl.y = clone(c, *in.y);
    for (auto &a : in.A) sl.A.push_back(clone(c, *a));
    sl.S = clone(c, *in.S);
    if (in.Xrep) sl.Xrep = clone(c, *in.Xrep);
    if (in.S_rep) sl.S_rep = clone(c, *in.S_rep);
    {
        // one call outside the capture: creates the second stream and its pool, fills the mask cache and
        // leaves every block size the call takes in the pools' free lists
        EncOutput warm;
        run_circuit(c, sl, warm, chunk);
    }
    sync(c);
    if (c.aux_stream) GCK_HIP(hipStreamSynchronize(c.aux_stream));
    g->out = std::make_unique<gwas_enc_output>();
    g->out->ctx = &c;
    g->out->lay = sl.lay;
    g->out->out.chunk = chunk;
    c.pool->capture_begin();
    if (c.aux_pool) c.aux_pool->capture_begin();
    c.capturing = true;
    GCK_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
    try {
        run_circuit(c, sl, g->out->out, chunk);
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(c.stream, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        c.capturing = false;
        g->main_blocks = c.pool->capture_end();
        if (c.aux_pool) g->aux_blocks = c.aux_pool->capture_end();
        throw;
    }
    c.capturing = false;
    hipError_t e = hipStreamEndCapture(c.stream, &g->graph);
    g->main_blocks = c.pool->capture_end();
    if (c.aux_pool) g->aux_blocks = c.aux_pool->capture_end();
    GCK_HIP(e);
    GCK_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    return g;
}

void graph_set_input(gwas_graph &g, const EncInput &in) {
    ckks_ctx &c = *g.ctx;
    EncInput &sl = *g.slot;
    same_shape(sl, in);
    if (in.S_host) throw Error(CKKS_E_INVALID_ARG, "a spilled input cannot be replayed");
    for (size_t j = 0; j < sl.x.size(); ++j) copy_into(c, *sl.x[j], *in.x[j]);
    copy_into(c, *sl.y, *in.y);
    for (size_t a = 0; a < sl.A.size(); ++a) copy_into(c, *sl.A[a], *in.A[a]);
    copy_into(c, *sl.S, *in.S);
    if (sl.Xrep) copy_into(c, *sl.Xrep, *in.Xrep);
    if (sl.S_rep) copy_into(c, *sl.S_rep, *in.S_rep);
}

void graph_launch(gwas_graph &g) { GCK_HIP(hipGraphLaunch(g.exec, g.ctx->stream)); }

// ---------------------------------------------------------------- autotuner

std::tuple<int, int, int, int> schedule_key(const EncInput &in) {
    return std::make_tuple(in.lay.R, in.lay.k, in.kappa, in.S->count);
}

// Times every candidate schedule on the job itself (HIP events on the context's stream around whole calls,
// after one untimed call per candidate) and keeps the fastest for the job's shape.  Candidates: SNP-batch
// chunks of all batches (at most 64), 32, 16 and 8, each on two streams and on one, each with the
// covariates' products stacked (up to 256 ciphertexts) and not; every one computes the same operations on
// the same ciphertexts, so the outputs are bit-identical (tested).
TuneResult tune_circuit(ckks_ctx &c, const EncInput &in, int reps) {
    if (c.timer.on) throw Error(CKKS_E_INVALID_ARG, "kernel timing is on");
    const int nb = in.S->count;
    std::vector<int> chunks;
    for (int ch : {std::min(64, nb), 32, 16, 8})
        if (ch >= 1 && ch <= nb && std::find(chunks.begin(), chunks.end(), ch) == chunks.end()) chunks.push_back(ch);
    const int saved_streams = c.n_streams, saved_stack = c.stack_cts;
    hipEvent_t e0, e1;
    GCK_HIP(hipEventCreate(&e0));
    GCK_HIP(hipEventCreate(&e1));
    TuneResult res;
    res.best.ms = 1e300;
    try {
        for (int streams : {2, 1})
            for (int ch : chunks)
                for (int stack : {0, 256}) {
                    c.n_streams = streams;
                    c.stack_cts = stack;
                    {
                        EncOutput warm;
                        run_circuit(c, in, warm, ch);
                    }
                    double best = 1e300;
                    for (int r = 0; r < std::max(1, reps); ++r) {
                        EncOutput o;
                        GCK_HIP(hipEventRecord(e0, c.stream));
                        run_circuit(c, in, o, ch);
                        GCK_HIP(hipEventRecord(e1, c.stream));
                        GCK_HIP(hipEventSynchronize(e1));
                        float ms = 0;
                        GCK_HIP(hipEventElapsedTime(&ms, e0, e1));
                        best = std::min(best, (double)ms);
                    }
                    ++res.candidates;
                    if (streams == 2 && ch == chunks[0] && stack == 0) res.ms_default = best;
                    if (best < res.best.ms) res.best = ckks_ctx::Schedule{ch, streams, stack, best};
                }
    } catch (...) {
        c.n_streams = saved_streams;
        c.stack_cts = saved_stack;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    c.n_streams = saved_streams;
    c.stack_cts = saved_stack;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.tuned[schedule_key(in)] = res.best;
    return res;
}

int m_xrep_depth(int kappa) { return snp_depth(kappa) + 1; }
int m_srep_depth(int kappa) { return snp_depth(kappa) + 2; }

// Attach the REP inputs of the M-materialised layout: xrep as the client encrypts it (sample-major,
// [i][j]), reordered to column-major [j][i]; srep batch-major [b][i].
void attach_m(ckks_ctx &c, EncInput &in, Ct xrep_row_major, Ct srep) {
    const Layout &lay = in.lay;
    const int n = lay.n, k = lay.k;
    if (xrep_row_major->count != n * k || xrep_row_major->depth != m_xrep_depth(in.kappa))
        throw Error(CKKS_E_INVALID_ARG, "X^T in REP form: n k ciphertexts at the SNP depth + 1");
    if (srep->count != lay.n_batches * n || srep->depth != m_srep_depth(in.kappa))
        throw Error(CKKS_E_INVALID_ARG, "REP SNP rows: n per SNP batch at the SNP depth + 2");
    if (c.p.n < 2 * lay.R) throw Error(CKKS_E_INVALID_ARG, "ring too small");
    Ct xr = new_ct(c, n * k, xrep_row_major->depth, xrep_row_major->scale);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < n; ++i) copy_ct(c, *xr, j * n + i, *xrep_row_major, i * k + j);
    in.Xrep = std::move(xr);
    in.S_rep = std::move(srep);
}

// Client side of the M-materialised layout: X_ij replicated over every slot (the exact constant encoding,
// at the SNP depth + 1 and its canonical scale) and row i of every SNP batch with each entry over its block of R slots (two SNPs
// per complex slot, depth snp_depth + 2); input ciphertext i of this part is encrypted with seed
// output_{2^21 + i}(SplitMix64(enc_seed)), sample-major for X, batch-major for S.
void pack_encrypt_m(ckks_ctx &c, EncInput &in, const double *X, const uint8_t *S, u64 enc_seed) {
    const Layout &lay = in.lay;
    const int N = c.p.n, slots = N / 2, n = lay.n, k = lay.k, m = lay.m;
    const int dx = m_xrep_depth(in.kappa), dsr = m_srep_depth(in.kappa);
    if (c.p.levels < circuit_levels(in.kappa)) throw Error(CKKS_E_LEVEL, "chain too short for kappa");
    Ct xr = new_ct(c, n * k, dx, c.p.scales[dx]);
    Ct sr = new_ct(c, lay.n_batches * n, dsr, c.p.scales[dsr]);
    std::vector<i64> poly(N);
    u64 idx = 2ULL << 20;
    const size_t per_x = (size_t)2 * xr->limbs * N, per_s = (size_t)2 * sr->limbs * N;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) {
            std::fill(poly.begin(), poly.end(), 0);
            poly[0] = round_half_away(X[(size_t)i * k + j] * c.p.scales[dx]);
            Ct one = encrypt(c, poly.data(), dx, c.p.scales[dx], input_seed(enc_seed, idx++));
            GCK_HIP(hipMemcpyAsync(xr->data.ptr + (size_t)(i * k + j) * per_x, one->data.ptr, per_x * 8,
                                   hipMemcpyDeviceToDevice, c.stream));
        }
    // host encodings of up to 256 REP rows at a time in parallel, then their encryptions in order
    const int total = lay.n_batches * n, group = 256;
    std::vector<std::vector<i64>> polys(std::min(group, total), std::vector<i64>(N));
    for (int q0 = 0; q0 < total; q0 += group) {
        const int cnt = std::min(group, total - q0);
        parallel_for(cnt, [&](int t) {
            const int b = (q0 + t) / n, i = (q0 + t) % n;
            std::vector<double> vre(slots, 0.0), vim(slots, 0.0);
            for (int cb = 0; cb < lay.blocks; ++cb) {
                const int j0 = b * lay.tau + 2 * cb;
                const double vr = j0 < m ? (double)S[(size_t)i * m + j0] : 0.0;
                const double vi = j0 + 1 < m ? (double)S[(size_t)i * m + j0 + 1] : 0.0;
                for (int r = 0; r < lay.R; ++r) {
                    vre[(size_t)cb * lay.R + r] = vr;
                    vim[(size_t)cb * lay.R + r] = vi;
                }
            }
            encode_poly(N, vre.data(), vim.data(), slots, c.p.scales[dsr], polys[t].data());
        });
        for (int t = 0; t < cnt; ++t) {
            Ct one = encrypt(c, polys[t].data(), dsr, c.p.scales[dsr], input_seed(enc_seed, idx++));
            GCK_HIP(hipMemcpyAsync(sr->data.ptr + (size_t)(q0 + t) * per_s, one->data.ptr, per_s * 8,
                                   hipMemcpyDeviceToDevice, c.stream));
        }
    }
    sync(c);
    in.Xrep = std::move(xr);
    Ct xr_col = new_ct(c, n * k, dx, c.p.scales[dx]);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < n; ++i) copy_ct(c, *xr_col, j * n + i, *in.Xrep, i * k + j);
    in.Xrep = std::move(xr_col);
    in.S_rep = std::move(sr);
}

}  // namespace gck

gwas_graph::~gwas_graph() {
    if (ctx) {
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->aux_stream) (void)hipStreamSynchronize(ctx->aux_stream);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    out.reset();    // its blocks go back to the pools they came from
    slot.reset();
    if (ctx) {
        // the reserved blocks came from the main pool or the second stream's pool (ensure_aux made it)
        ctx->pool->give_back(main_blocks);
        if (ctx->aux_pool) ctx->aux_pool->give_back(aux_blocks);
    }
}
