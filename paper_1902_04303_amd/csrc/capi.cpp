// extern "C" boundary of the library (include/gwas_ckks.h).  Every entry point catches all C++
// exceptions and turns them into a CKKS_E_* code with a thread-local message.
#include <cmath>
#include <cstring>

#include "gwas.h"

using namespace gck;

namespace {

thread_local std::string g_err;

}  // namespace

namespace gck {
void set_last_error(const std::string &s) { g_err = s; }
}  // namespace gck

namespace {

template <typename F>
int guard(F &&f) {
    try {
        f();
        return CKKS_OK;
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host out of memory";
        return CKKS_E_NOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return CKKS_E_INVALID_ARG;
    }
}

// guard() for entry points that use a context: also holds the context's lock
template <typename F>
int guard_ctx(const ckks_ctx *ctx, F &&f) {
    if (!ctx) {
        g_err = "null context";
        return CKKS_E_INVALID_ARG;
    }
    std::lock_guard<std::recursive_mutex> lk(const_cast<ckks_ctx *>(ctx)->mu);
    return guard(std::forward<F>(f));
}

void need(bool cond, const char *msg) {
    if (!cond) throw Error(CKKS_E_INVALID_ARG, msg);
}

u64 mont_inv64(u64 q) {
    u64 inv = q;   // Newton iteration for q^-1 mod 2^64 (q odd)
    for (int i = 0; i < 6; ++i) inv *= 2 - q * inv;
    return ~inv + 1;
}

u64 shoup_of(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

int bit_reverse(int x, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b)
        if (x & (1 << b)) r |= 1 << (bits - 1 - b);
    return r;
}

LimbScale limb_scale(u64 w, u64 q) { return LimbScale{w, shoup_of(w, q), (double)w}; }

ConvEntry conv_entry(int src, int nsrc, int chain, const u64 *cs, u64 q, const std::vector<u64> &src_mods,
                     bool centre = false) {
    ConvEntry e{};
    e.src = src;
    e.nsrc = nsrc;
    e.chain = chain;
    e.big = 0;
    e.centre = centre ? 1 : 0;
    for (int m = 0; m < nsrc; ++m) {
        e.c[m] = cs[m] % q;
        e.c_sh[m] = shoup_of(e.c[m], q);
        e.cd[m] = (double)e.c[m];
        if (src_mods[m] >= (1ULL << 47)) e.big |= 1 << m;   // source m's residues need splitting
        e.half[m] = src_mods[m] >> 1;
        e.negsq[m] = (q - src_mods[m] % q) % q;
        e.sqd[m] = (double)src_mods[m];
    }
    if (centre && e.big) throw Error(CKKS_E_INVALID_ARG, "centred conversion from a modulus of 2^47 or more");
    return e;
}

// key-switch tables (ModUp conversion per level, digit indices, inverse-NTT scales; ModDown conversion)
void build_ks_tables(ckks_ctx &c) {
    const Params &p = c.p;
    const int L = p.levels, nq = L + 1;
    std::vector<std::vector<ConvEntry>> ups(nq + 1);
    std::vector<std::vector<int>> didx(nq + 1);
    std::vector<std::vector<LimbScale>> scales(nq + 1);
    for (int l = 1; l <= nq; ++l) {
        const int gl = ks_groups(l, p.alpha), nt = l + p.alpha;
        didx[l].assign((size_t)gl * nt, -1);
        scales[l].resize(l);
        for (int b = 0; b < gl; ++b) {
            const int f = ks_group_first(b, p.alpha), m = ks_group_size(b, l, p.alpha);
            std::vector<u64> mods;
            for (int i = f; i < f + m; ++i) mods.push_back(p.q[i]);
            // y_i = d_i (Q_G / q_i)^-1, folded with N^-1 into the inverse NTT
            for (int i = f; i < f + m; ++i) {
                const u64 qi = p.q[i];
                u64 hat = 1;
                for (int j = f; j < f + m; ++j)
                    if (j != i) hat = mulmod_host(hat, p.q[j] % qi, qi);
                const u64 w = mulmod_host(invmod_host((u64)p.n % qi, qi), invmod_host(hat, qi), qi);
                scales[l][i] = limb_scale(w, qi);
            }
            for (int t = 0; t < nt; ++t) {
                if (t < l && t >= f && t < f + m) continue;   // the digit's own primes: the input residue
                const int chain = t < l ? t : L + 1 + (t - l);
                const u64 qt = p.mod(chain);
                u64 cs[kMaxSpecial] = {};
                for (int a = 0; a < m; ++a) {
                    u64 hat = 1;
                    for (int j = f; j < f + m; ++j)
                        if (j != f + a) hat = mulmod_host(hat, p.q[j] % qt, qt);
                    cs[a] = hat;
                }
                didx[l][(size_t)b * nt + t] = (int)ups[l].size();
                ups[l].push_back(conv_entry(f, m, chain, cs, qt, mods));
            }
        }
    }
    // ModDown: C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k); (P/p_k)^-1 and N^-1 folded into the special limbs'
    // inverse NTT, P/p_k mod q_i into the conversion, P^-1 mod q_i into the final store
    const int a = p.alpha;
    std::vector<ConvEntry> down(nq);
    for (int i = 0; i < nq; ++i) {
        u64 cs[kMaxSpecial] = {};
        for (int k = 0; k < a; ++k) {
            u64 hat = 1;
            for (int j = 0; j < a; ++j)
                if (j != k) hat = mulmod_host(hat, p.P[j] % p.q[i], p.q[i]);
            cs[k] = hat;
        }
        down[i] = conv_entry(0, a, i, cs, p.q[i], p.P, true);
    }
    std::vector<LimbScale> dscale(a);
    for (int k = 0; k < a; ++k) {
        const u64 pk = p.P[k];
        u64 hat = 1;
        for (int j = 0; j < a; ++j)
            if (j != k) hat = mulmod_host(hat, p.P[j] % pk, pk);
        dscale[k] = limb_scale(mulmod_host(invmod_host((u64)p.n % pk, pk), invmod_host(hat, pk), pk), pk);
    }
    for (int i = 0; i < p.n_mods(); ++i) {
        const u64 q = p.mod(i);
        u64 pm = 1;
        for (int k = 0; k < a; ++k) pm = mulmod_host(pm, p.P[k] % q, q);
        c.p_inv.v[i] = pm ? invmod_host(pm, q) : 0;
        c.p_inv.sh[i] = shoup_of(c.p_inv.v[i], q);
    }
    // fused relinearisation and rescale by q_j: B = P q_j with moduli b = (q_j, p_1 .. p_alpha);
    // C = sum_b [x (B/b)^-1]_b (B/b), the scales (B/b)^-1 and N^-1 folded into the inverse NTT of those
    // limbs, B/b mod q_i into the conversion to the remaining q_i (i < j), B^-1 mod q_i into the final store
    std::vector<std::vector<ConvEntry>> rconv(nq);
    std::vector<std::vector<LimbScale>> rscale(nq);
    std::vector<u64> binv((size_t)nq * 3 * kMaxMods, 0);   // [j][v, sh, d][kMaxMods]
    for (int j = 1; j < nq; ++j) {
        std::vector<u64> bm(1, p.q[j]);
        bm.insert(bm.end(), p.P.begin(), p.P.end());
        const int nb = a + 1;
        for (int k = 0; k < nb; ++k) {
            u64 hat = 1;
            for (int m = 0; m < nb; ++m)
                if (m != k) hat = mulmod_host(hat, bm[m] % bm[k], bm[k]);
            rscale[j].push_back(
                limb_scale(mulmod_host(invmod_host((u64)p.n % bm[k], bm[k]), invmod_host(hat, bm[k]), bm[k]), bm[k]));
        }
        for (int i = 0; i < j; ++i) {
            u64 cs[kMaxSpecial] = {};
            for (int k = 0; k < nb; ++k) {
                u64 hat = 1;
                for (int m = 0; m < nb; ++m)
                    if (m != k) hat = mulmod_host(hat, bm[m] % p.q[i], p.q[i]);
                cs[k] = hat;
            }
            rconv[j].push_back(conv_entry(0, nb, i, cs, p.q[i], bm, true));
        }
        u64 *v = &binv[(size_t)j * 3 * kMaxMods], *sh = v + kMaxMods;
        double *d = reinterpret_cast<double *>(sh + kMaxMods);
        for (int i = 0; i < j; ++i) {
            const u64 q = p.q[i];
            u64 bq = p.q[j] % q;   // B mod q_i
            for (int k = 0; k < a; ++k) bq = mulmod_host(bq, p.P[k] % q, q);
            v[i] = invmod_host(bq, q);
            sh[i] = shoup_of(v[i], q);
            d[i] = (double)v[i];
        }
    }
    // one device block for everything
    size_t bytes = 0;
    auto room = [&](size_t b) { size_t o = bytes; bytes += (b + 255) / 256 * 256; return o; };
    std::vector<size_t> o_up(nq + 1), o_didx(nq + 1), o_sc(nq + 1);
    for (int l = 1; l <= nq; ++l) {
        o_up[l] = room(ups[l].size() * sizeof(ConvEntry));
        o_didx[l] = room(didx[l].size() * sizeof(int));
        o_sc[l] = room(scales[l].size() * sizeof(LimbScale));
    }
    const size_t o_down = room(down.size() * sizeof(ConvEntry)), o_dsc = room(dscale.size() * sizeof(LimbScale));
    const size_t o_pinv = room(kMaxMods * 8), o_pinv_sh = room(kMaxMods * 8), o_pinv_d = room(kMaxMods * 8);
    const size_t o_qinv = room((size_t)nq * 3 * kMaxMods * 8);   // [j][v, sh, d][kMaxMods]
    std::vector<size_t> o_rconv(nq), o_rscale(nq);
    for (int j = 1; j < nq; ++j) {
        o_rconv[j] = room(rconv[j].size() * sizeof(ConvEntry));
        o_rscale[j] = room(rscale[j].size() * sizeof(LimbScale));
    }
    const size_t o_binv = room(binv.size() * 8);
    GCK_HIP(hipMalloc(&c.ks_mem, bytes));
    char *base = static_cast<char *>(c.ks_mem);
    c.ks_levels.assign(nq + 1, ckks_ctx::KsLevel{});
    for (int l = 1; l <= nq; ++l) {
        auto &kl = c.ks_levels[l];
        kl.K = (int)ups[l].size();
        kl.up = reinterpret_cast<ConvEntry *>(base + o_up[l]);
        kl.didx = reinterpret_cast<int *>(base + o_didx[l]);
        kl.up_scale = reinterpret_cast<LimbScale *>(base + o_sc[l]);
        GCK_HIP(hipMemcpy(kl.up, ups[l].data(), ups[l].size() * sizeof(ConvEntry), hipMemcpyHostToDevice));
        GCK_HIP(hipMemcpy(kl.didx, didx[l].data(), didx[l].size() * sizeof(int), hipMemcpyHostToDevice));
        GCK_HIP(hipMemcpy(kl.up_scale, scales[l].data(), scales[l].size() * sizeof(LimbScale), hipMemcpyHostToDevice));
    }
    c.down_conv = reinterpret_cast<ConvEntry *>(base + o_down);
    c.down_scale = reinterpret_cast<LimbScale *>(base + o_dsc);
    GCK_HIP(hipMemcpy(c.down_conv, down.data(), down.size() * sizeof(ConvEntry), hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.down_scale, dscale.data(), dscale.size() * sizeof(LimbScale), hipMemcpyHostToDevice));
    c.p_inv_dev = reinterpret_cast<u64 *>(base + o_pinv);
    c.p_inv_sh_dev = reinterpret_cast<u64 *>(base + o_pinv_sh);
    GCK_HIP(hipMemcpy(c.p_inv_dev, c.p_inv.v, kMaxMods * 8, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.p_inv_sh_dev, c.p_inv.sh, kMaxMods * 8, hipMemcpyHostToDevice));
    std::vector<double> pinv_d(kMaxMods, 0.0);
    for (int i = 0; i < p.n_mods(); ++i) pinv_d[i] = (double)c.p_inv.v[i];
    c.p_inv_d_dev = reinterpret_cast<double *>(base + o_pinv_d);
    GCK_HIP(hipMemcpy(c.p_inv_d_dev, pinv_d.data(), kMaxMods * 8, hipMemcpyHostToDevice));
    // rescale constants: q_j^-1 mod q_i (j the dropped prime)
    std::vector<u64> qinv((size_t)nq * 3 * kMaxMods, 0);
    c.q_inv.assign(nq, ckks_ctx::QInv{});
    for (int j = 1; j < nq; ++j) {
        u64 *v = &qinv[(size_t)j * 3 * kMaxMods], *sh = v + kMaxMods;
        double *d = reinterpret_cast<double *>(sh + kMaxMods);
        for (int i = 0; i < p.n_mods(); ++i) {
            const u64 q = p.mod(i), x = p.q[j] % q;
            v[i] = x ? invmod_host(x, q) : 0;
            sh[i] = shoup_of(v[i], q);
            d[i] = (double)v[i];
        }
        u64 *dev = reinterpret_cast<u64 *>(base + o_qinv) + (size_t)j * 3 * kMaxMods;
        c.q_inv[j] = ckks_ctx::QInv{dev, dev + kMaxMods, reinterpret_cast<double *>(dev + 2 * kMaxMods)};
    }
    GCK_HIP(hipMemcpy(base + o_qinv, qinv.data(), qinv.size() * 8, hipMemcpyHostToDevice));
    c.rs_levels.assign(nq, ckks_ctx::RsLevel{});
    for (int j = 1; j < nq; ++j) {
        auto &rl = c.rs_levels[j];
        rl.conv = reinterpret_cast<ConvEntry *>(base + o_rconv[j]);
        rl.scale = reinterpret_cast<LimbScale *>(base + o_rscale[j]);
        GCK_HIP(hipMemcpy(rl.conv, rconv[j].data(), rconv[j].size() * sizeof(ConvEntry), hipMemcpyHostToDevice));
        GCK_HIP(hipMemcpy(rl.scale, rscale[j].data(), rscale[j].size() * sizeof(LimbScale), hipMemcpyHostToDevice));
        u64 *dev = reinterpret_cast<u64 *>(base + o_binv) + (size_t)j * 3 * kMaxMods;
        rl.binv = dev;
        rl.binv_sh = dev + kMaxMods;
        rl.binv_d = reinterpret_cast<double *>(dev + 2 * kMaxMods);
    }
    GCK_HIP(hipMemcpy(base + o_binv, binv.data(), binv.size() * 8, hipMemcpyHostToDevice));
    c.ng = ks_groups(nq, p.alpha);
}

void build_tables(ckks_ctx &c) {
    const int n = c.p.n, n_mods = c.p.n_mods();
    const size_t N = (size_t)n;
    std::vector<u64> psi(N * n_mods), psi_sh(N * n_mods), ipsi(N * n_mods), ipsi_sh(N * n_mods);
    std::vector<double> psi_f(N * n_mods), ipsi_f(N * n_mods);
    c.h_mods.resize(n_mods);
    for (int mi = 0; mi < n_mods; ++mi) {
        const u64 q = c.p.mod(mi);
        const u64 root = find_psi(q, n), iroot = invmod_host(root, q);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (size_t i = 1; i < N; ++i) {
            pw[i] = mulmod_host(pw[i - 1], root, q);
            ipw[i] = mulmod_host(ipw[i - 1], iroot, q);
        }
        for (int k = 0; k < n; ++k) {
            int br = bit_reverse(k, c.p.log_n);
            psi[mi * N + k] = pw[br];
            psi_sh[mi * N + k] = shoup_of(pw[br], q);
            ipsi[mi * N + k] = ipw[br];
            ipsi_sh[mi * N + k] = shoup_of(ipw[br], q);
            psi_f[mi * N + k] = (double)pw[br];
            ipsi_f[mi * N + k] = (double)ipw[br];
        }
        ModInfo &M = c.h_mods[mi];
        M.q = q;
        M.mont_inv = mont_inv64(q);
        M.barrett = (u64)(((u128)1 << 64) / q);
        M.r_mod = (u64)(((u128)1 << 64) % q);
        M.r_mod_sh = shoup_of(M.r_mod, q);
        M.r2_mod = mulmod_host(M.r_mod, M.r_mod, q);
        M.ninv = invmod_host((u64)n % q, q);
        M.ninv_sh = shoup_of(M.ninv, q);
        M.w1ninv = mulmod_host(ipsi[mi * N + 1], M.ninv, q);
        M.w1ninv_sh = shoup_of(M.w1ninv, q);
        M.fp = q < ((u64)1 << kFpModBits) ? 1 : 0;
        M.qd = (double)q;
        M.qinv = 1.0 / (double)q;
        M.ninv_d = (double)M.ninv;
        M.rinv_d = (double)invmod_host(M.r_mod, q);
        M.c32_d = (double)(((u64)1 << 32) % q);
    }
    const size_t mods_bytes = ((sizeof(ModInfo) * n_mods + 255) / 256) * 256;
    const size_t tab_bytes = N * n_mods * 8;
    GCK_HIP(hipMalloc(&c.table_mem, mods_bytes + 6 * tab_bytes));
    char *base = static_cast<char *>(c.table_mem);
    c.tab.mods = reinterpret_cast<ModInfo *>(base);
    c.tab.psi = reinterpret_cast<u64 *>(base + mods_bytes);
    c.tab.psi_sh = reinterpret_cast<u64 *>(base + mods_bytes + tab_bytes);
    c.tab.ipsi = reinterpret_cast<u64 *>(base + mods_bytes + 2 * tab_bytes);
    c.tab.ipsi_sh = reinterpret_cast<u64 *>(base + mods_bytes + 3 * tab_bytes);
    c.tab.psi_f = reinterpret_cast<double *>(base + mods_bytes + 4 * tab_bytes);
    c.tab.ipsi_f = reinterpret_cast<double *>(base + mods_bytes + 5 * tab_bytes);
    c.tab.n = n;
    c.tab.log_n = c.p.log_n;
    c.tab.n_mods = n_mods;
    GCK_HIP(hipMemcpy(c.tab.mods, c.h_mods.data(), sizeof(ModInfo) * n_mods, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.psi, psi.data(), tab_bytes, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.psi_sh, psi_sh.data(), tab_bytes, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.ipsi, ipsi.data(), tab_bytes, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.ipsi_sh, ipsi_sh.data(), tab_bytes, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.psi_f, psi_f.data(), tab_bytes, hipMemcpyHostToDevice));
    GCK_HIP(hipMemcpy(c.tab.ipsi_f, ipsi_f.data(), tab_bytes, hipMemcpyHostToDevice));
}

Ct wrap(Ct r) { return r; }

ckks_ct *release(Ct r) { return r.release(); }

// Freeing returns device buffers to the context's pool, which a server's worker thread may be using: hold
// the context's lock (the pools' free lists are not thread-safe on their own).
template <typename T>
void free_locked(ckks_ctx *c, T *p) {
    if (!p) return;
    if (!c) {
        delete p;
        return;
    }
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    delete p;
}

void check_ct(const ckks_ctx *ctx, const ckks_ct *a) {
    need(ctx && a, "null handle");
    if (a->ctx != ctx) throw Error(CKKS_E_PARAM_MISMATCH, "ciphertext belongs to another context");
}

}  // namespace

extern "C" {

const char *ckks_last_error(void) { return g_err.c_str(); }

int ckks_params_ks_alpha(const ckks_params *params) {
    if (!params) return CKKS_E_INVALID_ARG;
    const int a = params->ks_alpha == 0 ? CKKS_DEFAULT_KS_ALPHA : params->ks_alpha;
    return (a >= 2 && a <= kMaxAlpha) ? a : CKKS_E_INVALID_ARG;
}

int ckks_chain(const ckks_params *params, uint64_t *moduli, double *scales) {
    return guard([&] {
        need(params && moduli && scales, "null argument");
        Params p = make_params(params->log_n, params->levels, params->log2_scale, params->ks_alpha);
        for (int i = 0; i < p.n_mods(); ++i) moduli[i] = p.mod(i);
        for (int i = 0; i <= p.levels; ++i) scales[i] = p.scales[i];
    });
}

int ckks_ctx_create(const ckks_params *params, const ckks_allocator *allocator, void *hip_stream,
                    size_t pool_budget_bytes, ckks_ctx **out) {
    return guard([&] {
        need(params && out, "null argument");
        *out = nullptr;
        auto c = std::make_unique<ckks_ctx>();
        c->p = make_params(params->log_n, params->levels, params->log2_scale, params->ks_alpha);
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->pool = std::make_unique<Pool>(allocator, pool_budget_bytes);
        c->pool->stream = c->stream;
        build_tables(*c);
        build_ks_tables(*c);
        noalloc_init();
        c->tab.timer = &c->timer;
        *out = c.release();
    });
}

void ckks_ctx_destroy(ckks_ctx *ctx) { delete ctx; }

int ckks_ctx_moduli(const ckks_ctx *ctx, uint64_t *moduli, int cap) {
    return guard_ctx(ctx, [&] {
        need(ctx && moduli && cap >= ctx->p.n_mods(), "bad buffer");
        for (int i = 0; i < ctx->p.n_mods(); ++i) moduli[i] = ctx->p.mod(i);
    });
}

int ckks_ctx_scales(const ckks_ctx *ctx, double *scales, int cap) {
    return guard_ctx(ctx, [&] {
        need(ctx && scales && cap >= ctx->p.levels + 1, "bad buffer");
        for (int i = 0; i <= ctx->p.levels; ++i) scales[i] = ctx->p.scales[i];
    });
}

int ckks_ctx_pool_stats(const ckks_ctx *ctx, size_t *in_use, size_t *cached, size_t *peak, size_t *n_alloc) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        const Pool *a = ctx->aux_pool.get();   // the auxiliary stream's pool, when it exists
        if (in_use) *in_use = ctx->pool->in_use + (a ? a->in_use : 0);
        if (cached) *cached = ctx->pool->cached + (a ? a->cached : 0);
        if (peak) *peak = ctx->pool->peak + (a ? a->peak : 0);
        if (n_alloc) *n_alloc = ctx->pool->n_alloc + (a ? a->n_alloc : 0);
    });
}

int ckks_ctx_pool_trim(ckks_ctx *ctx) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        if (ctx->aux_stream) GCK_HIP(hipStreamSynchronize(ctx->stream));   // main-stream readers of aux buffers
        ctx->pool->trim();
        if (ctx->aux_pool) ctx->aux_pool->trim();
    });
}

int ckks_ctx_counters(const ckks_ctx *ctx, uint64_t *keyswitches, uint64_t *limb_ntts, uint64_t *launches) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        if (keyswitches) *keyswitches = ctx->n_keyswitch;
        if (limb_ntts) *limb_ntts = ctx->n_limb_ntt;
        if (launches) *launches = ctx->n_launch;
    });
}

int ckks_ctx_keyswitch_ciphertexts(const ckks_ctx *ctx, uint64_t *n) {
    return guard_ctx(ctx, [&] {
        need(n, "null argument");
        *n = ctx->n_keyswitch_ct;
    });
}

int ckks_ctx_kernel_timing(ckks_ctx *ctx, int enable) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        if (enable) ctx->timer.reset();
        else ctx->timer.collect();
        ctx->timer.on = enable != 0;
    });
}

int ckks_ctx_kernel_timing_only(ckks_ctx *ctx, const char *name) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        ctx->timer.collect();
        ctx->timer.only = name ? name : "";
    });
}

int ckks_ctx_set_streams(ckks_ctx *ctx, int n) {
    return guard_ctx(ctx, [&] {
        need(ctx && (n == 1 || n == 2), "streams must be 1 or 2");
        ctx->n_streams = n;
    });
}

int ckks_ctx_set_stack(ckks_ctx *ctx, int n) {
    return guard_ctx(ctx, [&] {
        need(ctx && n >= 0, "stack size must be 0 or more");
        ctx->stack_cts = n;
    });
}

int ckks_ctx_kernel_report(ckks_ctx *ctx, char *buf, size_t cap) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf && cap > 0, "bad buffer");
        ctx->timer.collect();
        std::string s;
        char line[256];
        for (size_t i = 0; i < ctx->timer.names.size(); ++i) {
            const auto &st = ctx->timer.stats[i];
            std::snprintf(line, sizeof line, "%s %llu %.6f %.0f %.0f %.0f\n", ctx->timer.names[i].c_str(),
                          (unsigned long long)st.count, st.ms, st.bytes, st.flops, st.pass_bytes);
            s += line;
        }
        need(s.size() + 1 <= cap, "report buffer too small");
        std::memcpy(buf, s.c_str(), s.size() + 1);
    });
}

int ckks_keygen(ckks_ctx *ctx, uint64_t seed, const uint64_t *galois, int n_galois) {
    return guard_ctx(ctx, [&] {
        need(ctx && (n_galois == 0 || galois) && n_galois >= 0, "bad arguments");
        keygen(*ctx, seed, std::vector<u64>(galois, galois + n_galois));
    });
}

uint64_t ckks_galois_rotate(const ckks_ctx *ctx, int64_t r) { return ctx ? galois_rotate(*ctx, r) : 0; }
uint64_t ckks_galois_conj(const ckks_ctx *ctx) { return ctx ? galois_conj(*ctx) : 0; }

int ckks_export_switching_key(ckks_ctx *ctx, uint64_t key_id, uint64_t *buf, size_t cap_words) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf, "null argument");
        auto it = ctx->ksk.find(key_id);
        if (it == ctx->ksk.end()) throw Error(CKKS_E_KEY_MISSING, "no such key");
        const int L = ctx->p.levels, nt = ctx->p.n_mods(), ng = ctx->ng;
        const size_t N = (size_t)ctx->p.n, words = (size_t)2 * ng * nt * N;
        need(cap_words >= words, "buffer too small");
        DBuf t(ctx->pool.get(), words);
        GCK_HIP(hipMemcpyAsync(t.ptr, it->second.ptr, words * 8, hipMemcpyDeviceToDevice, ctx->stream));
        const ModMap mt{nt, L + 1, L + 1};
        k_from_mont(ctx->tab, t.ptr, 2 * ng * nt, mt, ctx->stream);
        ntt_inv(*ctx, t.ptr, 2 * ng * nt, mt);
        GCK_HIP(hipMemcpyAsync(buf, t.ptr, words * 8, hipMemcpyDeviceToHost, ctx->stream));
        sync(*ctx);
    });
}

int ckks_export_secret(ckks_ctx *ctx, int64_t *buf, size_t cap) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf && cap >= (size_t)ctx->p.n, "bad buffer");
        if (!ctx->have_secret) throw Error(CKKS_E_KEY_MISSING, "no secret key in this context");
        std::memcpy(buf, ctx->sk.data(), (size_t)ctx->p.n * 8);
    });
}

int ckks_export_public_key(ckks_ctx *ctx, uint64_t *buf, size_t cap_words) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf, "null argument");
        if (!ctx->have_pk) throw Error(CKKS_E_KEY_MISSING, "no public key in this context");
        const int l = ctx->p.levels + 1;
        const size_t N = (size_t)ctx->p.n, words = (size_t)2 * l * N;
        need(cap_words >= words, "buffer too small");
        DBuf t(ctx->pool.get(), words);
        GCK_HIP(hipMemcpyAsync(t.ptr, ctx->pk.ptr, words * 8, hipMemcpyDeviceToDevice, ctx->stream));
        ntt_inv(*ctx, t.ptr, 2 * l, map_q(l));
        GCK_HIP(hipMemcpyAsync(buf, t.ptr, words * 8, hipMemcpyDeviceToHost, ctx->stream));
        sync(*ctx);
    });
}

int ckks_import_public_key(ckks_ctx *ctx, const uint64_t *buf, size_t words) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf, "null argument");
        need(words == (size_t)2 * (ctx->p.levels + 1) * ctx->p.n, "public key size does not match the parameters");
        import_public_key(*ctx, buf);
    });
}

int ckks_import_switching_key(ckks_ctx *ctx, uint64_t key_id, const uint64_t *buf, size_t words) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf, "null argument");
        need(words == (size_t)2 * ctx->ng * ctx->p.n_mods() * ctx->p.n,
             "switching key size does not match the parameters");
        import_switching_key(*ctx, key_id, buf);
    });
}

int ckks_ctx_has_secret(const ckks_ctx *ctx) { return ctx && ctx->have_secret ? 1 : 0; }

int ckks_encode(ckks_ctx *ctx, const double *re, const double *im, size_t n, double scale, int64_t *coeffs_out) {
    return guard_ctx(ctx, [&] {
        need(ctx && coeffs_out && (re || n == 0), "null argument");
        encode_poly(ctx->p.n, re, im, n, scale, coeffs_out);
    });
}

int ckks_decode(ckks_ctx *ctx, const double *coeffs, double *re, double *im) {
    return guard_ctx(ctx, [&] {
        need(ctx && coeffs, "null argument");
        decode_poly(ctx->p.n, coeffs, re, im);
    });
}

int ckks_encrypt(ckks_ctx *ctx, const int64_t *m, int depth, double scale, uint64_t seed, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && m && out, "null argument");
        need(scale > 0, "scale must be positive");
        *out = release(encrypt(*ctx, m, depth, scale, seed));
    });
}

int ckks_decrypt_poly(ckks_ctx *ctx, const ckks_ct *ct, int index, double *coeffs) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, ct);
        need(coeffs && index >= 0 && index < ct->count, "bad arguments");
        auto v = decrypt_poly(*ctx, *ct, index);
        for (size_t i = 0; i < v.size(); ++i) coeffs[i] = (double)v[i];
    });
}

int ckks_decrypt(ckks_ctx *ctx, const ckks_ct *ct, int index, double *re, double *im) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, ct);
        need(index >= 0 && index < ct->count, "bad index");
        auto v = decrypt_poly(*ctx, *ct, index);
        std::vector<double> m(v.size());
        for (size_t i = 0; i < v.size(); ++i) m[i] = (double)(v[i] / (long double)ct->scale);
        decode_poly(ctx->p.n, m.data(), re, im);
    });
}

int ckks_ct_info(const ckks_ct *ct, int *count, int *depth, int *limbs, double *scale) {
    return guard([&] {
        need(ct, "null handle");
        if (count) *count = ct->count;
        if (depth) *depth = ct->depth;
        if (limbs) *limbs = ct->limbs;
        if (scale) *scale = ct->scale;
    });
}

int ckks_ct_export(ckks_ctx *ctx, const ckks_ct *ct, int index, uint64_t *buf, size_t cap_words) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, ct);
        need(buf && index >= 0 && index < ct->count, "bad arguments");
        need(cap_words >= (size_t)2 * ct->limbs * ctx->p.n, "buffer too small");
        export_ct(*ctx, *ct, index, buf);
    });
}

int ckks_ct_import(ckks_ctx *ctx, const uint64_t *buf, int depth, double scale, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && buf && out, "null argument");
        *out = release(import_ct(*ctx, buf, depth, scale));
    });
}

void ckks_ct_free(ckks_ct *ct) { free_locked(ct ? ct->ctx : nullptr, ct); }

#define CT_UNARY(name, expr)                                   \
    int name(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out) { \
        return guard_ctx(ctx, [&] {                                     \
            check_ct(ctx, a);                                  \
            need(out, "null output");                          \
            *out = release(expr);                              \
        });                                                    \
    }

CT_UNARY(ckks_rescale, rescale(*ctx, *a))
CT_UNARY(ckks_conjugate, conjugate(*ctx, *a))

int ckks_add(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        check_ct(ctx, b);
        need(out, "null output");
        *out = release(add(*ctx, *a, *b));
    });
}

int ckks_sub(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        check_ct(ctx, b);
        need(out, "null output");
        *out = release(sub(*ctx, *a, *b));
    });
}

int ckks_mul(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        check_ct(ctx, b);
        need(out, "null output");
        *out = release(mul(*ctx, *a, *b));
    });
}

int ckks_mul_noalloc(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        check_ct(ctx, b);
        check_ct(ctx, out);
        mul_noalloc(*ctx, *a, *b, *out);
    });
}

int ckks_mul_int(ckks_ctx *ctx, const ckks_ct *a, int64_t k, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(mul_int(*ctx, *a, k));
    });
}

int ckks_add_const(ckks_ctx *ctx, const ckks_ct *a, double v, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(add_const(*ctx, *a, v));
    });
}

int ckks_mul_const(ckks_ctx *ctx, const ckks_ct *a, double v, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(mul_const(*ctx, *a, v));
    });
}

int ckks_align(ckks_ctx *ctx, const ckks_ct *a, int depth, double scale, double factor, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(align(*ctx, *a, depth, scale, factor));
    });
}

int ckks_rotate(ckks_ctx *ctx, const ckks_ct *a, int64_t r, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(rotate(*ctx, *a, r));
    });
}

int ckks_rotate_sum(ckks_ctx *ctx, const ckks_ct *a, const int64_t *rots, int n, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out && rots && n >= 1 && n <= kMaxKeys, "need 1 to 16 rotations and an output");
        *out = release(rotate_sum(*ctx, *a, std::vector<i64>(rots, rots + n)));
    });
}

int ckks_mul_mask(ckks_ctx *ctx, const ckks_ct *a, int R, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        check_ct(ctx, a);
        need(out, "null output");
        *out = release(mul_mask(*ctx, *a, R));
    });
}

int ckks_ntt_device(ckks_ctx *ctx, uint64_t *dev_limbs, int count, const int *moduli_index, int dir) {
    return guard_ctx(ctx, [&] {
        need(ctx && dev_limbs && moduli_index && count >= 0 && (dir == 1 || dir == -1), "bad arguments");
        for (int i = 0; i < count; ++i) need(moduli_index[i] >= 0 && moduli_index[i] < ctx->p.n_mods(),
                                             "modulus index out of range");
        for (int i = 0; i < count;) {   // one launch per run of limbs with the same modulus
            int e = i + 1;
            while (e < count && moduli_index[e] == moduli_index[i]) ++e;
            const ModMap m{1, 0, moduli_index[i]};
            if (dir == 1) ntt_fwd(*ctx, dev_limbs + (size_t)i * ctx->p.n, e - i, m);
            else ntt_inv(*ctx, dev_limbs + (size_t)i * ctx->p.n, e - i, m);
            i = e;
        }
    });
}

int gwas_galois_elements(int log_n, int R, uint64_t *out, int cap, int *count) {
    return guard([&] {
        need(log_n >= 1 && log_n <= 17 && R >= 1 && 2 * R <= (1 << log_n) && count, "bad arguments");
        const std::vector<u64> g = required_galois(1 << log_n, R);
        *count = (int)g.size();
        need(out || cap == 0, "null output");
        for (int i = 0; i < cap && i < (int)g.size(); ++i) out[i] = g[i];
    });
}

int gwas_layout(const ckks_ctx *ctx, int n, int k, int m, int kappa, int *R, int *tau, int *n_batches,
                int *levels_needed) {
    return guard_ctx(ctx, [&] {
        need(ctx, "null context");
        Layout lay = make_layout(ctx->p.n, n, k, m);
        if (R) *R = lay.R;
        if (tau) *tau = lay.tau;
        if (n_batches) *n_batches = lay.n_batches;
        if (levels_needed) *levels_needed = circuit_levels(kappa);
    });
}

int gwas_pack_encrypt(ckks_ctx *ctx, const double *X, const double *y, const uint8_t *S, int n, int k, int m,
                      int kappa, uint64_t enc_seed, gwas_enc_input **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && X && y && S && out, "null argument");
        need(kappa >= 1, "kappa must be >= 1");
        if (ctx->p.levels < circuit_levels(kappa)) throw Error(CKKS_E_LEVEL, "chain too short for kappa");
        auto in = pack_encrypt(*ctx, X, y, S, n, k, m, kappa, enc_seed);
        *out = new gwas_enc_input{ctx, std::move(in)};
    });
}

int gwas_input_from_cts(ckks_ctx *ctx, int n, int k, int m, int kappa, ckks_ct *const *x, const ckks_ct *y,
                        ckks_ct *const *A, ckks_ct *const *S, int n_s, gwas_enc_input **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && x && y && A && S && out, "null argument");
        need(kappa >= 1, "kappa must be >= 1");
        auto in = std::make_unique<EncInput>();
        in->lay = make_layout(ctx->p.n, n, k, m);
        in->kappa = kappa;
        need(n_s == in->lay.n_batches, "wrong number of SNP batches");
        for (int j = 0; j < k; ++j) {
            check_ct(ctx, x[j]);
            in->x.push_back(clone(*ctx, *x[j]));
        }
        check_ct(ctx, y);
        in->y = clone(*ctx, *y);
        for (int i = 0; i < k * (k + 1) / 2; ++i) {
            check_ct(ctx, A[i]);
            in->A.push_back(clone(*ctx, *A[i]));
        }
        const int ds = snp_depth(kappa);
        for (int b = 0; b < n_s; ++b) {
            check_ct(ctx, S[b]);
            if (S[b]->depth != ds || S[b]->count != 1) throw Error(CKKS_E_LEVEL, "SNP batch at the wrong depth");
        }
        in->S = new_ct(*ctx, n_s, ds, S[0]->scale);
        const size_t per = (size_t)2 * in->S->limbs * ctx->p.n;
        for (int b = 0; b < n_s; ++b)
            GCK_HIP(hipMemcpyAsync(in->S->data.ptr + (size_t)b * per, S[b]->data.ptr, per * 8, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        *out = new gwas_enc_input{ctx, std::move(in)};
    });
}

void gwas_input_free(gwas_enc_input *in) { free_locked(in ? in->ctx : nullptr, in); }

int gwas_input_ct(const gwas_enc_input *in, int which, int index, const ckks_ct **ct) {
    return guard([&] {
        need(in && ct, "null argument");
        const EncInput &e = *in->in;
        switch (which) {
        case 0:
            need(index >= 0 && index < (int)e.x.size(), "x index out of range");
            *ct = e.x[index].get();
            return;
        case 1: *ct = e.y.get(); return;
        case 2:
            need(index >= 0 && index < (int)e.A.size(), "A index out of range");
            *ct = e.A[index].get();
            return;
        case 3:
            need(!e.S_host && e.S->data.ptr, "the SNP batches are spilled to the host");
            *ct = e.S.get();
            return;
        default: need(false, "unknown input");
        }
    });
}

int gwas_output_from_cts(ckks_ctx *ctx, int n, int k, int m, ckks_ct *const *num, ckks_ct *const *den_even,
                         ckks_ct *const *den_odd, int n_b, gwas_enc_output **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && num && den_even && den_odd && out, "null argument");
        auto o = std::make_unique<gwas_enc_output>();
        o->ctx = ctx;
        o->lay = make_layout(ctx->p.n, n, k, m);
        need(n_b == o->lay.n_batches, "wrong number of SNP batches");
        auto gather_all = [&](ckks_ct *const *v) {
            std::vector<const ckks_ct *> parts;
            for (int b = 0; b < n_b; ++b) {
                check_ct(ctx, v[b]);
                need(v[b]->count == 1, "one ciphertext per SNP batch");
                parts.push_back(v[b]);
            }
            return stack(*ctx, parts);
        };
        o->out.num.push_back(gather_all(num));
        o->out.den_even.push_back(gather_all(den_even));
        o->out.den_odd.push_back(gather_all(den_odd));
        o->out.chunk = n_b;
        *out = o.release();
    });
}

int gwas_input_spill(ckks_ctx *ctx, gwas_enc_input *in) {
    return guard_ctx(ctx, [&] {
        need(in && in->ctx == ctx, "bad input");
        spill_snp(*ctx, *in->in);
    });
}

int gwas_semiparallel_chunked(ckks_ctx *ctx, const gwas_enc_input *in, int chunk, gwas_enc_output **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && in && out, "null argument");
        need(in->ctx == ctx, "input belongs to another context");
        need(chunk >= 1, "chunk must be >= 1");
        auto o = std::make_unique<gwas_enc_output>();
        o->ctx = ctx;
        o->lay = in->in->lay;
        o->out.chunk = chunk;
        run_circuit(*ctx, *in->in, o->out, chunk);
        *out = o.release();
    });
}

int gwas_semiparallel_multi(ckks_ctx *ctx, const gwas_enc_input *const *in, int n_jobs, int chunk,
                            gwas_enc_output **out) {
    return guard_ctx(ctx, [&] {
        need(in && out && n_jobs >= 1 && chunk >= 1, "bad arguments");
        std::vector<const EncInput *> jobs;
        for (int i = 0; i < n_jobs; ++i) {
            need(in[i] && in[i]->ctx == ctx, "input belongs to another context");
            jobs.push_back(in[i]->in.get());
            out[i] = nullptr;
        }
        std::vector<EncOutput> outs;
        run_multi(*ctx, jobs, outs, chunk);
        for (int i = 0; i < n_jobs; ++i) {
            auto o = std::make_unique<gwas_enc_output>();
            o->ctx = ctx;
            o->lay = jobs[i]->lay;
            o->out = std::move(outs[i]);
            out[i] = o.release();
        }
    });
}

int gwas_semiparallel(ckks_ctx *ctx, const gwas_enc_input *in, gwas_enc_output **out) {
    const int chunk = in && in->in ? std::max(1, in->in->S->count) : 1;
    if (ctx && in && in->in && ctx->use_tuned) {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        auto it = ctx->tuned.find(schedule_key(*in->in));
        if (it != ctx->tuned.end()) {
            const int saved = ctx->n_streams, saved_stack = ctx->stack_cts;
            ctx->n_streams = it->second.streams;
            ctx->stack_cts = it->second.stack;
            const int rc = gwas_semiparallel_chunked(ctx, in, it->second.chunk, out);
            ctx->n_streams = saved;
            ctx->stack_cts = saved_stack;
            return rc;
        }
    }
    return gwas_semiparallel_chunked(ctx, in, chunk > 64 ? 64 : chunk, out);
}

int gwas_tune(ckks_ctx *ctx, const gwas_enc_input *in, int reps, int *chunk, int *streams, double *ms,
              double *ms_default, int *candidates, int *stack) {
    return guard_ctx(ctx, [&] {
        need(in && in->ctx == ctx, "bad arguments");
        const TuneResult r = tune_circuit(*ctx, *in->in, reps);
        if (chunk) *chunk = r.best.chunk;
        if (streams) *streams = r.best.streams;
        if (ms) *ms = r.best.ms;
        if (ms_default) *ms_default = r.ms_default;
        if (candidates) *candidates = r.candidates;
        if (stack) *stack = r.best.stack;
    });
}

int gwas_keep_projected(ckks_ctx *ctx, int keep) {
    return guard_ctx(ctx, [&] { ctx->keep_s_proj = keep != 0; });
}

int ckks_ctx_use_tuned(ckks_ctx *ctx, int enable) {
    return guard_ctx(ctx, [&] { ctx->use_tuned = enable != 0; });
}

int gwas_output_batches(const gwas_enc_output *out, int *n_batches) {
    return guard([&] {
        need(out && n_batches, "null argument");
        *n_batches = out->lay.n_batches;
    });
}

int gwas_output_ct(const gwas_enc_output *out, int which, int index, const ckks_ct **ct) {
    return guard([&] {
        need(out && ct, "null argument");
        const EncOutput &o = out->out;
        const std::vector<Ct> *vec = nullptr;
        switch (which) {
        case 0: vec = &o.num; break;
        case 1: vec = &o.den_even; break;
        case 2: vec = &o.den_odd; break;
        case 3: vec = &o.S_proj; break;
        case 4:
            need(index >= 0 && index < (int)o.beta.size(), "beta index out of range");
            *ct = o.beta[index].get();
            return;
        case 5:
        case 6:
            *ct = which == 5 ? o.w.get() : o.w_inv.get();
            if (!*ct) throw Error(CKKS_E_INVALID_ARG, "w and w^-1 are public constants for kappa = 1 (no ciphertext)");
            return;
        case 7: *ct = o.z_proj.get(); return;
        case 8: *ct = o.u.get(); return;
        case 9: vec = &o.div_b; break;
        case 10: vec = &o.div_inv; break;
        case 11:
            *ct = o.m_cols.get();
            if (!*ct) throw Error(CKKS_E_INVALID_ARG, "no M columns (the input has no M-materialised layout)");
            return;
        default: need(false, "unknown output");
        }
        need(index >= 0 && index < (int)vec->size(), "chunk index out of range");
        *ct = (*vec)[index].get();
    });
}

void gwas_output_free(gwas_enc_output *out) { free_locked(out ? out->ctx : nullptr, out); }

int gwas_graph_create(ckks_ctx *ctx, const gwas_enc_input *in, int chunk, gwas_graph **out) {
    return guard_ctx(ctx, [&] {
        need(in && out && in->ctx == ctx, "bad arguments");
        *out = nullptr;
        const int nb = in->in->S->count;
        if (chunk <= 0) chunk = std::min(64, std::max(1, nb));
        *out = capture_circuit(*ctx, *in->in, chunk).release();
    });
}

int gwas_graph_set_input(gwas_graph *g, const gwas_enc_input *in) {
    if (!g) return CKKS_E_INVALID_ARG;
    return guard_ctx(g->ctx, [&] {
        need(in && in->ctx == g->ctx, "bad arguments");
        graph_set_input(*g, *in->in);
    });
}

int gwas_graph_launch(gwas_graph *g) {
    if (!g) return CKKS_E_INVALID_ARG;
    return guard_ctx(g->ctx, [&] { graph_launch(*g); });
}

int gwas_graph_output(const gwas_graph *g, const gwas_enc_output **out) {
    return guard([&] {
        need(g && out, "null argument");
        *out = g->out.get();
    });
}

void gwas_graph_destroy(gwas_graph *g) {
    if (!g) return;
    std::lock_guard<std::recursive_mutex> lk(g->ctx->mu);
    delete g;
}

int gwas_div_levels(void) { return div_levels(); }

int gwas_input_attach_m(ckks_ctx *ctx, gwas_enc_input *in, const ckks_ct *const *xrep, int n_xrep,
                        const ckks_ct *const *srep, int n_srep) {
    return guard_ctx(ctx, [&] {
        need(in && xrep && srep && in->ctx == ctx, "bad arguments");
        need(n_xrep == in->in->lay.n * in->in->lay.k && n_srep == in->in->lay.n * in->in->lay.n_batches,
             "need n k REP entries of X^T and n REP rows per SNP batch");
        std::vector<const ckks_ct *> xs, ss;
        for (int i = 0; i < n_xrep; ++i) {
            check_ct(ctx, xrep[i]);
            xs.push_back(xrep[i]);
        }
        for (int i = 0; i < n_srep; ++i) {
            check_ct(ctx, srep[i]);
            ss.push_back(srep[i]);
        }
        attach_m(*ctx, *in->in, stack(*ctx, xs), stack(*ctx, ss));
    });
}

int gwas_pack_encrypt_m(ckks_ctx *ctx, gwas_enc_input *in, const double *X, const uint8_t *S, uint64_t enc_seed) {
    return guard_ctx(ctx, [&] {
        need(in && X && S && in->ctx == ctx, "bad arguments");
        pack_encrypt_m(*ctx, *in->in, X, S, enc_seed);
    });
}

int gwas_pack_normalisers(ckks_ctx *ctx, const uint8_t *S, int n, int m, int kappa, uint64_t enc_seed,
                          ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        need(ctx && S && out, "null argument");
        need(kappa >= 1 && n >= 2 && m >= 1, "bad sizes");
        *out = release(pack_normalisers(*ctx, S, n, m, kappa, enc_seed));
    });
}

int gwas_divide(ckks_ctx *ctx, gwas_enc_output *out, const ckks_ct *v) {
    return guard_ctx(ctx, [&] {
        need(out && v, "null argument");
        need(out->ctx == ctx, "output belongs to another context");
        check_ct(ctx, v);
        run_divide(*ctx, out->out, *v);
    });
}

int gwas_finalize_divided(ckks_ctx *ctx, const gwas_enc_output *out, int m, double *b, double *err, double *se) {
    return guard_ctx(ctx, [&] {
        need(ctx && out, "null argument");
        const Layout &lay = out->lay;
        need(m == lay.m, "m does not match the layout");
        need(!out->out.div_b.empty(), "no divided outputs (gwas_divide not run)");
        const int N = ctx->p.n, slots = N / 2;
        std::vector<double> vb((size_t)lay.n_batches * lay.tau, 0.0), ve(vb.size(), 0.0);
        std::vector<double> re(slots), im(slots), coeffs(N);
        auto dec = [&](const ckks_ct &ct, int idx) {
            auto v = decrypt_poly(*ctx, ct, idx);
            for (int t = 0; t < N; ++t) coeffs[t] = (double)(v[t] / (long double)ct.scale);
            decode_poly(N, coeffs.data(), re.data(), im.data());
        };
        int batch = 0;
        for (size_t ch = 0; ch < out->out.div_b.size(); ++ch) {
            const ckks_ct &cb = *out->out.div_b[ch], &ci = *out->out.div_inv[ch];
            const int cnt = cb.count / 2;
            for (int i = 0; i < cnt; ++i, ++batch) {
                const size_t base = (size_t)batch * lay.tau;
                for (int par = 0; par < 2; ++par) {
                    dec(cb, par * cnt + i);
                    for (int q = 0; q < lay.blocks; ++q)
                        vb[base + 2 * q + par] = par == 0 ? re[(size_t)q * lay.R] : im[(size_t)q * lay.R];
                    dec(ci, par * cnt + i);
                    for (int q = 0; q < lay.blocks; ++q) ve[base + 2 * q + par] = re[(size_t)q * lay.R];
                }
            }
        }
        for (int j = 0; j < m; ++j) {
            if (b) b[j] = vb[j];
            if (err) err[j] = ve[j];
            if (se) se[j] = std::sqrt(std::max(ve[j], 0.0));
        }
    });
}

int ckks_ct_stack(ckks_ctx *ctx, const ckks_ct *const *parts, int n, ckks_ct **out) {
    return guard_ctx(ctx, [&] {
        need(parts && out && n >= 1, "bad arguments");
        std::vector<const ckks_ct *> v;
        for (int i = 0; i < n; ++i) {
            check_ct(ctx, parts[i]);
            v.push_back(parts[i]);
        }
        *out = release(stack(*ctx, v));
    });
}

int gwas_finalize(ckks_ctx *ctx, const gwas_enc_output *out, int m, double *b, double *err, double *se, double *num,
                  double *den) {
    return guard_ctx(ctx, [&] {
        need(ctx && out, "null argument");
        const Layout &lay = out->lay;
        need(m == lay.m, "m does not match the layout");
        const int N = ctx->p.n, slots = N / 2;
        std::vector<double> vnum((size_t)lay.n_batches * lay.tau, 0.0), vden(vnum.size(), 0.0);
        std::vector<double> re(slots), im(slots), coeffs(N);
        int batch = 0;
        for (size_t ch = 0; ch < out->out.num.size(); ++ch) {
            const ckks_ct &cn = *out->out.num[ch], &ce = *out->out.den_even[ch], &co = *out->out.den_odd[ch];
            for (int i = 0; i < cn.count; ++i, ++batch) {
                auto dec = [&](const ckks_ct &ct, int idx) {
                    auto v = decrypt_poly(*ctx, ct, idx);
                    for (int t = 0; t < N; ++t) coeffs[t] = (double)(v[t] / (long double)ct.scale);
                    decode_poly(N, coeffs.data(), re.data(), im.data());
                };
                const size_t base = (size_t)batch * lay.tau;
                dec(cn, i);
                for (int cb = 0; cb < lay.blocks; ++cb) {
                    vnum[base + 2 * cb] = re[(size_t)cb * lay.R];
                    vnum[base + 2 * cb + 1] = im[(size_t)cb * lay.R];
                }
                dec(ce, i);
                for (int cb = 0; cb < lay.blocks; ++cb) vden[base + 2 * cb] = re[(size_t)cb * lay.R];
                dec(co, i);
                for (int cb = 0; cb < lay.blocks; ++cb) vden[base + 2 * cb + 1] = re[(size_t)cb * lay.R];
            }
        }
        for (int j = 0; j < m; ++j) {
            if (num) num[j] = vnum[j];
            if (den) den[j] = vden[j];
            if (b) b[j] = vnum[j] / vden[j];
            if (err) err[j] = 1.0 / vden[j];
            if (se) se[j] = std::sqrt(1.0 / vden[j]);
        }
    });
}

}  // extern "C"
