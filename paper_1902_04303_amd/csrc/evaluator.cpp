// Host driver of the RNS-CKKS evaluator: context and tables, device memory pool, keys, encryption and
// the scheme operations of the paper's Methods ("Homomorphic Encryption") in RNS form.
#include <cmath>
#include <cstring>
#include <fstream>
#include <random>

#include "evaluator.h"

namespace gck {

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) throw Error(CKKS_E_NOMEM, std::string("device out of memory in ") + what);
        throw Error(CKKS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

// ---------------------------------------------------------------- pool

Pool::Pool(const ckks_allocator *alloc, size_t b) : budget(b) {
    if (alloc && alloc->alloc && alloc->free) {
        alloc_ = *alloc;
        have_alloc_ = true;
    }
}

Pool::~Pool() {
    if (arena_base_) return;
    if (stream) hipStreamSynchronize(stream);
    else hipDeviceSynchronize();
    for (auto &kv : free_) raw_free(kv.second, kv.first);
    free_.clear();
}

void *Pool::raw_alloc(size_t bytes) {
    void *p = nullptr;
    if (have_alloc_) {
        p = alloc_.alloc(bytes, alloc_.user);
        if (!p) throw Error(CKKS_E_NOMEM, "allocator callback returned NULL");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(CKKS_E_NOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
        }
    }
    ++n_alloc;
    return p;
}

void Pool::raw_free(void *p, size_t bytes) {
    if (have_alloc_) alloc_.free(p, bytes, alloc_.user);
    else hipFree(p);
}

static size_t round_bytes(size_t b) { return (b + 255) & ~size_t(255); }

std::unique_ptr<Pool> Pool::arena(void *base, size_t bytes) {
    auto p = std::make_unique<Pool>(nullptr, 0);
    p->arena_base_ = static_cast<char *>(base);
    p->arena_bytes_ = bytes;
    return p;
}

void *Pool::get(size_t bytes) {
    bytes = round_bytes(bytes ? bytes : 8);
    if (arena_base_) {
        if (bytes > arena_bytes_ - arena_top_)
            throw Error(CKKS_E_NOMEM, "scratch region exhausted (" + std::to_string(arena_top_ + bytes) + " > " +
                                          std::to_string(arena_bytes_) + " bytes)");
        void *p = arena_base_ + arena_top_;
        arena_top_ += bytes;
        in_use += bytes;
        peak = std::max(peak, in_use);
        return p;
    }
    auto it = free_.find(bytes);
    if (it != free_.end()) {
        void *p = it->second;
        free_.erase(it);
        cached -= bytes;
        in_use += bytes;
        peak = std::max(peak, in_use);
        if (capturing_) captured_[p] = bytes;
        return p;
    }
    if (budget && in_use + cached + bytes > budget) {
        trim();
        if (in_use + bytes > budget)
            throw Error(CKKS_E_NOMEM, "pool budget exceeded (" + std::to_string(in_use + bytes) + " > " +
                                          std::to_string(budget) + " bytes)");
    }
    void *p;
    try {
        p = raw_alloc(bytes);
    } catch (const Error &) {
        trim();
        p = raw_alloc(bytes);
    }
    in_use += bytes;
    peak = std::max(peak, in_use);
    if (capturing_) captured_[p] = bytes;
    return p;
}

void Pool::capture_begin() {
    capturing_ = true;
    captured_.clear();
}

std::vector<std::pair<void *, size_t>> Pool::capture_end() {
    capturing_ = false;
    std::vector<std::pair<void *, size_t>> out;
    for (auto it = free_.begin(); it != free_.end();) {
        if (captured_.count(it->second)) {
            out.push_back({it->second, it->first});
            cached -= it->first;
            in_use += it->first;
            it = free_.erase(it);
        } else {
            ++it;
        }
    }
    captured_.clear();
    return out;
}

void Pool::give_back(const std::vector<std::pair<void *, size_t>> &blocks) {
    for (auto &b : blocks) {
        free_.emplace(b.second, b.first);
        in_use -= b.second;
        cached += b.second;
    }
}

void Pool::put(void *p, size_t bytes) {
    bytes = round_bytes(bytes ? bytes : 8);
    if (arena_base_) {
        if (static_cast<char *>(p) + bytes == arena_base_ + arena_top_) {
            arena_top_ -= bytes;
            in_use -= bytes;
        }
        return;
    }
    free_.emplace(bytes, p);
    in_use -= bytes;
    cached += bytes;
}

std::unique_ptr<Pool> Pool::sibling() const {
    auto p = std::make_unique<Pool>(nullptr, 0);
    p->alloc_ = alloc_;
    p->have_alloc_ = have_alloc_;
    return p;
}

void Pool::trim() {
    if (arena_base_ || free_.empty()) return;
    if (stream) hipStreamSynchronize(stream);
    else hipDeviceSynchronize();
    for (auto &kv : free_) raw_free(kv.second, kv.first);
    free_.clear();
    cached = 0;
}

void sync(ckks_ctx &c) { GCK_HIP(hipStreamSynchronize(c.stream)); }

void ensure_aux(ckks_ctx &c) {
    // non-blocking (default priority): no implicit ordering with a legacy default main stream; the two
    // streams are ordered by events only
    if (!c.aux_stream) GCK_HIP(hipStreamCreateWithFlags(&c.aux_stream, hipStreamNonBlocking));
    if (!c.aux_pool) {
        c.aux_pool = c.pool->sibling();
        c.aux_pool->stream = c.aux_stream;
    }
}

OnStream::OnStream(ckks_ctx &ctx) : c(ctx) {
    ensure_aux(c);
    std::swap(c.stream, c.aux_stream);
    c.pool.swap(c.aux_pool);
}

OnStream::~OnStream() {
    std::swap(c.stream, c.aux_stream);
    c.pool.swap(c.aux_pool);
}

void stream_wait(hipStream_t to, hipStream_t from) {
    hipEvent_t ev;
    GCK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    GCK_HIP(hipEventRecord(ev, from));
    GCK_HIP(hipStreamWaitEvent(to, ev, 0));
    (void)hipEventDestroy(ev);
}

// ---------------------------------------------------------------- ciphertext helpers

Ct new_ct(ckks_ctx &c, int count, int depth, double scale) {
    if (depth < 0 || depth > c.p.levels) throw Error(CKKS_E_LEVEL, "depth " + std::to_string(depth) + " out of range");
    Ct r(new ckks_ct());
    r->ctx = &c;
    r->count = count;
    r->depth = depth;
    r->limbs = c.p.limbs_at(depth);
    r->scale = scale;
    r->data = DBuf(c.pool.get(), (size_t)count * 2 * r->limbs * c.p.n);
    return r;
}

Ct clone(ckks_ctx &c, const ckks_ct &a) {
    Ct r = new_ct(c, a.count, a.depth, a.scale);
    GCK_HIP(hipMemcpyAsync(r->data.ptr, a.data.ptr, a.data.words * 8, hipMemcpyDeviceToDevice, c.stream));
    return r;
}

Ct view(const ckks_ct &a, int first, int n) {
    if (first < 0 || n < 1 || first + n > a.count) throw Error(CKKS_E_INVALID_ARG, "view out of range");
    const size_t per = (size_t)2 * a.limbs * a.ctx->p.n;
    Ct r(new ckks_ct());
    r->ctx = a.ctx;
    r->count = n;
    r->depth = a.depth;
    r->limbs = a.limbs;
    r->scale = a.scale;
    r->data.pool = nullptr;   // not owned: nothing is returned to the pool
    r->data.ptr = a.data.ptr + (size_t)first * per;
    r->data.words = (size_t)n * per;
    return r;
}

Ct stack(ckks_ctx &c, const std::vector<const ckks_ct *> &parts) {
    if (parts.empty()) throw Error(CKKS_E_INVALID_ARG, "nothing to stack");
    int count = 0;
    for (auto *p : parts) {
        if (p->depth != parts[0]->depth || p->scale != parts[0]->scale)
            throw Error(CKKS_E_PARAM_MISMATCH, "stacked ciphertexts differ in depth or scale");
        count += p->count;
    }
    Ct r = new_ct(c, count, parts[0]->depth, parts[0]->scale);
    size_t off = 0;
    for (auto *p : parts) {
        GCK_HIP(hipMemcpyAsync(r->data.ptr + off, p->data.ptr, p->data.words * 8, hipMemcpyDeviceToDevice, c.stream));
        off += p->data.words;
    }
    return r;
}

void ntt_fwd(ckks_ctx &c, u64 *buf, int n_limbs, ModMap m) {
    k_ntt_forward(c.tab, buf, n_limbs, m, c.stream);
    c.n_limb_ntt += n_limbs;
    c.n_launch += 2;
}
void ntt_inv(ckks_ctx &c, u64 *buf, int n_limbs, ModMap m) {
    k_ntt_inverse(c.tab, buf, n_limbs, m, c.stream);
    c.n_limb_ntt += n_limbs;
    c.n_launch += 2;
}

static ChainConst chain_const_of(const ckks_ctx &c, i64 k) {
    ChainConst cc{};
    for (int i = 0; i < c.p.n_mods(); ++i) {
        u64 q = c.p.mod(i);
        u64 v = k >= 0 ? (u64)k % q : q - 1 - (u64)(-(k + 1)) % q;
        cc.v[i] = v;
        cc.sh[i] = (u64)(((u128)v << 64) / q);
    }
    return cc;
}

static void check_same(const ckks_ct &a, const ckks_ct &b) {
    if (a.depth != b.depth || a.scale != b.scale)
        throw Error(CKKS_E_PARAM_MISMATCH, "operands differ in depth (" + std::to_string(a.depth) + ", " +
                                               std::to_string(b.depth) + ") or scale");
    if (std::max(a.count, b.count) % std::min(a.count, b.count) != 0)
        throw Error(CKKS_E_PARAM_MISMATCH, "batch counts differ");
}

// ---------------------------------------------------------------- scheme operations

Ct add(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b) {
    check_same(a, b);
    int count = std::max(a.count, b.count), l = a.limbs;
    Ct r = new_ct(c, count, a.depth, a.scale);
    k_add(c.tab, r->data.ptr, a.data.ptr, b.data.ptr, count * 2 * l, map_q(l), a.count * 2 * l, b.count * 2 * l, c.stream);
    ++c.n_launch;
    return r;
}

Ct sub(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b) {
    check_same(a, b);
    int count = std::max(a.count, b.count), l = a.limbs;
    Ct r = new_ct(c, count, a.depth, a.scale);
    k_sub(c.tab, r->data.ptr, a.data.ptr, b.data.ptr, count * 2 * l, map_q(l), a.count * 2 * l, b.count * 2 * l, c.stream);
    ++c.n_launch;
    return r;
}

Ct mul_int(ckks_ctx &c, const ckks_ct &a, i64 k) {
    Ct r = new_ct(c, a.count, a.depth, a.scale);
    k_mul_const(c.tab, r->data.ptr, a.data.ptr, a.count * 2 * a.limbs, map_q(a.limbs), chain_const_of(c, k), c.stream);
    ++c.n_launch;
    return r;
}

Ct neg(ckks_ctx &c, const ckks_ct &a) { return mul_int(c, a, -1); }

Ct add_const(ckks_ctx &c, const ckks_ct &a, double v) {
    Ct r = new_ct(c, a.count, a.depth, a.scale);
    i64 k = round_half_away(v * a.scale);
    k_add_const_c0(c.tab, r->data.ptr, a.data.ptr, a.count, a.limbs, chain_const_of(c, k), c.stream);
    ++c.n_launch;
    return r;
}

// Rescale: round(c / q_last) on the centred integer, per limb (c_i - [c_last]_centred) * q_last^-1 mod q_i.
// The last limb of every polynomial is gathered by the inverse NTT, centred-lifted to the other limbs
// while loading the forward NTT, and the forward NTT's final store (the ModDown epilogue with q_last^-1
// in place of P^-1) subtracts and scales straight into the result.
Ct rescale(ckks_ctx &c, const ckks_ct &a) {
    const int l = a.limbs, rows = a.count * 2;
    if (l < 2) throw Error(CKKS_E_LEVEL, "no limb left to rescale");
    const size_t N = (size_t)c.p.n;
    DBuf last(c.pool.get(), (size_t)rows * N);
    k_ntt_inverse_g(c.tab, last.ptr, Gather{a.data.ptr, 1, l, l - 1, 0, kPlain, 0}, rows, ModMap{1, 0, l - 1}, c.stream);
    Ct r = new_ct(c, a.count, a.depth + 1, a.scale);
    const ckks_ctx::QInv &qi = c.q_inv.at(l - 1);
    const ModDownEpi epi{Gather{a.data.ptr, l - 1, l, 0, 1, kPlain, 0}, Gather{}, 0, l - 1, qi.v, qi.sh, qi.d, nullptr,
                         0, 0, {}};
    k_ntt_forward_g(c.tab, r->data.ptr, Gather{last.ptr, l - 1, 1, 0, 0, kCentred, l - 1}, rows * (l - 1),
                    map_q(l - 1), c.stream, &epi);
    c.n_limb_ntt += (uint64_t)rows * l;
    c.n_launch += 4;
    return r;
}

// rescale(k a) of the first lt limbs of a (lt <= a.limbs): the last of them is multiplied by k while the
// forward NTT gathers it (before centring), the others in the epilogue; the same residues as mod_drop,
// mul_int and rescale in turn, without their intermediate batches
static Ct rescale_mul(ckks_ctx &c, const ckks_ct &a, int lt, i64 k) {
    const int la = a.limbs, rows = a.count * 2;
    if (lt < 2 || lt > la) throw Error(CKKS_E_LEVEL, "no limb left to rescale");
    const size_t N = (size_t)c.p.n;
    DBuf last(c.pool.get(), (size_t)rows * N);
    k_ntt_inverse_g(c.tab, last.ptr, Gather{a.data.ptr, 1, la, lt - 1, 0, kPlain, 0}, rows, ModMap{1, 0, lt - 1},
                    c.stream);
    Ct r = new_ct(c, a.count, c.p.levels + 2 - lt, a.scale);   // lt - 1 limbs
    const ckks_ctx::QInv &qi = c.q_inv.at(lt - 1);
    const ChainConst cc = chain_const_of(c, k);
    ModDownEpi epi{Gather{a.data.ptr, lt - 1, la, 0, 1, kPlain, 0}, Gather{}, 0, lt - 1, qi.v, qi.sh, qi.d, nullptr,
                   0, 0, {}};
    epi.acc_mul = 1;
    for (int i = 0; i < lt - 1; ++i) epi.km[i] = cc.v[i];
    Gather gl{last.ptr, lt - 1, 1, 0, 0, kCentred, lt - 1};
    gl.cmul = cc.v[lt - 1];
    gl.cmul_sh = cc.sh[lt - 1];
    k_ntt_forward_g(c.tab, r->data.ptr, gl, rows * (lt - 1), map_q(lt - 1), c.stream, &epi);
    c.n_limb_ntt += (uint64_t)rows * lt;
    c.n_launch += 4;
    return r;
}

Ct mod_drop(ckks_ctx &c, const ckks_ct &a, int depth) {
    if (depth == a.depth) return clone(c, a);
    if (depth < a.depth) throw Error(CKKS_E_LEVEL, "mod-drop to a shallower depth");
    Ct r = new_ct(c, a.count, depth, a.scale);
    const size_t N = (size_t)c.p.n;
    k_copy_rows(r->data.ptr, (size_t)r->limbs * N, a.data.ptr, (size_t)a.limbs * N, a.count * 2, (size_t)r->limbs * N,
                c.stream);
    ++c.n_launch;
    return r;
}

Ct mul_const(ckks_ctx &c, const ckks_ct &a, double v) {
    const u64 q = c.p.dropped_at(a.depth);
    Ct r = rescale_mul(c, a, a.limbs, round_half_away(v * a.scale));
    r->scale = (a.scale * a.scale) / (double)q;
    return r;
}

// 1 at the slots s = j mod P for j0 <= j < j1 at `scale`, in NTT form over l limbs: the sum over j of the
// block-start mask of period P moved by the automorphism X -> X^(5^-j) of a right rotation by j (a signed
// permutation of its integer coefficients, so the encoding stays exact).  Made once per (P, j0, j1, l,
// scale) and kept in the context; a new entry is completed (stream synchronised) before it is used, so any
// stream may read it later
static const u64 *class_mask_plain(ckks_ctx &c, int P, int j0, int j1, int l, double scale) {
    uint64_t bits;
    std::memcpy(&bits, &scale, sizeof bits);
    const auto key = std::make_tuple(P, j0, j1, l, bits);
    auto it = c.mask_cache.find(key);
    if (it != c.mask_cache.end()) return it->second.ptr;
    const int n = c.p.n;
    if (j0 < 0 || j1 <= j0 || j1 > P) throw Error(CKKS_E_INVALID_ARG, "slot classes out of range");
    std::vector<i64> m0(n), h(n, 0);
    mask_poly(n, P, scale, m0.data());
    const u64 two_n = 2ULL * (u64)n;
    for (int j = j0; j < j1; ++j) {
        const u64 g = galois_rotate_n(n, -j);
        for (int i = 0; i < n; ++i) {
            if (!m0[i]) continue;
            const u64 e = ((u64)i * g) % two_n;
            if (e < (u64)n) h[e] += m0[i];
            else h[e - n] -= m0[i];
        }
    }
    DBuf small(c.pool.get(), (size_t)n);
    GCK_HIP(hipMemcpyAsync(small.ptr, h.data(), (size_t)n * 8, hipMemcpyHostToDevice, c.stream));
    DBuf pt(c.pool.get(), (size_t)l * n);
    k_signed_to_limbs(c.tab, pt.ptr, reinterpret_cast<const i64 *>(small.ptr), l, map_q(l), c.stream);
    ntt_fwd(c, pt.ptr, l, map_q(l));
    sync(c);   // the host vector goes out of scope; the entry is complete for every stream
    const u64 *p = pt.ptr;
    c.mask_cache.emplace(key, std::move(pt));
    return p;
}

static const u64 *mask_plain(ckks_ctx &c, int R, int l, double scale) { return class_mask_plain(c, R, 0, 1, l, scale); }

Ct mask_sum(ckks_ctx &c, const std::vector<MaskTerm> &terms) {
    if (terms.empty()) throw Error(CKKS_E_INVALID_ARG, "empty mask sum");
    const ckks_ct &a0 = *terms[0].a;
    const u64 q = c.p.dropped_at(a0.depth);
    const int l = a0.limbs, rows = a0.count * 2 * l;
    Ct acc = new_ct(c, a0.count, a0.depth, a0.scale);
    Ct tmp;
    for (size_t i = 0; i < terms.size(); ++i) {
        const MaskTerm &m = terms[i];
        check_same(*m.a, a0);
        if (m.a->count != a0.count) throw Error(CKKS_E_PARAM_MISMATCH, "mask sum operands of unequal counts");
        const u64 *pt = class_mask_plain(c, m.P, m.j0, m.j1, l, a0.scale);
        if (i == 0) {
            k_mul(c.tab, acc->data.ptr, m.a->data.ptr, pt, rows, map_q(l), rows, l, c.stream);
        } else {
            if (!tmp) tmp = new_ct(c, a0.count, a0.depth, a0.scale);
            k_mul(c.tab, tmp->data.ptr, m.a->data.ptr, pt, rows, map_q(l), rows, l, c.stream);
            k_add(c.tab, acc->data.ptr, acc->data.ptr, tmp->data.ptr, rows, map_q(l), rows, rows, c.stream);
            ++c.n_launch;
        }
        ++c.n_launch;
    }
    Ct r = rescale(c, *acc);
    r->scale = (a0.scale * a0.scale) / (double)q;
    return r;
}

Ct mul_mask(ckks_ctx &c, const ckks_ct &a, int R) {
    const u64 q = c.p.dropped_at(a.depth);
    const int l = a.limbs;
    const u64 *pt = mask_plain(c, R, l, a.scale);
    Ct t = new_ct(c, a.count, a.depth, a.scale);
    k_mul(c.tab, t->data.ptr, a.data.ptr, pt, a.count * 2 * l, map_q(l), a.count * 2 * l, l, c.stream);
    c.n_launch += 1;
    Ct r = rescale(c, *t);
    r->scale = (a.scale * a.scale) / (double)q;
    return r;
}

// a + b X^(N/2) over l limbs in NTT form, kept in the context like the masks.  Slot j of a plaintext is its
// value at zeta^(5^j) with zeta = exp(i pi / N); X^(N/2) takes the value zeta^(5^j N / 2) = i there because
// 5^j = 1 mod 4, so a product with this polynomial multiplies every slot by a + b i with no rounding.
static const u64 *monomial_plain(ckks_ctx &c, int l, i64 a, i64 b) {
    const auto key = std::make_tuple(l, a, b);
    auto it = c.mono_cache.find(key);
    if (it != c.mono_cache.end()) return it->second.ptr;
    const int n = c.p.n;
    std::vector<i64> h(n, 0);
    h[0] = a;
    h[n / 2] = b;
    DBuf small(c.pool.get(), (size_t)n);
    GCK_HIP(hipMemcpyAsync(small.ptr, h.data(), (size_t)n * 8, hipMemcpyHostToDevice, c.stream));
    DBuf pt(c.pool.get(), (size_t)l * n);
    k_signed_to_limbs(c.tab, pt.ptr, reinterpret_cast<const i64 *>(small.ptr), l, map_q(l), c.stream);
    ntt_fwd(c, pt.ptr, l, map_q(l));
    sync(c);   // the host vector goes out of scope; the entry is complete for every stream
    const u64 *p = pt.ptr;
    c.mono_cache.emplace(key, std::move(pt));
    return p;
}

Ct mul_gauss(ckks_ctx &c, const ckks_ct &a, i64 re, i64 im) {
    const int l = a.limbs;
    const u64 *pt = monomial_plain(c, l, re, im);
    Ct r = new_ct(c, a.count, a.depth, a.scale);
    k_mul(c.tab, r->data.ptr, a.data.ptr, pt, a.count * 2 * l, map_q(l), a.count * 2 * l, l, c.stream);
    ++c.n_launch;
    return r;
}

Ct mul_i(ckks_ctx &c, const ckks_ct &a, bool neg) { return mul_gauss(c, a, 0, neg ? -1 : 1); }

Ct align(ckks_ctx &c, const ckks_ct &a, int depth, double scale, double factor) {
    if (depth == a.depth && scale == a.scale && factor == 1.0) return clone(c, a);
    if (depth <= a.depth) throw Error(CKKS_E_LEVEL, "align needs a deeper target depth");
    const u64 q = c.p.dropped_at(depth - 1);
    i64 k = round_half_away(((scale * factor) * (double)q) / a.scale);
    // mod_drop to depth - 1, times k, rescale: one chain over the first limbs of a
    Ct r = rescale_mul(c, a, c.p.limbs_at(depth - 1), k);
    r->scale = scale;
    return r;
}

Ct set_scale(ckks_ctx &, Ct a, double factor) {
    a->scale *= factor;
    return a;
}

bool has_key(const ckks_ctx &c, u64 id) { return c.ksk.count(id) != 0; }

static const u64 *key_of(const ckks_ctx &c, u64 id) {
    auto it = c.ksk.find(id);
    if (it == c.ksk.end()) {
        if (id == 0) throw Error(CKKS_E_KEY_MISSING, "missing relinearisation key");
        throw Error(CKKS_E_KEY_MISSING, "missing Galois key for element " + std::to_string(id));
    }
    return it->second.ptr;
}

// Key switch of the polynomial gathered by `d` (count ciphertexts, l limbs, NTT form) with the keys of
// `keys` (hybrid decomposition, digit groups of alpha primes {q_0 .. q_{alpha-2}}, {q_{alpha-1} ..}, ...):
//   ModUp    y_i = d_i (Q_G/q_i)^-1 (folded into the inverse NTT), then each group's digit
//            D = sum_{i in G} y_i (Q_G/q_i) converted to every other target while loading the forward
//            NTT (its residues at its own primes are the input limbs themselves);
//   inner    x = sum_i sum_b sigma_i(D_b) ksk_{i,b} over the targets q_0..q_{l-1}, p_1..p_alpha, the digits
//            read through each key's automorphism;
//   ModDown  (x - C) / P with C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k) (the scales folded into the
//            inverse NTT of the special limbs, the conversion into the forward NTT's load, the
//            subtraction, the multiply by P^-1 and the added term into its final store);
// plus the gathered `add` term (on every row, or on the first polynomial of each ciphertext when
// add_even).  Output [count][2][l][N] in NTT form.
// ModUp of a key switch: the digits of the polynomial gathered by `d` at every target ([count][K][N])
static DBuf mod_up(ckks_ctx &c, const Gather &d, int count, int l) {
    const size_t N = (size_t)c.p.n;
    const ckks_ctx::KsLevel &kl = c.ks_levels.at(l);
    DBuf dc(c.pool.get(), (size_t)count * l * N);
    k_ntt_inverse_g(c.tab, dc.ptr, d, count * l, map_q(l), c.stream, kl.up_scale, l);
    DBuf dig(c.pool.get(), (size_t)count * kl.K * N);
    k_ntt_forward_g(c.tab, dig.ptr, Gather{dc.ptr, 1, 1, 0, 0, kConv, 0, kl.up, kl.K, l}, count * kl.K, map_q(l),
                    c.stream);
    c.n_limb_ntt += (uint64_t)count * (l + kl.K);
    c.n_launch += 2;
    return dig;
}

// inner product and ModDown of a key switch whose digits `dig` come from mod_up of `d` (see keyswitch);
// `own`, when given, holds the digits and is released after the inner product
static DBuf ks_inner_down(ckks_ctx &c, const u64 *dig, const Gather &d, int count, int l, const KsKeys &keys,
                          const Gather &add, bool add_even, const u64 *aut, int aut_self, bool aut_gather,
                          DBuf *own = nullptr);

static DBuf keyswitch(ckks_ctx &c, const Gather &d, int count, int l, const KsKeys &keys, const Gather &add,
                      bool add_even, const u64 *aut = nullptr, int aut_self = 0, bool aut_gather = true) {
    const size_t N = (size_t)c.p.n;
    const int a = c.p.alpha, nt = l + a;
    // algorithmic bytes of the key switch: the input polynomial (l limbs per ciphertext), each key's digit
    // groups below l at every target (read once per call, shared by the ciphertexts) and the two output
    // polynomials read and written once (2 x 2 l limbs per ciphertext)
    const int groups = 1 + l / a;
    const double ks_bytes = 8.0 * (double)N *
                            ((double)count * l + (double)keys.m * 2.0 * groups * nt + (double)count * 4.0 * l);
    KRegion region_(c.tab.timer, "keyswitch", ks_bytes, c.stream);
    DBuf dig = mod_up(c, d, count, l);
    return ks_inner_down(c, dig.ptr, d, count, l, keys, add, add_even, aut, aut_self, aut_gather, &dig);
}

static DBuf ks_inner_down(ckks_ctx &c, const u64 *dig, const Gather &d, int count, int l, const KsKeys &keys,
                          const Gather &add, bool add_even, const u64 *aut, int aut_self, bool aut_gather,
                          DBuf *own) {
    const size_t N = (size_t)c.p.n;
    const ckks_ctx::KsLevel &kl = c.ks_levels.at(l);
    const int a = c.p.alpha, nt = l + a, P = c.p.p_index();
    DBuf acc(c.pool.get(), (size_t)count * 2 * nt * N);
    k_ks_inner(c.tab, acc.ptr, dig, kl.K, kl.didx, d, keys, c.ng, count, l, c.p.levels, a, c.stream);
    if (own) own->release();
    const int rows = count * 2;
    DBuf ap(c.pool.get(), (size_t)rows * a * N);
    k_ntt_inverse_g(c.tab, ap.ptr, Gather{acc.ptr, a, nt, l, 1, kPlain, 0}, rows * a, ModMap{a, 0, P}, c.stream,
                    c.down_scale, a);
    DBuf out(c.pool.get(), (size_t)rows * l * N);
    ModDownEpi epi{Gather{acc.ptr, l, nt, 0, 1, kPlain, 0}, add, add_even ? 1 : 0, l, c.p_inv_dev, c.p_inv_sh_dev,
                   c.p_inv_d_dev, aut, aut_self, aut && aut_gather ? keys.m : 0, {}};
    for (int i = 0; i < keys.m; ++i) epi.g[i] = keys.g[i];
    k_ntt_forward_g(c.tab, out.ptr, Gather{ap.ptr, 1, 1, 0, 0, kConv, 0, c.down_conv, l, a}, rows * l, map_q(l),
                    c.stream, &epi);
    c.n_limb_ntt += (uint64_t)rows * (a + l);
    c.n_launch += 7;
    ++c.n_keyswitch;
    c.n_keyswitch_ct += (uint64_t)count;
    return out;
}

static KsKeys ks_keys(const ckks_ctx &c, const std::vector<u64> &ids, bool permute) {
    if (ids.empty() || ids.size() > (size_t)kMaxKeys) throw Error(CKKS_E_INVALID_ARG, "1 to 16 keys per key switch");
    KsKeys k{};
    k.m = (int)ids.size();
    for (size_t i = 0; i < ids.size(); ++i) {
        k.key[i] = key_of(c, ids[i]);
        k.g[i] = permute ? ids[i] : 0;
    }
    return k;
}

// Relinearisation of the tensors d ([count][3][l][N], NTT form) fused with the rescale by q_{l-1}: the
// key switch of d2 up to its inner product x (targets q_0..q_{l-1}, p_1..p_alpha) as in keyswitch, then
// one division of x' = x + P (d0, d1) by B = P q_{l-1} in place of ModDown's division by P and the
// rescale's by q_{l-1}:
//   x' at q_{l-1} formed in place (acc += (P mod q_{l-1}) d; x' = x at the special primes);
//   y_b = [x' (B/b)^-1]_b for b = q_{l-1}, p_1..p_alpha (the scales folded into one inverse NTT of those
//   limbs);  C = sum_b y_b (B/b) converted while loading the forward NTT of the l - 1 remaining limbs,
//   whose final store forms (x - C) B^-1 + (d0, d1) q_{l-1}^-1.
// Output [count][2][l-1][N] in NTT form, written into out.
static void keyswitch_rescale(ckks_ctx &c, const u64 *d, int count, int l, u64 *out) {
    if (l < 2) throw Error(CKKS_E_LEVEL, "no limb left to rescale");
    const size_t N = (size_t)c.p.n;
    const ckks_ctx::KsLevel &kl = c.ks_levels.at(l);
    const ckks_ctx::RsLevel &rl = c.rs_levels.at(l - 1);
    const ckks_ctx::QInv &qi = c.q_inv.at(l - 1);
    const int a = c.p.alpha, nt = l + a, P = c.p.p_index(), nb = a + 1, lo = l - 1, rows = count * 2;
    const KsKeys keys = ks_keys(c, {0}, false);
    // algorithmic bytes: d2 (l limbs per ciphertext), the key's digit groups below l at every target
    // (read once per call), d0 and d1 read (2 l) and the two output polynomials written (2 (l - 1))
    const int groups = 1 + l / a;
    const double ks_bytes = 8.0 * (double)N *
                            ((double)count * l + 2.0 * groups * nt + (double)count * 2.0 * l + (double)count * 2.0 * lo);
    KRegion region_(c.tab.timer, "keyswitch", ks_bytes, c.stream);
    const Gather d2{d, l, 3 * l, 2 * l, 1, kPlain, 0};
    DBuf dc(c.pool.get(), (size_t)count * l * N);
    k_ntt_inverse_g(c.tab, dc.ptr, d2, count * l, map_q(l), c.stream, kl.up_scale, l);
    DBuf dig(c.pool.get(), (size_t)count * kl.K * N);
    k_ntt_forward_g(c.tab, dig.ptr, Gather{dc.ptr, 1, 1, 0, 0, kConv, 0, kl.up, kl.K, l}, count * kl.K, map_q(l),
                    c.stream);
    dc.release();
    DBuf acc(c.pool.get(), (size_t)count * 2 * nt * N);
    k_ks_inner(c.tab, acc.ptr, dig.ptr, kl.K, kl.didx, d2, keys, c.ng, count, l, c.p.levels, a, c.stream);
    dig.release();
    const u64 ql = c.p.q[l - 1];
    u64 pm = 1;   // P mod q_{l-1}
    for (int k = 0; k < a; ++k) pm = mulmod_host(pm, c.p.P[k] % ql, ql);
    k_add_scaled_last(c.tab, acc.ptr, d, count, nt, l, pm, (u64)(((unsigned __int128)pm << 64) / ql), ql, c.stream);
    DBuf yb(c.pool.get(), (size_t)rows * nb * N);
    k_ntt_inverse_g(c.tab, yb.ptr, Gather{acc.ptr, nb, nt, l - 1, 1, kPlain, 0}, rows * nb, ModMap{nb, 1, P, l - 1},
                    c.stream, rl.scale, nb);
    ModDownEpi epi{Gather{acc.ptr, lo, nt, 0, 1, kPlain, 0}, Gather{d, 1, 1, 0, 0, kPlain, 0}, 0, lo, rl.binv,
                   rl.binv_sh, rl.binv_d, nullptr, 0, 0, {}};
    epi.addmul = qi.v;
    epi.addmul_sh = qi.sh;
    epi.addmul_d = qi.d;
    epi.add_ct = 3 * l;
    epi.add_poly = l;
    k_ntt_forward_g(c.tab, out, Gather{yb.ptr, 1, 1, 0, 0, kConv, 0, rl.conv, lo, nb}, rows * lo, map_q(lo), c.stream,
                    &epi);
    c.n_limb_ntt += (uint64_t)count * (l + kl.K) + (uint64_t)rows * (nb + lo);
    c.n_launch += 10;
    ++c.n_keyswitch;
    c.n_keyswitch_ct += (uint64_t)count;
}


Ct mul_sum(ckks_ctx &c, const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &pairs) {
    if (pairs.empty()) throw Error(CKKS_E_INVALID_ARG, "empty product sum");
    const ckks_ct &a0 = *pairs[0].first, &b0 = *pairs[0].second;
    const double s = a0.scale * b0.scale;
    int count = 1;
    for (auto &pr : pairs) {
        if (pr.first->depth != a0.depth || pr.second->depth != a0.depth)
            throw Error(CKKS_E_PARAM_MISMATCH, "product operands at different depths");
        if (pr.first->scale * pr.second->scale != s)
            throw Error(CKKS_E_PARAM_MISMATCH, "lazy sum of products with different scales");
        count = std::max(count, std::max(pr.first->count, pr.second->count));
    }
    for (auto &pr : pairs)
        if (count % pr.first->count != 0 || count % pr.second->count != 0)
            throw Error(CKKS_E_PARAM_MISMATCH, "batch counts differ");
    const int l = a0.limbs;
    const size_t N = (size_t)c.p.n;
    DBuf d(c.pool.get(), (size_t)count * 3 * l * N);
    if (pairs.size() == 1) {
        k_tensor(c.tab, d.ptr, a0.data.ptr, b0.data.ptr, count, l, a0.count, b0.count, false, c.stream);
        ++c.n_launch;
    } else {
        // the pairs' tensors summed in registers, kMaxTensorPairs per launch
        for (size_t i0 = 0; i0 < pairs.size(); i0 += kMaxTensorPairs) {
            TensorPairs tp{};
            tp.n = (int)std::min(pairs.size() - i0, (size_t)kMaxTensorPairs);
            for (int p = 0; p < tp.n; ++p) {
                tp.a[p] = pairs[i0 + p].first->data.ptr;
                tp.b[p] = pairs[i0 + p].second->data.ptr;
                tp.na[p] = pairs[i0 + p].first->count;
                tp.nb[p] = pairs[i0 + p].second->count;
            }
            k_tensor_sum(c.tab, d.ptr, tp, count, l, i0 > 0, c.stream);
            ++c.n_launch;
        }
    }
    return relin_rescale(c, std::move(d), count, a0.depth, l, a0.scale, b0.scale);
}

// relinearise the tensors d ([count][3][l][N]): (d0, d1) + KS(d2, s^2 key), then rescale; result scale
// (sa * sb) / q
Ct relin_rescale(ckks_ctx &c, DBuf d, int count, int depth, int l, double sa, double sb) {
    const u64 q = c.p.dropped_at(depth);
    Ct r = new_ct(c, count, depth + 1, (sa * sb) / (double)q);
    keyswitch_rescale(c, d.ptr, count, l, r->data.ptr);
    return r;
}

// the products a_i * b_i of several pairs (each relinearised and rescaled, as mul) as consecutive
// ciphertexts of one batch: pair i gives max(a_i.count, b_i.count) ciphertexts.  One tensor launch per pair
// and one key switch for the whole batch; every pair at one depth and one product scale.
Ct mul_stack(ckks_ctx &c, const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &pairs) {
    if (pairs.empty()) throw Error(CKKS_E_INVALID_ARG, "empty product stack");
    const ckks_ct &a0 = *pairs[0].first, &b0 = *pairs[0].second;
    const double s = a0.scale * b0.scale;
    int total = 0;
    std::vector<int> cnt;
    for (auto &pr : pairs) {
        if (pr.first->depth != a0.depth || pr.second->depth != a0.depth)
            throw Error(CKKS_E_PARAM_MISMATCH, "product operands at different depths");
        if (pr.first->scale * pr.second->scale != s)
            throw Error(CKKS_E_PARAM_MISMATCH, "stacked products with different scales");
        const int n = std::max(pr.first->count, pr.second->count);
        if (n % pr.first->count != 0 || n % pr.second->count != 0)
            throw Error(CKKS_E_PARAM_MISMATCH, "batch counts differ");
        cnt.push_back(n);
        total += n;
    }
    const int l = a0.limbs;
    const size_t N = (size_t)c.p.n;
    DBuf d(c.pool.get(), (size_t)total * 3 * l * N);
    size_t off = 0;
    for (size_t i = 0; i < pairs.size(); ++i) {
        k_tensor(c.tab, d.ptr + off, pairs[i].first->data.ptr, pairs[i].second->data.ptr, cnt[i], l,
                 pairs[i].first->count, pairs[i].second->count, false, c.stream);
        ++c.n_launch;
        off += (size_t)cnt[i] * 3 * l * N;
    }
    return relin_rescale(c, std::move(d), total, a0.depth, l, a0.scale, b0.scale);
}

// sum_i cols_i (x) rep_{b, i} for every batch b (CP-REP-MatMult of the M-materialised layout): one
// tensor-sum launch, one relinearisation and one rescale for the chunk
Ct mul_sum_rep(ckks_ctx &c, const ckks_ct &cols, const ckks_ct &rep) {
    const int n_rows = cols.count, cnt = rep.count / cols.count;
    if (cnt * n_rows != rep.count || cnt < 1) throw Error(CKKS_E_PARAM_MISMATCH, "REP rows do not fill whole batches");
    if (cols.depth != rep.depth) throw Error(CKKS_E_PARAM_MISMATCH, "product operands at different depths");
    const int l = cols.limbs;
    DBuf d(c.pool.get(), (size_t)cnt * 3 * l * c.p.n);
    k_tensor_rep_sum(c.tab, d.ptr, cols.data.ptr, rep.data.ptr, cnt, n_rows, l, c.stream);
    ++c.n_launch;
    return relin_rescale(c, std::move(d), cnt, cols.depth, l, cols.scale, rep.scale);
}

// c0 of ciphertext i plus the exact indicator of the slots = i mod R at a's scale (the block-start mask
// moved by the automorphism of a right rotation by i)
Ct add_slot_indicators(ckks_ctx &c, const ckks_ct &a, int R) {
    const int l = a.limbs;
    const u64 *pt = mask_plain(c, R, l, a.scale);
    Ct r = new_ct(c, a.count, a.depth, a.scale);
    k_add_rotated_plain(c.tab, r->data.ptr, a.data.ptr, pt, a.count, l, R, c.stream);
    ++c.n_launch;
    return r;
}

Ct mul(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b) { return mul_sum(c, {{&a, &b}}); }

u64 galois_rotate_n(int n, i64 r) {
    const u64 m = 2ULL * (u64)n;
    i64 rr = r % (n / 2);
    if (rr < 0) rr += n / 2;   // 5 has order N/2 modulo 2N
    return powmod_host(5, (u64)rr, m);
}

u64 galois_rotate(const ckks_ctx &c, i64 r) { return galois_rotate_n(c.p.n, r); }

u64 galois_conj(const ckks_ctx &c) { return 2ULL * (u64)c.p.n - 1; }

// sigma_g(a) switched back to s: c0 permuted, and the key switch of sigma_g(c1) reads the digits of c1
// through the automorphism after the basis extension
Ct apply_galois(ckks_ctx &c, const ckks_ct &a, u64 g) {
    const int l = a.limbs;
    const KsKeys keys = ks_keys(c, {g}, true);
    // (sigma_g(a c0), 0) added by the ModDown epilogue
    DBuf ks = keyswitch(c, Gather{a.data.ptr, l, 2 * l, l, 1, kPlain, 0}, a.count, l, keys, Gather{}, false,
                        a.data.ptr, false);
    Ct r(new ckks_ct());
    r->ctx = &c;
    r->count = a.count;
    r->depth = a.depth;
    r->limbs = l;
    r->scale = a.scale;
    r->data = std::move(ks);
    return r;
}

Ct rotate_sum(ckks_ctx &c, const ckks_ct &a, const std::vector<i64> &rots) {
    const int l = a.limbs;
    std::vector<u64> gs;
    for (i64 r : rots) gs.push_back(galois_rotate(c, r));
    const KsKeys keys = ks_keys(c, gs, true);
    // a + (sum_i sigma_i(a c0), 0), added by the ModDown epilogue; beyond 3 rotations the sum of the
    // automorphisms is formed first (aut_sum, along the rotation lines) and added as one term
    DBuf ks;
    if (keys.m <= 3) {
        ks = keyswitch(c, Gather{a.data.ptr, l, 2 * l, l, 1, kPlain, 0}, a.count, l, keys, Gather{}, false, a.data.ptr,
                       true);
    } else {
        DBuf z(c.pool.get(), (size_t)a.count * l * c.p.n);
        // rotations r1, 2 r1, .., (m - 1) r1 (a grouped rotate-and-sum step): the doubling form
        bool arith = true;
        for (size_t i = 0; i < rots.size(); ++i) arith = arith && rots[i] == (i64)(i + 1) * rots[0];
        if (!(arith && aut_sum_doubling(c.tab, z.ptr, a.data.ptr, a.count, l, rots[0], (int)rots.size() + 1, gs[0],
                                        c.stream)))
            k_aut_sum(c.tab, z.ptr, a.data.ptr, a.count, l, keys, c.stream);
        // z = c0 + sum_i sigma_i(c0) on the even rows; the odd rows add c1 itself
        ks = keyswitch(c, Gather{a.data.ptr, l, 2 * l, l, 1, kPlain, 0}, a.count, l, keys,
                       Gather{z.ptr, 2 * l, l, 0, 1, kPlain, 0}, true, a.data.ptr, 2, false);
    }
    Ct r(new ckks_ct());
    r->ctx = &c;
    r->count = a.count;
    r->depth = a.depth;
    r->limbs = l;
    r->scale = a.scale;
    r->data = std::move(ks);
    return r;
}

Ct rotate(ckks_ctx &c, const ckks_ct &a, i64 r) { return apply_galois(c, a, galois_rotate(c, r)); }

std::vector<Ct> rotate_many(ckks_ctx &c, const ckks_ct &a, const std::vector<i64> &rots) {
    const int l = a.limbs;
    const Gather d{a.data.ptr, l, 2 * l, l, 1, kPlain, 0};
    std::vector<Ct> out;
    if (rots.empty()) return out;
    // algorithmic bytes as for keyswitch: the input once, then per rotation its key and the two outputs
    const int al = c.p.alpha, nt = l + al, groups = 1 + l / al;
    const double bytes = 8.0 * (double)c.p.n *
                         ((double)a.count * l + (double)rots.size() * (2.0 * groups * nt + (double)a.count * 4.0 * l));
    KRegion region_(c.tab.timer, "keyswitch", bytes, c.stream);
    DBuf dig = mod_up(c, d, a.count, l);
    for (i64 rr : rots) {
        const KsKeys keys = ks_keys(c, {galois_rotate(c, rr)}, true);
        Ct r(new ckks_ct());
        r->ctx = &c;
        r->count = a.count;
        r->depth = a.depth;
        r->limbs = l;
        r->scale = a.scale;
        r->data = ks_inner_down(c, dig.ptr, d, a.count, l, keys, Gather{}, false, a.data.ptr, false, true);
        out.push_back(std::move(r));
    }
    return out;
}
Ct conjugate(ckks_ctx &c, const ckks_ct &a) { return apply_galois(c, a, galois_conj(c)); }

// ---------------------------------------------------------------- keys

static u64 os_seed() {
    std::random_device rd;
    u64 s = ((u64)rd() << 32) ^ (u64)rd();
    return s ? s : 1;
}

static u64 sm_mix_host(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static u64 sm_out_host(u64 x, u64 i) { return sm_mix_host(x + (i + 1) * 0x9E3779B97F4A7C15ULL); }

// HWT(h) secret: positions w mod N of successive stream words, sign from the top bit, repeats skipped.
static std::vector<i64> sample_hwt_host(u64 seed, u64 sid, int n, int h) {
    std::vector<i64> s(n, 0);
    const u64 st = sm_out_host(seed, sid);
    int got = 0;
    if (h > n) h = n;
    for (u64 cc = 0; got < h; ++cc) {
        u64 w = sm_out_host(st, cc);
        int pos = (int)(w % (u64)n);
        if (s[pos]) continue;
        s[pos] = (w >> 63) ? -1 : 1;
        ++got;
    }
    return s;
}

static u64 ksk_sid_base(u64 key_id) { return (1ULL << 40) | (key_id << 20); }

// switching key for target secret sp (NTT form, L+1 limbs over q_0..q_L) under key id:
// [2][ng][L+1+alpha][N], for group b and target t (q_0..q_L, p_1..p_alpha)
//   key[0][b][t] = -a_b s + e_b + [t in group b] (P mod q_t) s'_t,  key[1][b][t] = a_b,
// a_b uniform (stream base + 2b, modulus index t), e_b centred binomial (stream base + 2b + 1); stored in
// NTT and Montgomery form.
static void make_switching_key(ckks_ctx &c, u64 seed, u64 key_id, const u64 *sp) {
    const int L = c.p.levels, nt = c.p.n_mods(), ng = c.ng, P = c.p.p_index();
    const size_t N = (size_t)c.p.n;
    const ModMap mt{nt, L + 1, P};          // targets q_0..q_L, p_1..p_alpha
    DBuf key(c.pool.get(), (size_t)2 * ng * nt * N);
    DBuf e_small(c.pool.get(), N);
    DBuf as(c.pool.get(), (size_t)nt * N);
    const u64 base = ksk_sid_base(key_id);
    for (int b = 0; b < ng; ++b) {
        u64 *kb = key.ptr + (size_t)b * nt * N;
        u64 *ka = key.ptr + ((size_t)ng + b) * nt * N;
        k_sample_uniform(c.tab, ka, seed, base + 2ULL * b, nt, mt, P, c.stream);
        ntt_fwd(c, ka, nt, mt);
        k_sample_cbd(reinterpret_cast<i64 *>(e_small.ptr), seed, base + 2ULL * b + 1, (int)N, c.stream);
        k_signed_to_limbs(c.tab, kb, reinterpret_cast<const i64 *>(e_small.ptr), nt, mt, c.stream);
        ntt_fwd(c, kb, nt, mt);
        k_mul(c.tab, as.ptr, ka, c.sk_ntt.ptr, nt, mt, nt, nt, c.stream);
        k_sub(c.tab, kb, kb, as.ptr, nt, mt, nt, nt, c.stream);
        const int f = ks_group_first(b, c.p.alpha), m = ks_group_size(b, L + 1, c.p.alpha);
        for (int t = f; t < f + m; ++t) {   // + (P mod q_t) s'_t on the group's own targets
            const u64 q = c.p.q[t];
            u64 v = 1;
            for (u64 pk : c.p.P) v = mulmod_host(v, pk % q, q);
            ChainConst pj{};
            pj.v[t] = v;
            pj.sh[t] = (u64)(((u128)v << 64) / q);
            k_mul_const(c.tab, as.ptr, sp + (size_t)t * N, 1, ModMap{1, 0, t}, pj, c.stream);
            k_add(c.tab, kb + (size_t)t * N, kb + (size_t)t * N, as.ptr, 1, ModMap{1, 0, t}, 1, 1, c.stream);
        }
        c.n_launch += 8;
    }
    k_to_mont(c.tab, key.ptr, 2 * ng * nt, mt, c.stream);
    c.ksk[key_id] = std::move(key);
}

void keygen(ckks_ctx &c, u64 seed, const std::vector<u64> &galois) {
    if (seed == 0) seed = os_seed();
    const int L = c.p.levels, P = c.p.p_index(), nt = c.p.n_mods();
    const int n = c.p.n;
    const size_t N = (size_t)n;
    const ModMap mt{nt, L + 1, P};
    c.ksk.clear();
    c.sk = sample_hwt_host(seed, 1, n, std::min(64, n / 2));
    DBuf small(c.pool.get(), N);
    GCK_HIP(hipMemcpyAsync(small.ptr, c.sk.data(), N * 8, hipMemcpyHostToDevice, c.stream));
    c.sk_ntt = DBuf(c.pool.get(), (size_t)nt * N);
    k_signed_to_limbs(c.tab, c.sk_ntt.ptr, reinterpret_cast<const i64 *>(small.ptr), nt, mt, c.stream);
    ntt_fwd(c, c.sk_ntt.ptr, nt, mt);
    // public key over q_0..q_L
    c.pk = DBuf(c.pool.get(), (size_t)2 * (L + 1) * N);
    u64 *pb = c.pk.ptr, *pa = c.pk.ptr + (size_t)(L + 1) * N;
    k_sample_uniform(c.tab, pa, seed, 2, L + 1, map_q(L + 1), P, c.stream);
    ntt_fwd(c, pa, L + 1, map_q(L + 1));
    k_sample_cbd(reinterpret_cast<i64 *>(small.ptr), seed, 3, n, c.stream);
    k_signed_to_limbs(c.tab, pb, reinterpret_cast<const i64 *>(small.ptr), L + 1, map_q(L + 1), c.stream);
    ntt_fwd(c, pb, L + 1, map_q(L + 1));
    DBuf as(c.pool.get(), (size_t)(L + 1) * N);
    k_mul(c.tab, as.ptr, pa, c.sk_ntt.ptr, L + 1, map_q(L + 1), L + 1, L + 1, c.stream);
    k_sub(c.tab, pb, pb, as.ptr, L + 1, map_q(L + 1), L + 1, L + 1, c.stream);
    // relinearisation key: s' = s^2
    DBuf sp(c.pool.get(), (size_t)(L + 1) * N);
    k_mul(c.tab, sp.ptr, c.sk_ntt.ptr, c.sk_ntt.ptr, L + 1, map_q(L + 1), L + 1, L + 1, c.stream);
    make_switching_key(c, seed, 0, sp.ptr);
    // Galois keys: s' = s(X^g), an NTT-domain permutation of s
    for (u64 g : galois) {
        if ((g & 1) == 0 || g >= 2ULL * N) throw Error(CKKS_E_INVALID_ARG, "Galois element must be odd and < 2N");
        if (c.ksk.count(g)) continue;
        k_automorph(c.tab, sp.ptr, c.sk_ntt.ptr, L + 1, g, c.stream);
        make_switching_key(c, seed, g, sp.ptr);
    }
    c.have_secret = true;
    c.have_pk = true;
    sync(c);
}

// every residue of limb i of buf (limbs of N words) below the modulus of chain index chain(i)
template <typename F>
static void check_residues(const ckks_ctx &c, const u64 *buf, size_t limbs, F chain) {
    const size_t N = (size_t)c.p.n;
    for (size_t i = 0; i < limbs; ++i) {
        const u64 q = c.h_mods[chain(i)].q;
        const u64 *row = buf + i * N;
        for (size_t k = 0; k < N; ++k)
            if (row[k] >= q) throw Error(CKKS_E_INVALID_ARG, "imported key residue out of range");
    }
}

void import_public_key(ckks_ctx &c, const u64 *buf) {
    const int l = c.p.levels + 1;
    const size_t N = (size_t)c.p.n;
    check_residues(c, buf, (size_t)2 * l, [&](size_t i) { return (int)(i % l); });
    DBuf pk(c.pool.get(), (size_t)2 * l * N);
    GCK_HIP(hipMemcpyAsync(pk.ptr, buf, (size_t)2 * l * N * 8, hipMemcpyHostToDevice, c.stream));
    ntt_fwd(c, pk.ptr, 2 * l, map_q(l));
    sync(c);   // the caller's buffer may be reused after return
    c.pk = std::move(pk);
    c.have_pk = true;
}

void import_switching_key(ckks_ctx &c, u64 key_id, const u64 *buf) {
    const int L = c.p.levels, nt = c.p.n_mods(), ng = c.ng, P = c.p.p_index();
    const size_t N = (size_t)c.p.n;
    if (key_id != 0 && ((key_id & 1) == 0 || key_id >= 2 * N))
        throw Error(CKKS_E_INVALID_ARG, "key id must be 0 (relinearisation) or an odd Galois element < 2N");
    const ModMap mt{nt, L + 1, P};
    check_residues(c, buf, (size_t)2 * ng * nt, [&](size_t i) {
        const int t = (int)(i % nt);
        return t <= L ? t : P + (t - (L + 1));
    });
    DBuf key(c.pool.get(), (size_t)2 * ng * nt * N);
    GCK_HIP(hipMemcpyAsync(key.ptr, buf, key.words * 8, hipMemcpyHostToDevice, c.stream));
    ntt_fwd(c, key.ptr, 2 * ng * nt, mt);
    k_to_mont(c.tab, key.ptr, 2 * ng * nt, mt, c.stream);
    sync(c);
    c.ksk[key_id] = std::move(key);
}

Ct encrypt(ckks_ctx &c, const i64 *m, int depth, double scale, u64 seed) {
    if (!c.have_pk) throw Error(CKKS_E_KEY_MISSING, "no public key in this context (keygen or import one)");
    if (seed == 0) seed = os_seed();
    const int n = c.p.n;
    const size_t N = (size_t)n;
    Ct r = new_ct(c, 1, depth, scale);
    const int l = r->limbs;
    DBuf sm(c.pool.get(), 4 * N);   // m, v, e0, e1 (signed)
    i64 *dm = reinterpret_cast<i64 *>(sm.ptr), *dv = dm + N, *de0 = dm + 2 * N, *de1 = dm + 3 * N;
    GCK_HIP(hipMemcpyAsync(dm, m, N * 8, hipMemcpyHostToDevice, c.stream));
    k_sample_ternary(dv, seed, 1, n, c.stream);
    k_sample_cbd(de0, seed, 2, n, c.stream);
    k_sample_cbd(de1, seed, 3, n, c.stream);
    DBuf v(c.pool.get(), (size_t)l * N), t(c.pool.get(), (size_t)l * N);
    k_signed_to_limbs(c.tab, v.ptr, dv, l, map_q(l), c.stream);
    ntt_fwd(c, v.ptr, l, map_q(l));
    u64 *c0 = r->data.ptr, *c1 = r->data.ptr + (size_t)l * N;
    // c0 = v pk0 + m + e0
    k_mul(c.tab, c0, v.ptr, c.pk.ptr, l, map_q(l), l, l, c.stream);
    k_signed_to_limbs(c.tab, t.ptr, dm, l, map_q(l), c.stream);
    ntt_fwd(c, t.ptr, l, map_q(l));
    k_add(c.tab, c0, c0, t.ptr, l, map_q(l), l, l, c.stream);
    k_signed_to_limbs(c.tab, t.ptr, de0, l, map_q(l), c.stream);
    ntt_fwd(c, t.ptr, l, map_q(l));
    k_add(c.tab, c0, c0, t.ptr, l, map_q(l), l, l, c.stream);
    // c1 = v pk1 + e1
    k_mul(c.tab, c1, v.ptr, c.pk.ptr + (size_t)(c.p.levels + 1) * N, l, map_q(l), l, l, c.stream);
    k_signed_to_limbs(c.tab, t.ptr, de1, l, map_q(l), c.stream);
    ntt_fwd(c, t.ptr, l, map_q(l));
    k_add(c.tab, c1, c1, t.ptr, l, map_q(l), l, l, c.stream);
    sync(c);   // the caller's host buffer m may be reused after return
    return r;
}

std::vector<long double> decrypt_poly(ckks_ctx &c, const ckks_ct &a, int index) {
    if (!c.have_secret) throw Error(CKKS_E_KEY_MISSING, "no secret key in this context (an evaluating context)");
    const int n = c.p.n;
    const size_t N = (size_t)n;
    const int l = a.limbs, lu = std::min(l, 2);
    const u64 *c0 = a.data.ptr + (size_t)index * 2 * l * N, *c1 = c0 + (size_t)l * N;
    DBuf t(c.pool.get(), (size_t)lu * N);
    k_mul(c.tab, t.ptr, c1, c.sk_ntt.ptr, lu, map_q(lu), lu, lu, c.stream);
    k_add(c.tab, t.ptr, t.ptr, c0, lu, map_q(lu), lu, lu, c.stream);
    ntt_inv(c, t.ptr, lu, map_q(lu));
    std::vector<u64> h((size_t)lu * N);
    GCK_HIP(hipMemcpyAsync(h.data(), t.ptr, h.size() * 8, hipMemcpyDeviceToHost, c.stream));
    sync(c);
    std::vector<long double> out(N);
    const u64 q0 = c.p.q[0];
    if (lu == 1) {
        for (size_t k = 0; k < N; ++k) {
            u64 x = h[k];
            out[k] = x > q0 / 2 ? -(long double)(q0 - x) : (long double)x;
        }
    } else {
        const u64 q1 = c.p.q[1];
        const u64 inv = invmod_host(q0 % q1, q1);
        const u128 Q = (u128)q0 * q1;
        for (size_t k = 0; k < N; ++k) {
            u64 x0 = h[k], x1 = h[N + k];
            u64 d = (x1 + q1 - x0 % q1) % q1;
            u64 tq = mulmod_host(d, inv, q1);
            u128 x = (u128)x0 + (u128)q0 * tq;
            out[k] = x > Q / 2 ? -(long double)(Q - x) : (long double)x;
        }
    }
    return out;
}

void export_ct(ckks_ctx &c, const ckks_ct &a, int index, u64 *out) {
    const size_t N = (size_t)c.p.n;
    const int l = a.limbs;
    DBuf t(c.pool.get(), (size_t)2 * l * N);
    GCK_HIP(hipMemcpyAsync(t.ptr, a.data.ptr + (size_t)index * 2 * l * N, (size_t)2 * l * N * 8,
                           hipMemcpyDeviceToDevice, c.stream));
    ntt_inv(c, t.ptr, 2 * l, map_q(l));
    GCK_HIP(hipMemcpyAsync(out, t.ptr, (size_t)2 * l * N * 8, hipMemcpyDeviceToHost, c.stream));
    sync(c);
}

Ct import_ct(ckks_ctx &c, const u64 *in, int depth, double scale) {
    Ct r = new_ct(c, 1, depth, scale);
    const int l = r->limbs;
    const size_t N = (size_t)c.p.n;
    for (int i = 0; i < 2 * l; ++i) {
        const u64 q = c.p.q[i % l];
        for (size_t k = 0; k < N; ++k)
            if (in[(size_t)i * N + k] >= q) throw Error(CKKS_E_INVALID_ARG, "imported residue out of range");
    }
    GCK_HIP(hipMemcpyAsync(r->data.ptr, in, (size_t)2 * l * N * 8, hipMemcpyHostToDevice, c.stream));
    ntt_fwd(c, r->data.ptr, 2 * l, map_q(l));
    sync(c);
    return r;
}

}  // namespace gck

// ---------------------------------------------------------------- context teardown
ckks_ctx::~ckks_ctx() {
    if (stream) hipStreamSynchronize(stream);
    else hipDeviceSynchronize();
    if (aux_stream) hipStreamSynchronize(aux_stream);
    mask_cache.clear();   // entries may come from either pool
    mono_cache.clear();
    aux_pool.reset();
    ksk.clear();   // every pool-backed member goes back to the pool before the pool is destroyed
    sk_ntt.release();
    pk.release();
    pool.reset();
    if (table_mem) (void)hipFree(table_mem);
    if (ks_mem) (void)hipFree(ks_mem);
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    if (aux_stream) (void)hipStreamDestroy(aux_stream);
}
