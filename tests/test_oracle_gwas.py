"""Pins of the FP64 GWAS oracle and of the encrypted circuit on the CPU oracle (no GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import ckks as C
from oracle import gwas_circuit as G
from oracle import gwas_fp64 as F
from synth import config_seed, make_gwas_data

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        return json.load(f)


def test_sigma7_coefficients_and_sign_reading():
    g = _golden()["sigma7_coefficients"]
    assert (F.SIGMA7_C1, F.SIGMA7_C3, F.SIGMA7_C5, F.SIGMA7_C7) == (g["c1"], g["c3"], g["c5"], g["c7"])
    x = np.linspace(-8, 8, 2001)
    sig = 1 / (1 + np.exp(-x))
    # sign-corrected polynomial approximates the sigmoid on [-8, 8]; the printed one is its mirror image
    assert np.max(np.abs(F.sigma7(x) - sig)) < 0.033
    assert np.allclose(F.sigma7_printed(x), F.sigma7(-x))
    assert F.sigma7(np.array([0.0]))[0] == g["constant"]
    # closed form at x = 8 (u = 1)
    assert abs(F.sigma7(np.array([8.0]))[0] - (0.5 + g["c1"] - g["c3"] + g["c5"] - g["c7"])) < 1e-15


def test_inverse_slots_closed_form():
    g = _golden()["inverse_slots"]
    w = np.linspace(1e-3, g["w_upper_bound"], 500)
    got = F.inverse_slots(w, g["iterations"], g["guess"])
    # Newton from g0 = 3: 1 - w g_k = (1 - 3 w)^(2^k)
    assert np.allclose(got, (1 - (1 - 3 * w) ** 8) / w, rtol=1e-12, atol=0)
    assert abs(F.inverse_slots(np.array([0.25]))[0] * 0.25 - 1) < 2e-5


def test_complex_packing_identities():
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(100), rng.standard_normal(100)
    z = x + 1j * y
    assert np.allclose(((z * np.conj(z) + z * z) / 2).real, x * x)
    assert np.allclose(((z * np.conj(z) - z * z) / 2).real, y * y)


@pytest.fixture(scope="module")
def data():
    return make_gwas_data(245, 4, 33, seed=config_seed(1))


def test_projection_invariants(data):
    r = F.modified_gwas(data.X, data.y, data.S, 3)
    X = data.X
    scale = np.max(np.abs(X.T @ data.S.astype(float)))
    assert np.max(np.abs(X.T @ r.S_proj)) < 1e-10 * scale
    assert np.max(np.abs(X.T @ r.z_proj)) < 1e-10 * np.max(np.abs(X.T @ r.z))
    A = F.xtx_inverse(X)
    M = np.eye(X.shape[0]) - X @ A @ X.T
    assert np.allclose(M, M.T, atol=1e-12)
    assert np.allclose(M @ M, M, atol=1e-10)
    assert np.allclose(A @ (X.T @ X), np.eye(X.shape[1]), atol=1e-10)
    # the packed (two SNPs per complex slot) numerator / denominator equal the plain ones
    num, den = F.packed_num_den(r.w, r.z_proj, r.S_proj)
    assert np.allclose(num, r.num, rtol=1e-12, atol=1e-9)
    assert np.allclose(den, r.den, rtol=1e-12)
    # z' does not depend on beta (M X = 0): with beta's sign flipped it is the same
    z2 = -X @ r.beta + r.w_inv * (data.y - r.p)
    assert np.allclose(z2 - X @ (A @ (X.T @ z2)), r.z_proj, atol=1e-9)


def test_fixed_hessian_newton_converges_to_mle(data):
    """homomorphic_logreg_plain with the exact sigmoid and many passes reaches the IRLS maximum-likelihood
    fit (pins the ascent sign of the update, reading of eq. updateBeta with the lower-bound Hessian)."""
    X, y = data.X, data.y
    A = F.xtx_inverse(X)
    beta, _ = F.homomorphic_logreg_plain(X, y, A, 300, sig=F.sigmoid)
    assert np.allclose(beta, F.irls_logreg(X, y), atol=1e-8)


def test_homomorphic_logreg_iterates(data):
    """Closed forms of the first passes: p^(0) = sigma7(0) = 1/2 everywhere and beta^(1) = 4 A X^T (y - 1/2);
    the p returned with beta^(kappa) is the one of the last pass, p^(kappa-1) = sigma7(X beta^(kappa-1))."""
    X, y = data.X, data.y
    A = F.xtx_inverse(X)
    b1, p0 = F.homomorphic_logreg_plain(X, y, A, 1)
    assert np.all(p0 == 0.5)
    assert np.allclose(b1, 4 * A @ (X.T @ (y - 0.5)), rtol=1e-13, atol=1e-15)
    b2, p1 = F.homomorphic_logreg_plain(X, y, A, 2)
    assert np.allclose(p1, F.sigma7(X @ b1), rtol=1e-14)
    assert np.allclose(b2, b1 + 4 * A @ (X.T @ (y - p1)), rtol=1e-12, atol=1e-15)
    b3, p2 = F.homomorphic_logreg_plain(X, y, A, 3)
    assert np.allclose(p2, F.sigma7(X @ b2), rtol=1e-14)
    assert not np.allclose(p2, F.sigma7(X @ b3), rtol=1e-6)   # not the p of beta^(kappa)


def test_sikorska_close_to_brute_force():
    d = make_gwas_data(120, 3, 8, seed=5)
    b_sp, err = F.sikorska_gwas(d.X, d.y, d.S)
    b_bf, se_bf = F.per_snp_logreg(d.X, d.y, d.S)
    # a one-step score approximation of the per-SNP fits: close, not equal
    assert np.max(np.abs(b_sp - b_bf) / np.maximum(se_bf, 1e-9)) < 0.2
    assert np.allclose(np.sqrt(err), se_bf, rtol=0.2)


def test_modified_gwas_tracks_exact_semi_parallel(data):
    r = F.modified_gwas(data.X, data.y, data.S, 3)
    b_sp, err = F.sikorska_gwas(data.X, data.y, data.S)
    ok = np.isfinite(r.b)
    assert np.corrcoef(r.b[ok], b_sp[ok])[0, 1] > 0.95


@pytest.mark.slow
def test_encrypted_circuit_on_oracle_matches_fp64_small():
    """The whole encrypted circuit on the oracle (N = 2^10, 40-bit scale) against the FP64 GWAS."""
    n, k, m, kappa = 30, 4, 70, 3
    p = C.make_params(10, G.circuit_depth(kappa), 40)
    d = make_gwas_data(n, k, m, seed=77)
    lay = G.make_layout(p.N, n, k, m)
    assert lay.n_batches == 3 and m % lay.tau != 0       # ragged last batch
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    pts = G.encode_inputs(p, d.X, d.y, d.S, kappa)
    inp = G.encrypt_inputs(o, pts, n, k, m, kappa, 11)
    out = G.Circuit(o, lay).run(inp)
    assert out.den_even[0].depth == p.L and out.num[0].depth == p.L - 1
    num, den, b, err, se = G.finalize(o, lay, out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    tol = np.maximum(np.abs(ref.b), ref.se)
    assert np.max(np.abs(b - ref.b) / tol) < 1e-4
    beta = np.array([o.decrypt(c)[0].real for c in out.beta])
    assert np.allclose(beta, ref.beta, atol=1e-5)


@pytest.mark.slow
def test_encrypted_circuit_on_oracle_config1_accuracy():
    """Workload n=245, k=4, m=32, N=2^13, scale 2^30: decrypted b' within 1e-3 of the FP64 GWAS."""
    n, k, m, kappa = 245, 4, 32, 3
    p = C.make_params(13, G.circuit_depth(kappa), 30)
    d = make_gwas_data(n, k, m, seed=config_seed(1))
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    out = G.Circuit(o, lay).run(inp)
    num, den, b, err, se = G.finalize(o, lay, out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    assert np.max(np.abs(b - ref.b) / np.maximum(np.abs(ref.b), ref.se)) < 1e-3


def test_accuracy_methods_against_paper_tables():
    """The paper's two accuracy methods: the count of entries differing by more than e with the accuracy
    percentage 100 (1 - count / m) (both printed in the HEAAN and SEAL accuracy tables, m = 10643), and the
    least-squares line of b' (y) against b (x)."""
    g = _golden()["accuracy_tables"]
    m = g["m"]
    rng = np.random.default_rng(12)
    b_ref = rng.standard_normal(m)
    for lib in ("heaan", "seal"):
        rows = g[lib]["rows"]
        # differences placed so that exactly the printed number of entries exceeds each e
        diff = np.zeros(m)
        order = rng.permutation(m)
        n01, n001, n0005 = (r[1] for r in rows)
        diff[order[:n0005]] = 0.0075                 # above 0.005 only
        diff[order[:n001]] = 0.05                    # above 0.01 too
        diff[order[:n01]] = 0.5                      # above 0.1 too
        got = F.accuracy_counts(b_ref, b_ref + diff * np.sign(rng.standard_normal(m)))
        for e, count, pct in rows:
            assert got[e][0] == count
            assert round(got[e][1], 2) == pct, (lib, e, got[e])
        slope, icpt = g[lib]["fit_line"]
        s, c = F.fit_line(b_ref, slope * b_ref + icpt)
        assert abs(s - slope) < 1e-12 and abs(c - icpt) < 1e-12
        s2, _ = F.fit_line(slope * b_ref + icpt, b_ref)   # swapped axes give the inverse slope
        assert abs(s2 - 1 / slope) < 1e-12


def test_kappa1_weights_are_public_constants(data):
    """kappa = 1 (Discussion: the SEAL run): the only Newton pass starts at beta = 0, so p = sigma7(0) = 1/2,
    w = 1/4 and w^-1 = inverseSlots(1/4) = 4 - 2^-14 = (1 - (1 - 3/4)^8) / (1/4) exactly."""
    r = F.modified_gwas(data.X, data.y, data.S, 1)
    assert np.all(r.p == 0.5) and np.all(r.w == 0.25)
    assert np.all(r.w_inv == 4 - 2.0 ** -14) and G.W_INV_KAPPA1 == 4 - 2.0 ** -14
    assert G.W_KAPPA1 == 0.25
    A = F.xtx_inverse(data.X)
    assert np.allclose(r.beta, 4 * A @ (data.X.T @ (data.y - 0.5)), rtol=1e-13, atol=1e-15)
    assert G.circuit_depth(1) == 8 and G.snp_depth(1) == 4
    assert [G.circuit_depth(k) for k in (2, 3)] == [19, 26]


@pytest.mark.parametrize("kappa", [1, 2])
def test_encrypted_circuit_on_oracle_other_kappa_matches_fp64(kappa):
    """The encrypted circuit on the oracle for kappa = 1 (public weights) and 2 against the FP64 GWAS of
    the same kappa (N = 2^10, 40-bit scale, a ragged last SNP batch)."""
    n, k, m = 30, 4, 70
    p = C.make_params(10, G.circuit_depth(kappa), 40)
    d = make_gwas_data(n, k, m, seed=78)
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    out = G.Circuit(o, lay).run(inp)
    assert out.den_even[0].depth == p.L and out.den_odd[0].depth == p.L
    assert (out.w is None) == (kappa == 1) and (out.w_inv is None) == (kappa == 1)
    num, den, b, err, se = G.finalize(o, lay, out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    assert np.max(np.abs(b - ref.b) / np.maximum(np.abs(ref.b), ref.se)) < 1e-4
    assert np.allclose(den, ref.den, rtol=1e-6)
    beta = np.array([o.decrypt(c)[0].real for c in out.beta])
    assert np.allclose(beta, ref.beta, atol=1e-5)
    zp = o.decrypt(out.z_proj).real
    assert np.allclose(zp[:n], ref.z_proj, atol=1e-5)


def test_reciprocal_newton_closed_form():
    """Newton's reciprocal from g_0 = 1 (the division extension): 1 - x g_t = (1 - x)^(2^t) exactly in real
    arithmetic, so t = 5 steps leave a relative error (1 - x)^32 (below 1e-3 for x >= 0.2)."""
    x = np.linspace(0.05, 1.0, 400)
    g = F.reciprocal_newton(x, F.DIV_ITERS, F.DIV_GUESS)
    assert np.allclose(1 - x * g, (1 - x) ** (2 ** F.DIV_ITERS), rtol=1e-9, atol=1e-15)
    assert np.max(np.abs(g * x - 1)[x >= 0.2]) < 1e-3
    assert G.DIV_LEVELS == 3 + 2 * (F.DIV_ITERS - 1)


@pytest.mark.parametrize("kappa", [1, 2, 3])
def test_snp_normalisers_bound_the_denominators(data, kappa):
    """d_j = ||S_j - mean(S_j)||^2 / 4 bounds den_j = sum_i w_i S'_ij^2 from above (w <= 1/4; S' = M S is
    the shortest residual after projecting out X, whose first column is the intercept), so x = den / d lies
    in (0, 1]; a monomorphic SNP has d = 0."""
    r = F.modified_gwas(data.X, data.y, data.S, kappa)
    d = F.snp_normalisers(data.S)
    ok = d > 0
    assert np.all(r.den[ok] <= d[ok] * (1 + 1e-12))
    assert np.all(r.den[ok] > 0.2 * d[ok])
    Sc = data.S.astype(float) - data.S.astype(float).mean(axis=0)
    assert np.all((r.S_proj ** 2).sum(axis=0) <= (Sc ** 2).sum(axis=0) * (1 + 1e-12))
    S0 = data.S.copy()
    S0[:, 0] = 1
    assert F.snp_normalisers(S0)[0] == 0
    b, inv = F.divide_plain(r.num, r.den, d)
    assert np.max(np.abs(b - r.b)[ok] / np.maximum(np.abs(r.b), r.se)[ok]) < 1e-4
    assert np.allclose(inv[ok], r.err[ok], rtol=1e-4)


@pytest.mark.parametrize("kappa", [1, 2])
def test_encrypted_division_on_oracle(kappa):
    """b' and err' as ciphertexts (Newton reciprocal of the normalised denominators) on a chain longer by
    DIV_LEVELS: decrypted directly, they match the FP64 division of the same steps and the FP64 GWAS."""
    n, k, m = 30, 4, 70
    p = C.make_params(10, G.circuit_depth(kappa) + G.DIV_LEVELS, 40)
    d = make_gwas_data(n, k, m, seed=77)
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    out = G.Circuit(o, lay).run(inp)
    v = G.encrypt_normalisers(o, G.encode_normalisers(p, d.S, lay, kappa), kappa, 11)
    assert len(v) == 2 * lay.n_batches and v[0].scale == G.normaliser_scale(p, kappa)
    dv = G.divide_all(o, out, v)
    assert dv.b_even[0].depth == p.L and dv.inv_odd[-1].depth == p.L - 1
    b, err, se = G.finalize_divided(o, lay, dv)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    bd, invd = F.divide_plain(ref.num, ref.den, F.snp_normalisers(d.S))
    assert np.max(np.abs(b - bd)[ok] / np.maximum(np.abs(bd), np.sqrt(invd))[ok]) < 1e-6
    assert np.allclose(err[ok], invd[ok], rtol=1e-6)
    assert np.max(np.abs(b - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok]) < 1e-4


def test_slot_class_indicator_is_the_rotated_mask():
    """Dup(e_i) of the M layout: the exact encoding of 1 at slots = i mod R is the block-start mask moved
    by the automorphism of a right rotation by i; it decodes to the indicator and is the mask for i = 0."""
    N, R, sc = 1024, 32, 2.0 ** 40
    assert np.array_equal(C.slot_class_indicator_poly(N, R, 0, sc), C.mask_block_start_poly(N, R, sc))
    for i in (1, 7, 31):
        m = C.slot_class_indicator_poly(N, R, i, sc)
        assert np.count_nonzero(m) == np.count_nonzero(C.mask_block_start_poly(N, R, sc))
        z = C.decode_poly(m.astype(np.float64) / sc, N)
        assert np.max(np.abs(z - (np.arange(N // 2) % R == i))) < 1e-9


@pytest.mark.parametrize("kappa", [1, 3])
def test_m_materialised_layout_on_oracle(kappa):
    """The M-materialised layout (Alg. CP-REP-MatMult): the n duplicated columns of M = I - X A X^T decrypt
    to FP64 M, S' = sum_i Dup(M_i) S_rep(i) decrypts to the S' of the factorised layout, and b' matches the
    FP64 GWAS (N = 2^10, n = 30, a ragged last batch)."""
    n, k, m = 30, 4, 70
    p = C.make_params(10, G.circuit_depth(kappa), 40)
    d = make_gwas_data(n, k, m, seed=77)
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    mi = G.encrypt_inputs_m(o, G.encode_inputs_m(p, d.X, d.S, kappa), n, k, 11)
    assert len(mi.Xrep) == n and len(mi.S_rep) == lay.n_batches and len(mi.S_rep[0]) == n
    out_m = G.Circuit(o, lay, mi).run(inp)
    out = G.Circuit(o, lay).run(inp)
    A = F.xtx_inverse(d.X)
    M = np.eye(n) - d.X @ A @ d.X.T
    cols = np.array([o.decrypt(c).real for c in out_m.m_cols])    # [i][slot]
    for blk in (0, lay.blocks - 1):
        got = cols[:, blk * lay.R:blk * lay.R + lay.R]
        assert np.max(np.abs(got[:, :n].T - M)) < 1e-7          # column i of M over every block
        assert np.max(np.abs(got[:, n:])) < 1e-7                 # padding rows
    for b in range(lay.n_batches):
        assert out_m.S_proj[b].depth == out.S_proj[b].depth
        assert np.max(np.abs(o.decrypt(out_m.S_proj[b]) - o.decrypt(out.S_proj[b]))) < 1e-6
    num, den, bb, err, se = G.finalize(o, lay, out_m)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    assert np.max(np.abs(bb - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok]) < 1e-4


def test_stride_groups_sum_the_multiples_of_k():
    """The stride sums of the packed projection: the rotations of stride_groups(R, K), one shared key
    switch per group, reach every multiple of K below R exactly once (brute force over the products
    of the groups' exponent sets), and every rotation is one of the per-batch rotate-and-sum's."""
    for R in (2, 8, 32, 256, 2048):
        full = {r for grp in G.rotation_groups(R, G.BATCH_RADIX) for r in grp}
        for K in (1, 2, 4, 8, 16):
            if K > min(G.BATCH_RADIX, R):
                continue
            sums = [0]
            for grp in G.stride_groups(R, K):
                sums = [s + r for s in sums for r in [0] + grp]
            assert sorted(sums) == list(range(0, R, K)), (R, K)
            assert all(r in full for grp in G.stride_groups(R, K) for r in grp)


def test_diag_width_conditions():
    lay = lambda n, k, R: G.Layout(N=2 * R, n=n, k=k, m=1, R=R)   # noqa: E731
    assert G.diag_width(lay(245, 4, 256)) == 4
    assert G.diag_width(lay(253, 4, 256)) == 4 and G.diag_width(lay(254, 4, 256)) == 0   # n + K - 1 <= R
    assert G.diag_width(lay(245, 3, 256)) == 4 and G.diag_width(lay(245, 5, 256)) == 8
    assert G.diag_width(lay(200, 16, 256)) == 16 and G.diag_width(lay(200, 17, 256)) == 0   # K <= 16
    assert G.diag_width(lay(245, 1, 256)) == 0                                             # k = 1
    assert G.diag_width(lay(5, 4, 8)) == 4 and G.diag_width(lay(5, 5, 8)) == 0             # K <= R


@pytest.mark.parametrize("kappa,k", [(3, 4), (2, 3), (1, 2)])
def test_packed_projection_on_oracle(kappa, k):
    """The packed projection (reading 21, n = 24 <= R - K + 1 at R = 32): the diagonals decode to
    Z_t[r] = r_{(r + t) mod K}[r] (rotated right by t) and X_t[r] = x_{(r + t) mod K}[r]; S' decrypts to the
    FP64 M S of every batch and to the S' of the M-materialised layout (Alg. CP-REP-MatMult, computed
    without any stride sum); b' matches the FP64 GWAS."""
    n, m = 24, 70
    p = C.make_params(10, G.circuit_depth(kappa), 40)
    d = make_gwas_data(n, k, m, seed=79)
    lay = G.make_layout(p.N, n, k, m)
    K = G.diag_width(lay)
    assert K == (4 if k > 2 else 2) and lay.R == 32 and m % lay.tau != 0
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    circ = G.Circuit(o, lay)
    out = circ.run(inp)
    # the diagonals, from the same r_j and x_j as the circuit
    rr = circ._xa(inp)
    zt, xt = circ.diagonals(inp, rr, G.snp_depth(kappa), K)
    A = F.xtx_inverse(d.X)
    XA = d.X @ A
    rows = np.arange(lay.N // 2) % lay.R
    for t in range(K):
        want_z = np.zeros(lay.N // 2)
        want_x = np.zeros(lay.N // 2)
        for s in range(lay.N // 2):
            r = rows[s]
            j = (r + t) % K
            if r < n and j < k:
                want_z[s] = XA[r, j]
                want_x[s] = d.X[r, j]
        assert np.max(np.abs(o.decrypt(zt[t]) - np.roll(want_z, t))) < 1e-6
        assert np.max(np.abs(o.decrypt(xt[t]) - want_x)) < 1e-6
    M = np.eye(n) - d.X @ A @ d.X.T
    MS = M @ d.S.astype(np.float64)
    mi = G.encrypt_inputs_m(o, G.encode_inputs_m(p, d.X, d.S, kappa), n, k, 11)
    out_m = G.Circuit(o, lay, mi).run(inp)
    for b in range(lay.n_batches):
        got = o.decrypt(out.S_proj[b])
        assert np.max(np.abs(got - G.snp_batch_slots(MS, lay, b))) < 1e-6
        assert out_m.S_proj[b].depth == out.S_proj[b].depth
        assert np.max(np.abs(got - o.decrypt(out_m.S_proj[b]))) < 1e-6
    num, den, bb, err, se = G.finalize(o, lay, out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    assert np.max(np.abs(bb - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok]) < 1e-4
