"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Ciphertexts, keys and every intermediate are compared bit for bit in the
canonical form (coefficient domain, residues in [0, q)); decrypted GWAS results
are compared with the FP64 plaintext GWAS.  Inputs of the circuit test are the
oracle's own ciphertexts, imported into the library, so that no oracle input or
expected value comes from the HIP path.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from oracle import ckks as C  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402
from oracle import gwas_fp64 as F  # noqa: E402
from synth import config_seed, make_gwas_data  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    return torch


def make_pair(log_n, levels, b, galois_fn, seed=7, alpha=None):
    """Library context and oracle with the same parameters (alpha None: each side's default)."""
    ctx = P.Context(log_n, levels, b) if alpha is None else P.Context(log_n, levels, b, alpha=alpha)
    p = C.make_params(log_n, levels, b) if alpha is None else C.make_params(log_n, levels, b, alpha)
    assert ctx.alpha == p.alpha
    o = C.Oracle(p)
    g = galois_fn(p.N)
    ctx.keygen(seed, g)
    o.keygen(seed, g)
    return ctx, o, p


@pytest.fixture(scope="module", params=[None, 2, 4])
def small(torch_dev, request):
    """N = 2^10, L = 5 with the default digit-group size (3: {q_0 q_1} {q_2 q_3 q_4} {q_5}, a cut last
    group), alpha = 2 ({q_0} {q_1 q_2} {q_3 q_4} {q_5}) and alpha = 4 ({q_0 q_1 q_2} {q_3 q_4 q_5}); the
    tests' deeper ciphertexts cut the groups further."""
    say("[gpu] small ring N=2^10 L=5 alpha=%s" % request.param)
    return make_pair(10, 5, 30, lambda N: [C.galois_rotate(N, 1), C.galois_rotate(N, -2), C.galois_rotate(N, 4),
                                           C.galois_conj(N)], alpha=request.param)


def rand_ct(p, depth, rng):
    l = p.limbs_at_depth(depth)
    return np.stack([np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in p.q[:l]]) for _ in range(2)])


@pytest.mark.parametrize("log_n", [10, 11, 12, 13, 16, 17])
def test_ntt_negacyclic_products_match_oracle(torch_dev, log_n):
    """Forward NTT, pointwise product, inverse NTT on the GPU equals the oracle's negacyclic product,
    for every modulus kind (q_0 of 60 bits, rescale primes of 40 bits, P of 62 bits), every sub-transform
    size the two-pass NTT uses, random residues and the all-(q - 1) worst case; inverse(forward(a)) == a."""
    say("[gpu] ntt log_n=%d" % log_n)
    ctx = P.Context(log_n, 3, 40)
    p = C.make_params(log_n, 3, 40)
    o = C.Oracle(p)
    N = p.N
    rng = np.random.default_rng(log_n)
    dev = torch_dev.device("cuda:0")

    def run(x, mi, direction):
        t = torch_dev.from_numpy(x.view(np.int64).copy()).to(dev)
        ctx.ntt_device(t.data_ptr(), x.shape[0], [mi] * x.shape[0], direction)
        torch_dev.cuda.synchronize()
        return t.cpu().numpy().view(np.uint64)

    for mi, q in enumerate(o.mods):
        for case in ("random", "max"):
            if case == "random":
                a = rng.integers(0, q, size=N, dtype=np.uint64)
                b = rng.integers(0, q, size=N, dtype=np.uint64)
            else:
                a = np.full(N, q - 1, dtype=np.uint64)
                b = np.full(N, q - 1, dtype=np.uint64)
            ev = run(np.stack([a, b]), mi, 1)
            assert int(ev.max()) < q
            assert np.array_equal(run(ev.copy(), mi, -1), np.stack([a, b])), (mi, case)
            prod = ((ev[0].astype(object) * ev[1].astype(object)) % q).astype(np.uint64)
            got = run(prod[None, :].copy(), mi, -1)[0]
            want = np.zeros(N, dtype=np.uint64)
            C.lib().ref_polymul(o._ctx, mi, C._p(a), C._p(b), C._p(want))
            assert np.array_equal(got, want), (mi, case)
    ctx.close()


def test_keys_match_oracle(small):
    ctx, o, p = small
    assert np.array_equal(ctx.export_secret(), o.sk)
    assert np.array_equal(ctx.export_public_key(), o.pk)
    for K in list(o.keys):
        assert np.array_equal(ctx.export_switching_key(K), o.keys[K]), K


def test_encrypt_matches_oracle(small):
    ctx, o, p = small
    rng = np.random.default_rng(1)
    z = rng.standard_normal(p.slots) + 1j * rng.standard_normal(p.slots)
    m = C.encode(z, p.N, p.scales[0])
    for depth in (0, 2):
        ct = ctx.encrypt(m, depth, p.scales[depth], 99 + depth)
        ref = o.encrypt(m, depth, p.scales[depth], 99 + depth)
        assert np.array_equal(ctx.export(ct), ref.data)
    # decrypt of the library's own ciphertext
    ct = ctx.encrypt(m, 0, p.scales[0], 5)
    assert np.max(np.abs(ctx.decrypt(ct) - z)) < 1e-4


def test_encode_matches_oracle_within_one(small):
    ctx, o, p = small
    rng = np.random.default_rng(2)
    z = rng.standard_normal(p.slots) + 1j * rng.standard_normal(p.slots)
    assert np.max(np.abs(ctx.encode(z, p.scales[0]) - C.encode(z, p.N, p.scales[0]))) <= 1


def test_import_export_roundtrip(small):
    ctx, o, p = small
    rng = np.random.default_rng(3)
    for depth in (0, 3, p.L):
        data = rand_ct(p, depth, rng)
        ct = ctx.import_ct(data, depth, p.scales[depth])
        assert np.array_equal(ctx.export(ct), data)


def _both(ctx, o, p, data, depth, scale=None):
    scale = p.scales[depth] if scale is None else scale
    return ctx.import_ct(data, depth, scale), C.Ct(data.copy(), depth, scale)


def test_elementwise_and_rescale_match_oracle(small):
    ctx, o, p = small
    rng = np.random.default_rng(4)
    ga, oa = _both(ctx, o, p, rand_ct(p, 1, rng), 1)
    gb, ob = _both(ctx, o, p, rand_ct(p, 1, rng), 1)
    cases = [
        ("add", ctx.add(ga, gb), o.add(oa, ob)),
        ("sub", ctx.sub(ga, gb), o.sub(oa, ob)),
        ("mul_int", ctx.mul_int(ga, -123456789), o.mul_int(oa, -123456789)),
        ("add_const", ctx.add_const(ga, -0.7351), o.add_const(oa, -0.7351)),
        ("rescale", ctx.rescale(ga), o.rescale(oa)),
        ("mul_const", ctx.mul_const(ga, 0.3141), o.mul_const(oa, 0.3141)),
        ("align", ctx.align(ga, 3, p.scales[3], 0.125), o.align(oa, 3, p.scales[3], 0.125)),
        ("mask", ctx.mul_mask(ga, 8), o.mul_mask(oa, 8)),
    ]
    for name, g, r in cases:
        say("[gpu] op", name)
        assert g.depth == r.depth and g.scale == r.scale, name
        assert np.array_equal(ctx.export(g), r.data), name


def test_mul_relinearise_and_galois_match_oracle(small):
    ctx, o, p = small
    rng = np.random.default_rng(5)
    for depth in (0, 2, p.L - 1):
        ga, oa = _both(ctx, o, p, rand_ct(p, depth, rng), depth)
        gb, ob = _both(ctx, o, p, rand_ct(p, depth, rng), depth)
        say("[gpu] mul at depth", depth)
        assert np.array_equal(ctx.export(ctx.mul(ga, gb)), o.mul(oa, ob).data)
        for r in (1, -2, 4):
            say("[gpu] rotate", r, "at depth", depth)
            assert np.array_equal(ctx.export(ctx.rotate(ga, r)), o.rotate(oa, r).data)
        assert np.array_equal(ctx.export(ctx.conjugate(ga)), o.conjugate(oa).data)
        for rots in ([1, -2, 4], [4], [-2, 1]):
            say("[gpu] rotate_sum", rots, "at depth", depth)
            assert np.array_equal(ctx.export(ctx.rotate_sum(ga, rots)), o.rotate_sum(oa, rots).data)


@pytest.fixture(scope="module")
def wide(torch_dev):
    """N = 2^10, L = 5 with the keys of the rotations +-1..+-15 and 16, 32, 48: rotate-and-sums of up to 16
    rotations sharing one key switch."""
    say("[gpu] small ring N=2^10 L=5, keys of 33 rotations")
    rots = list(range(1, 16)) + [-r for r in range(1, 16)] + [16, 32, 48]
    return make_pair(10, 5, 30, lambda N: [C.galois_rotate(N, r) for r in rots])


@pytest.mark.parametrize("rots", [list(range(1, 16)), [-r for r in range(1, 16)], list(range(1, 8)), [1, 2, 3, 4],
                                  [2, -5], list(range(1, 16)) + [16], [16, 32, 48, -7, 9], [2, 4, -6], [4, 8, 12],
                                  [16, 32, 48]])
def test_wide_rotate_sum_matches_oracle(wide, rots):
    """One key switch shared by 2 to 16 rotations (the inner product's key chunks of 3, the last one
    padded, and the loop over 2 keys; the automorphism sum of more than 3 rotations; rotation lines with shift
    units 1, 2, 4 and, at N = 2^10 where 16 slots is a multiple of N / 128, lines of one group) equals the
    oracle's, at every depth."""
    ctx, o, p = wide
    rng = np.random.default_rng(len(rots))
    for depth in (0, 2, p.L - 1):
        ga, oa = _both(ctx, o, p, rand_ct(p, depth, rng), depth)
        say("[gpu] rotate_sum of", len(rots), "rotations at depth", depth)
        assert np.array_equal(ctx.export(ctx.rotate_sum(ga, rots)), o.rotate_sum(oa, rots).data)


@pytest.fixture(scope="module")
def full_ring(torch_dev):
    """The workload's ring and chain (N = 2^16, L = 26, 40-bit scale primes, digit groups of 3) with the
    keys of the per-batch rotate-and-sums (rotations 1..15 and 16..240 step 16) and conjugation.  The
    library holds full keys; one oracle holds the same keys restricted to ciphertexts of at most 6 limbs
    (the per-batch levels), a second one full-height keys for relinearisation, rotation by 1 and 16."""
    say("[gpu] full ring N=2^16 L=26: library keys")
    rots = list(range(1, 16)) + [16 * i for i in range(1, 16)]
    ctx = P.Context(16, 26, 40)
    p = C.make_params(16, 26, 40)
    assert ctx.moduli() == [int(q) for q in p.q] + [int(q) for q in p.P]
    g = [C.galois_rotate(p.N, r) for r in rots] + [C.galois_conj(p.N)]
    ctx.keygen(7, g)
    say("[gpu] full ring: oracle keys (6 limbs, then full height)")
    low = C.Oracle(p)
    low.keygen(7, g, max_limbs=p.limbs_at_depth(21))
    top = C.Oracle(p)
    top.keygen(7, [C.galois_rotate(p.N, 1), C.galois_rotate(p.N, 16)])
    return ctx, low, top, p


@pytest.mark.parametrize("depth", [21, 24])
def test_full_ring_batch_level_ops_match_oracle(full_ring, depth):
    """At the workload's own ring and levels, the key switches of the per-batch part (relinearisation, the
    15-rotation rotate-and-sums on the lines of shift 1 and 16, a single rotation, conjugation) equal the
    oracle's bit for bit."""
    ctx, o, _, p = full_ring
    rng = np.random.default_rng(100 + depth)
    ga, oa = _both(ctx, o, p, rand_ct(p, depth, rng), depth)
    gb, ob = _both(ctx, o, p, rand_ct(p, depth, rng), depth)
    say("[gpu] full ring mul at depth", depth)
    assert np.array_equal(ctx.export(ctx.mul(ga, gb)), o.mul(oa, ob).data)
    for rots in (list(range(1, 16)), [16 * i for i in range(1, 16)], [1, 2, 3], [16]):
        say("[gpu] full ring rotate_sum of", len(rots), "rotations from", rots[0], "at depth", depth)
        assert np.array_equal(ctx.export(ctx.rotate_sum(ga, rots)), o.rotate_sum(oa, rots).data)
    say("[gpu] full ring rotate and conjugate at depth", depth)
    assert np.array_equal(ctx.export(ctx.rotate(ga, 7)), o.rotate(oa, 7).data)
    assert np.array_equal(ctx.export(ctx.conjugate(ga)), o.conjugate(oa).data)


def test_full_ring_top_level_ops_match_oracle(full_ring):
    """At 27 limbs (all nine digit groups, the fixed part's first key switches) relinearisation and
    rotations equal the oracle's bit for bit."""
    ctx, _, o, p = full_ring
    rng = np.random.default_rng(99)
    ga, oa = _both(ctx, o, p, rand_ct(p, 0, rng), 0)
    gb, ob = _both(ctx, o, p, rand_ct(p, 0, rng), 0)
    say("[gpu] full ring mul at depth 0")
    assert np.array_equal(ctx.export(ctx.mul(ga, gb)), o.mul(oa, ob).data)
    say("[gpu] full ring rotate 1, rotate_sum [1, 16] at depth 0")
    assert np.array_equal(ctx.export(ctx.rotate(ga, 1)), o.rotate(oa, 1).data)
    assert np.array_equal(ctx.export(ctx.rotate_sum(ga, [1, 16])), o.rotate_sum(oa, [1, 16]).data)


def test_kernel_timing_report(small):
    """Per-kernel timing: every launched kernel appears with its launches and a positive time, a timing
    restricted to one kernel records that kernel only, and timing leaves the results unchanged."""
    ctx, o, p = small
    rng = np.random.default_rng(8)
    ga, _ = _both(ctx, o, p, rand_ct(p, 1, rng), 1)
    want = ctx.export(ctx.rotate_sum(ga, [1, -2, 4]))
    ctx.kernel_timing(True)
    got = ctx.export(ctx.rotate_sum(ga, [1, -2, 4]))
    ctx.kernel_timing(False)
    rep = ctx.kernel_report()
    assert np.array_equal(got, want)
    assert any(k.startswith("ks_inner<") for k in rep) and any(k.startswith("ntt_pass<") for k in rep)
    for name, (cnt, ms, by, fl, pb) in rep.items():
        assert cnt >= 1 and ms > 0 and by > 0 and fl >= 0 and pb >= by, name
    # a two-pass NTT moves more than the transform's own bytes (its intermediate round trip)
    assert any(v[4] > v[2] for k, v in rep.items() if k.startswith("ntt_pass<"))
    # the inner product declares its FP64 operations: 18 per multiply-accumulate
    assert all(rep[k][3] > 0 for k in rep if k.startswith("ks_inner<"))
    name = next(k for k in rep if k.startswith("ks_inner<"))
    ctx.kernel_timing_only(name)
    ctx.kernel_timing(True)
    got = ctx.export(ctx.rotate_sum(ga, [1, -2, 4]))
    ctx.kernel_timing(False)
    ctx.kernel_timing_only(None)
    only = {k: v for k, v in ctx.kernel_report().items() if v[0]}
    assert list(only) == [name] and np.array_equal(got, want)
    # whole key switches as regions: one per rotate-and-sum, with the key switch's algorithmic bytes
    ctx.kernel_timing_only("keyswitch")
    ctx.kernel_timing(True)
    got = ctx.export(ctx.rotate_sum(ga, [1, -2, 4]))
    ctx.kernel_timing(False)
    ctx.kernel_timing_only(None)
    ks = {k: v for k, v in ctx.kernel_report().items() if v[0]}
    l, a, N = ga.limbs, ctx.alpha, p.N
    assert list(ks) == ["keyswitch"] and ks["keyswitch"][0] == 1 and ks["keyswitch"][1] > 0
    assert ks["keyswitch"][2] == 8.0 * N * (l + 3 * 2 * (1 + l // a) * (l + a) + 4 * l)
    assert np.array_equal(got, want)


def test_missing_key_and_level_errors(small):
    ctx, o, p = small
    rng = np.random.default_rng(6)
    ga = ctx.import_ct(rand_ct(p, p.L, rng), p.L, p.scales[p.L])
    with pytest.raises(P.CkksError) as e:
        ctx.rotate(ga, 3)
    assert e.value.code == -4
    with pytest.raises(P.CkksError) as e:
        ctx.rescale(ga)
    assert e.value.code == -3


def test_decrypted_semantics(small):
    ctx, o, p = small
    rng = np.random.default_rng(7)
    z = rng.standard_normal(p.slots) + 1j * rng.standard_normal(p.slots)
    w = rng.standard_normal(p.slots)
    a = ctx.encrypt(ctx.encode(z, p.scales[0]), 0, p.scales[0], 1)
    b = ctx.encrypt(ctx.encode(w, p.scales[0]), 0, p.scales[0], 2)
    assert np.max(np.abs(ctx.decrypt(ctx.mul(a, b)) - z * w)) < 1e-3
    assert np.max(np.abs(ctx.decrypt(ctx.rotate(a, 1)) - np.roll(z, -1))) < 1e-4
    assert np.max(np.abs(ctx.decrypt(ctx.rotate(a, -2)) - np.roll(z, 2))) < 1e-4
    assert np.max(np.abs(ctx.decrypt(ctx.conjugate(a)) - np.conj(z))) < 1e-4


# ------------------------------------------------------------------ the whole circuit

def _oracle_circuit(n, k, m, kappa, log_n, b, data_seed):
    p = C.make_params(log_n, G.circuit_depth(kappa), b)
    d = make_gwas_data(n, k, m, seed=data_seed)
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    pts = G.encode_inputs(p, d.X, d.y, d.S, kappa)
    inp = G.encrypt_inputs(o, pts, n, k, m, kappa, 11)
    ks0 = o.n_keyswitch
    out = G.Circuit(o, lay).run(inp)
    o.n_keyswitch_circuit = o.n_keyswitch - ks0
    return p, d, lay, o, inp, out


@pytest.mark.parametrize("n,k,m,log_n,b,chunk,kappa", [(30, 4, 70, 10, 30, 2, 3), (30, 4, 150, 10, 30, None, 3),
                                                         (245, 4, 32, 13, 30, None, 3), (30, 4, 70, 10, 30, 2, 2),
                                                         (30, 4, 150, 10, 30, None, 1), (245, 4, 32, 13, 30, 1, 1),
                                                         (24, 4, 70, 10, 30, 2, 3), (24, 3, 70, 10, 30, None, 2),
                                                         (20, 2, 40, 10, 30, None, 1), (24, 6, 40, 10, 30, None, 2)])
def test_circuit_bit_exact_against_oracle(torch_dev, n, k, m, log_n, b, chunk, kappa):
    """Every output ciphertext of the circuit bit for bit against the oracle, for kappa = 3, 2 and 1 (the
    reduced kappa of the paper's Discussion, with public weights).  n = 30 at R = 32 takes one colSum and
    broadcast per covariate; n = 245 at R = 256 and n <= 24 at R = 32 take the packed projection (K = 4,
    K = 2 for k = 2, K = 8 for k = 6)."""
    say("[gpu] circuit n=%d k=%d m=%d logN=%d kappa=%d" % (n, k, m, log_n, kappa))
    p, d, lay, o, inp, ref = _oracle_circuit(n, k, m, kappa, log_n, b, config_seed(1))
    ctx = P.Context(log_n, p.L, b)
    ctx.keygen(7, G.required_galois(p.N, lay.R))
    imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
    x = [imp(c) for c in inp.x]
    A = [imp(inp.A[pr]) for pr in G.a_pairs(k)]
    S = [imp(c) for c in inp.S]
    gin = ctx.gwas_input_from_cts(n, k, m, kappa, x, imp(inp.y), A, S)
    ks0 = ctx.counters()["keyswitch_ciphertexts"]
    out = ctx.gwas_semiparallel(gin, chunk)
    # the same work as the oracle's ciphertext-at-a-time circuit: one key switch per ciphertext and step
    assert ctx.counters()["keyswitch_ciphertexts"] - ks0 == o.n_keyswitch_circuit
    for j in range(k):
        assert np.array_equal(ctx.export(out.ct(P.GwasOutput.BETA, j)), ref.beta[j].data)
    for which, r in [(P.GwasOutput.W, ref.w), (P.GwasOutput.W_INV, ref.w_inv), (P.GwasOutput.Z_PROJ, ref.z_proj),
                     (P.GwasOutput.U, ref.u)]:
        if r is None:   # kappa = 1: w and w^-1 are public constants
            with pytest.raises(P.CkksError):
                out.ct(which)
            continue
        assert np.array_equal(ctx.export(out.ct(which)), r.data), which
    ch = chunk or lay.n_batches
    for bi in range(lay.n_batches):
        for which, r in [(P.GwasOutput.NUM, ref.num), (P.GwasOutput.DEN_EVEN, ref.den_even),
                         (P.GwasOutput.DEN_ODD, ref.den_odd), (P.GwasOutput.S_PROJ, ref.S_proj)]:
            g = out.ct(which, bi // ch)
            assert np.array_equal(ctx.export(g, bi % ch), r[bi].data), (which, bi)
    # the client finalisation decodes num and den as the oracle's does, to FP64 rounding of the two
    # decoders; b = num / den is compared where den is not tiny against its largest value (a SNP column
    # nearly constant over the few samples amplifies the decoders' rounding differences)
    res = ctx.gwas_finalize(out)
    num, den, bb, err, se = G.finalize(o, lay, ref)
    for got, want in ((res["num"], num), (res["den"], den)):
        assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.max(np.abs(want)))
    ok = np.abs(den) > 1e-3 * np.max(np.abs(den))
    assert np.allclose(res["b"][ok], bb[ok], rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("n,k,m,log_n,b,tol,kappa", [(245, 4, 32, 13, 30, 1e-3, 3), (245, 4, 600, 16, 40, 1e-3, 3),
                                                       (245, 4, 10643, 16, 40, 1e-3, 3),
                                                       (245, 4, 10643, 16, 40, 1e-3, 1)])
def test_end_to_end_accuracy_against_fp64(torch_dev, n, k, m, log_n, b, tol, kappa):
    """Decrypted b' within tol of the FP64 modified GWAS (relative to max(|b'|, se)) and se within 1e-3,
    up to the benchmark's full workload (42 SNP batches of 256, the batched launches it times)."""
    say("[gpu] end-to-end n=%d m=%d logN=%d kappa=%d" % (n, m, log_n, kappa))
    L = G.circuit_depth(kappa)
    ctx = P.Context(log_n, L, b)
    lay = ctx.gwas_layout(n, k, m, kappa)
    N = 1 << log_n
    ctx.keygen(7, G.required_galois(N, lay["R"]))
    d = make_gwas_data(n, k, m, seed=config_seed(2 if log_n == 16 else 1))
    gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11)
    out = ctx.gwas_semiparallel(gin)
    res = ctx.gwas_finalize(out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    rel = np.abs(res["b"] - ref.b) / np.maximum(np.abs(ref.b), ref.se)
    say("[gpu] max G26 error", float(np.max(rel[ok])))
    assert np.max(rel[ok]) < tol
    assert np.allclose(res["se"][ok], ref.se[ok], rtol=1e-3)


def test_planted_effects_relative_accuracy(torch_dev):
    """Planted SNP effects (1 % of the SNPs with logit effect 0.5) at the paper's dataset shape: on every
    SNP with |b'| > se the decrypted b' is within 1e-3 relative error of the FP64 modified GWAS (the
    relative bound exercised on large effects, not only on null SNPs), and the planted SNPs stand out."""
    n, k, m, kappa, log_n, b = 245, 4, 10643, 3, 16, 40
    say("[gpu] planted effects n=%d m=%d" % (n, m))
    ctx = P.Context(log_n, G.circuit_depth(kappa), b)
    lay = ctx.gwas_layout(n, k, m, kappa)
    ctx.keygen(7, G.required_galois(1 << log_n, lay["R"]))
    d = make_gwas_data(n, k, m, seed=config_seed(2, 7), planted_frac=0.01, planted_effect=0.5)
    out = ctx.gwas_semiparallel(ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11))
    res = ctx.gwas_finalize(out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    big = ok & (np.abs(ref.b) > ref.se)
    planted = ok & (d.planted != 0)
    rel = np.abs(res["b"] - ref.b) / np.abs(ref.b)
    say("[gpu] SNPs with |b'| > se: %d (planted %d); max relative error %.3g (planted %.3g)"
        % (big.sum(), (big & planted).sum(), np.max(rel[big]), np.max(rel[planted & big])))
    assert (big & planted).sum() >= 40 and big.sum() >= 1000
    assert np.max(rel[big]) < 1e-3
    # the planted effects are recovered: their mean estimate stands far above that of the null SNPs (the
    # 106 planted SNPs share the phenotype's variance, so each marginal estimate is about half the effect)
    assert np.mean(res["b"][planted]) > 0.15 > 10 * abs(np.mean(res["b"][ok & ~planted]))
    ctx.close()
