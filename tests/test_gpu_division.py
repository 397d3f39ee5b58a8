"""GPU parity of the homomorphic division (b' and err' as ciphertexts; an extension of Alg. Semi Parallel
GWAS, which decrypts num and den separately and divides on the client).

* Bit for bit against the oracle (``oracle.gwas_circuit.divide_all``) for kappa = 1 (public weights) and
  kappa = 2, with the SNP batches in one chunk and in chunks of 2 (a ragged last chunk).
* At the paper's dataset shape (245 x 4 x 10643, N = 2^16, kappa = 1, the SEAL run's kappa): the
  decrypted b' and err' against the FP64 division of the same steps and against the FP64 GWAS.
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


@pytest.mark.parametrize("kappa,chunk", [(1, None), (1, 2), (2, 2)])
def test_division_bit_exact_against_oracle(torch_dev, kappa, chunk):
    n, k, m, log_n, b = 30, 4, 150, 10, 40
    say("[gpu] division kappa=%d chunk=%s" % (kappa, chunk))
    p = C.make_params(log_n, G.circuit_depth(kappa) + G.DIV_LEVELS, b)
    assert P.gwas_div_levels() == G.DIV_LEVELS
    d = make_gwas_data(n, k, m, seed=91)
    lay = G.make_layout(p.N, n, k, m)
    assert lay.n_batches == 5
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    ref = G.Circuit(o, lay).run(inp)
    v = G.encrypt_normalisers(o, G.encode_normalisers(p, d.S, lay, kappa), kappa, 11)
    dv = G.divide_all(o, ref, v)
    ctx = P.Context(log_n, p.L, b)
    ctx.keygen(7, G.required_galois(p.N, lay.R))
    imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
    gin = ctx.gwas_input_from_cts(n, k, m, kappa, [imp(c) for c in inp.x], imp(inp.y),
                                  [imp(inp.A[pr]) for pr in G.a_pairs(k)], [imp(c) for c in inp.S])
    out = ctx.gwas_semiparallel(gin, chunk)
    V = ctx.stack([imp(c) for c in v])
    ctx.gwas_divide(out, V)
    ch = chunk or lay.n_batches
    for bi in range(lay.n_batches):
        cnt = min(ch, lay.n_batches - (bi // ch) * ch)
        i = bi % ch
        for which, even, odd in ((P.GwasOutput.DIV_B, dv.b_even, dv.b_odd),
                                 (P.GwasOutput.DIV_ERR, dv.inv_even, dv.inv_odd)):
            g = out.ct(which, bi // ch)
            assert g.count == 2 * cnt
            assert np.array_equal(ctx.export(g, i), even[bi].data), (which, bi, "even")
            assert np.array_equal(ctx.export(g, cnt + i), odd[bi].data), (which, bi, "odd")
    res = ctx.gwas_finalize_divided(out)
    bb, err, se = G.finalize_divided(o, lay, dv)
    assert np.allclose(res["b"], bb, rtol=1e-9, atol=1e-9)
    assert np.allclose(res["err"], err, rtol=1e-9, atol=1e-12)
    # the library's own normalisers (its encoder, within one unit of the oracle's) decrypt to the same values
    Vl = ctx.gwas_pack_normalisers(d.S, kappa, 11)
    assert Vl.info()[:3] == (2 * lay.n_batches, G.circuit_depth(kappa), p.L + 1 - G.circuit_depth(kappa))
    for i in (0, lay.n_batches, 2 * lay.n_batches - 1):
        assert np.allclose(ctx.decrypt(Vl, i), o.decrypt(v[i]), atol=1e-6)
    ctx.close()


def test_division_at_dataset_shape_kappa1(torch_dev):
    n, k, m, kappa, log_n, b = 245, 4, 10643, 1, 16, 40
    say("[gpu] division at n=%d m=%d kappa=%d" % (n, m, kappa))
    L = G.circuit_depth(kappa) + P.gwas_div_levels()
    ctx = P.Context(log_n, L, b)
    lay = ctx.gwas_layout(n, k, m, kappa)
    ctx.keygen(7, G.required_galois(1 << log_n, lay["R"]))
    d = make_gwas_data(n, k, m, seed=config_seed(2))
    out = ctx.gwas_semiparallel(ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11))
    ctx.gwas_divide(out, ctx.gwas_pack_normalisers(d.S, kappa, 11))
    res = ctx.gwas_finalize_divided(out)
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    bd, invd = F.divide_plain(ref.num, ref.den, F.snp_normalisers(d.S))
    e_div = np.max(np.abs(res["b"] - bd)[ok] / np.maximum(np.abs(bd), np.sqrt(invd))[ok])
    e_ref = np.max(np.abs(res["b"] - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok])
    say("[gpu] division: max error %.3g against the FP64 division, %.3g against the FP64 GWAS" % (e_div, e_ref))
    assert e_div < 1e-4 and e_ref < 1e-3
    assert np.allclose(res["err"][ok], ref.err[ok], rtol=1e-3)
    ctx.close()
