"""GPU parity of the M-materialised layout (Alg. CP-REP-MatMult: M = I - X A X^T as n duplicated columns,
S' = sum_i Dup(M_i) (.) S_rep(i) with the SNP batches in REP form), bit for bit against the oracle's
``Circuit(o, lay, m_in)``: the columns of M, S', the numerator and both denominators of every batch, and
the fixed part's outputs; plus the library's own REP packing against the factorised layout's results.
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


@pytest.mark.parametrize("n,m,log_n,b,kappa,chunk", [(30, 70, 10, 30, 3, 2), (30, 150, 10, 30, 1, None),
                                                     (245, 32, 13, 30, 1, None)])
def test_m_layout_bit_exact_against_oracle(torch_dev, n, m, log_n, b, kappa, chunk):
    k = 4
    say("[gpu] M layout n=%d m=%d logN=%d kappa=%d" % (n, m, log_n, kappa))
    p = C.make_params(log_n, G.circuit_depth(kappa), b)
    d = make_gwas_data(n, k, m, seed=config_seed(1) if n == 245 else 93)
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    mi = G.encrypt_inputs_m(o, G.encode_inputs_m(p, d.X, d.S, kappa), n, k, 11)
    ref = G.Circuit(o, lay, mi).run(inp)
    ctx = P.Context(log_n, p.L, b)
    ctx.keygen(7, G.required_galois(p.N, lay.R))
    imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
    gin = ctx.gwas_input_from_cts(n, k, m, kappa, [imp(c) for c in inp.x], imp(inp.y),
                                  [imp(inp.A[pr]) for pr in G.a_pairs(k)], [imp(c) for c in inp.S])
    ctx.gwas_input_attach_m(gin, [imp(c) for row in mi.Xrep for c in row], [imp(c) for bt in mi.S_rep for c in bt])
    out = ctx.gwas_semiparallel(gin, chunk)
    cols = out.ct(P.GwasOutput.M_COLS)
    assert cols.count == n
    for i in range(n):
        assert np.array_equal(ctx.export(cols, i), ref.m_cols[i].data), ("M column", i)
    for j in range(k):
        assert np.array_equal(ctx.export(out.ct(P.GwasOutput.BETA, j)), ref.beta[j].data)
    assert np.array_equal(ctx.export(out.ct(P.GwasOutput.Z_PROJ)), ref.z_proj.data)
    ch = chunk or lay.n_batches
    for bi in range(lay.n_batches):
        for which, r in [(P.GwasOutput.S_PROJ, ref.S_proj), (P.GwasOutput.NUM, ref.num),
                         (P.GwasOutput.DEN_EVEN, ref.den_even), (P.GwasOutput.DEN_ODD, ref.den_odd)]:
            assert np.array_equal(ctx.export(out.ct(which, bi // ch), bi % ch), r[bi].data), (which, bi)
    ctx.close()


def test_m_layout_library_packing_matches_factorised(torch_dev):
    """The library's own client packing of the REP inputs: b' of the M-materialised layout equals that of
    the factorised layout to CKKS precision, and both match the FP64 GWAS (n = 245, N = 2^13, kappa = 1)."""
    n, k, m, kappa, log_n, b = 245, 4, 64, 1, 13, 30
    say("[gpu] M layout vs factorised, library packing")
    ctx = P.Context(log_n, G.circuit_depth(kappa), b)
    lay = ctx.gwas_layout(n, k, m, kappa)
    ctx.keygen(7, G.required_galois(1 << log_n, lay["R"]))
    d = make_gwas_data(n, k, m, seed=config_seed(1, 3))
    g0 = ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11)
    r0 = ctx.gwas_finalize(ctx.gwas_semiparallel(g0))
    g1 = ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11)
    ctx.gwas_pack_encrypt_m(g1, d.X, d.S, 11)
    r1 = ctx.gwas_finalize(ctx.gwas_semiparallel(g1))
    ref = F.modified_gwas(d.X, d.y, d.S, kappa)
    ok = ref.den > 1e-9 * np.max(ref.den)
    tol = np.maximum(np.abs(ref.b), ref.se)[ok]
    assert np.max(np.abs(r1["b"] - r0["b"])[ok] / tol) < 1e-3
    assert np.max(np.abs(r1["b"] - ref.b)[ok] / tol) < 1e-3
    ctx.close()
