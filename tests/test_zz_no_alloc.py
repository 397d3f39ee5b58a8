"""GPU tests of ckks_mul_noalloc, the relinearised product that allocates no device memory.

Its output must be bit-identical to ckks_mul's on the same operands (the same kernels run on buffers
carved from the library's static scratch array).  Two calls in a row, the second with a smaller input
(fewer ciphertexts and fewer limbs), check that nothing depends on what the first call left in the
array; the pool's allocation count must not move during either call; a product whose buffers exceed the
array is refused before any work is enqueued.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from synth import make_gwas_data  # noqa: E402


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    return torch


def _same(ctx, got, ref):
    c_got, d_got, l_got, s_got = got.info()
    c_ref, d_ref, l_ref, s_ref = ref.info()
    assert (c_got, d_got, l_got, s_got) == (c_ref, d_ref, l_ref, s_ref)
    for i in range(c_ref):
        assert np.array_equal(ctx.export(got, i), ctx.export(ref, i)), ("ciphertext", i)


def test_mul_noalloc_matches_mul_on_two_calls(torch_dev):
    torch = torch_dev
    ctx = P.Context(13, 19, 30)   # N = 2^13, L = 19 (kappa = 2 circuit depth)
    ctx.keygen(7, [])
    N = 1 << 13
    # first call: a batch of 3 SNP ciphertexts (6 limbs) times x_0 brought to their depth
    d = make_gwas_data(30, 4, 700, seed=77)
    gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, 2, 11)
    S = gin.ct(P.GwasInput.S, 0)
    cS, dS, lS, sS = S.info()
    assert cS == 3 and lS == 6
    xa = ctx.align(gin.ct(P.GwasInput.X, 0), dS, sS)
    ref1 = ctx.mul(S, xa)
    out1 = ctx.mul_int(ctx.mul(S, xa), 0)       # the caller's output: 3 zero ciphertexts at dS + 1
    torch.cuda.synchronize()
    n_alloc0 = ctx.pool_stats()["n_alloc"]
    got1 = ctx.mul_noalloc(S, xa, out1)
    torch.cuda.synchronize()
    assert ctx.pool_stats()["n_alloc"] == n_alloc0
    _same(ctx, got1, ref1)
    # second call, smaller: one ciphertext at 4 limbs
    rng = np.random.default_rng(3)
    sc = ctx.scales()[16]
    a = ctx.encrypt(rng.integers(-2 ** 25, 2 ** 25, size=N, dtype=np.int64), 16, sc, 21)
    b = ctx.encrypt(rng.integers(-2 ** 25, 2 ** 25, size=N, dtype=np.int64), 16, sc, 22)
    ref2 = ctx.mul(a, b)
    out2 = ctx.import_ct(np.zeros((2, 3, N), dtype=np.uint64), 17, sc)
    torch.cuda.synchronize()
    n_alloc1 = ctx.pool_stats()["n_alloc"]
    got2 = ctx.mul_noalloc(a, b, out2)
    torch.cuda.synchronize()
    assert ctx.pool_stats()["n_alloc"] == n_alloc1
    _same(ctx, got2, ref2)
    # the first output is untouched by the second call
    _same(ctx, got1, ref1)
    ctx.close()


def test_mul_noalloc_rejects_products_beyond_the_scratch(torch_dev):
    ctx = P.Context(16, 26, 40)
    ctx.keygen(7, [])
    N = 1 << 16
    sc = ctx.scales()[0]
    rng = np.random.default_rng(4)
    a = ctx.encrypt(rng.integers(-2 ** 30, 2 ** 30, size=N, dtype=np.int64), 0, sc, 5)
    out = ctx.import_ct(np.zeros((2, 26, N), dtype=np.uint64), 1, sc)
    with pytest.raises(P.CkksError) as e:
        ctx.mul_noalloc(a, a, out)
    assert e.value.code == -1 and "maximum" in str(e.value)
    # a shape mismatch of the output is refused too
    out_bad = ctx.import_ct(np.zeros((2, 25, N), dtype=np.uint64), 2, sc)
    with pytest.raises(P.CkksError) as e:
        ctx.mul_noalloc(a, a, out_bad)
    assert e.value.code == -2
    ctx.close()
