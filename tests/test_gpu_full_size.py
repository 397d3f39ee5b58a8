"""GPU parity at full workload sizes: every ciphertext of the encrypted GWAS circuit, bit for bit.

The CPU oracle's ciphertexts for these workloads take minutes to compute, so a committed script
(``tests/golden/make_circuit_digests.py``, which calls only ``oracle/`` and ``synth/``) stored their
SHA-256 digests in ``tests/golden/circuit_digests.json``.  This test rebuilds the same plaintexts with
the oracle's encoder, encrypts them with the library under the same keys and seeds, runs the circuit in
the launch configuration the benchmark times (``gwas_semiparallel``: the logistic-regression part on a
second stream, all SNP batches of a job in one chunk of launches) and compares the digest of every
exported ciphertext (canonical form) with the oracle's:

* ``gwas_n245_k4_m10643``: the paper's dataset shape, 42 SNP batches of 256 SNPs (the last holds 147)
  at N = 2^16, L = 26, scale 2^40, kappa = 3: beta_j, w, w^-1, z', u and S', num, denEven, denOdd of
  every batch.
* ``gwas_n1100_k4_m100``: R = 2048 (three per-batch and four fixed-part rotation groups), 4 batches.
"""
import hashlib
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "circuit_digests.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _script():
    spec = importlib.util.spec_from_file_location(
        "make_circuit_digests", os.path.join(ROOT, "tests", "golden", "make_circuit_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _cases():
    if not os.path.exists(GOLDEN):
        return []
    with open(GOLDEN) as f:
        data = json.load(f)
    return sorted(k for k in data if not k.startswith("_"))


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).astype("<u8", copy=False).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    return torch


@pytest.mark.parametrize("name", _cases())
def test_full_size_circuit_bit_exact_against_oracle_digests(torch_dev, name):
    mk = _script()
    with open(GOLDEN) as f:
        rec = json.load(f)[name]
    case = mk.CASES[name]
    for key in ("n", "k", "m", "kappa", "log_n", "log2_scale", "data_seed", "key_seed", "enc_seed"):
        assert rec[key] == case[key], key
    say("[gpu] full size %s: plaintexts" % name)
    p, lay, d, pts = mk.case_inputs(case)
    got = [mk.poly_digest(m) for m in pts.polys]
    bad = [i for i, (a, b) in enumerate(zip(got, rec["plaintexts"])) if a != b]
    assert not bad, "the oracle's encoder gives other plaintexts on this host (indices %s)" % bad[:8]
    n, k, m, kappa = case["n"], case["k"], case["m"], case["kappa"]
    ctx = P.Context(case["log_n"], p.L, case["log2_scale"])
    assert ctx.moduli() == rec["moduli"]
    say("[gpu] %s: keygen (%d Galois keys)" % (name, len(rec["galois"])))
    ctx.keygen(case["key_seed"], rec["galois"])
    # inputs, encrypted by the library in the oracle's order and with its seeds
    scales = [p.scales[dd] for dd in pts.depths]
    for i in range(k + 1, k + 1 + len(G.a_pairs(k))):
        scales[i] = G.a_scale(p, lay)
    cts = [ctx.encrypt(pt, dd, s, G.input_seed(case["enc_seed"], i))
           for i, (pt, dd, s) in enumerate(zip(pts.polys, pts.depths, scales))]
    x, y, A, S = cts[:k], cts[k], cts[k + 1:k + 1 + len(G.a_pairs(k))], cts[k + 1 + len(G.a_pairs(k)):]
    ins = rec["inputs"]
    assert [digest(ctx.export(c)) for c in x] == ins["x"]
    assert digest(ctx.export(y)) == ins["y"]
    assert [digest(ctx.export(c)) for c in A] == ins["A"]
    assert [digest(ctx.export(c)) for c in S] == ins["S"]
    say("[gpu] %s: circuit (%d SNP batches)" % (name, lay.n_batches))
    gin = ctx.gwas_input_from_cts(n, k, m, kappa, x, y, A, S)
    outs = rec["outputs"]
    nb = lay.n_batches
    # the launch configuration the benchmark times, then the covariates' products stacked into one batch
    for stack in (0, 256):
        ctx.set_stack(stack)
        out = ctx.gwas_semiparallel(gin)
        assert [digest(ctx.export(out.ct(P.GwasOutput.BETA, j))) for j in range(k)] == outs["beta"]
        for which, key in ((P.GwasOutput.W, "w"), (P.GwasOutput.W_INV, "w_inv"), (P.GwasOutput.Z_PROJ, "z_proj"),
                           (P.GwasOutput.U, "u")):
            assert digest(ctx.export(out.ct(which))) == outs[key], key
        assert out.ct(P.GwasOutput.NUM, 0).count == nb   # every SNP batch in one chunk of launches
        for which, key in ((P.GwasOutput.S_PROJ, "S_proj"), (P.GwasOutput.NUM, "num"),
                           (P.GwasOutput.DEN_EVEN, "den_even"), (P.GwasOutput.DEN_ODD, "den_odd")):
            ct = out.ct(which, 0)
            got = [digest(ctx.export(ct, b)) for b in range(nb)]
            bad = [b for b in range(nb) if got[b] != outs[key][b]]
            assert not bad, (key, stack, bad)
        say("[gpu] %s: stack %d, %d output ciphertexts bit-exact" % (name, stack, k + 4 + 4 * nb))
    ctx.set_stack(0)
    ctx.close()
