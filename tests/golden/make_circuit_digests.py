"""Writes ``circuit_digests.json``: SHA-256 digests of every ciphertext of the oracle's encrypted GWAS
circuit at full workload sizes.  TEST INFRASTRUCTURE: this script calls only ``oracle/`` and the seeded
input generators in ``synth/``.

The GPU parity test ``tests/test_gpu_full_size.py`` encrypts the same plaintexts with the library under
the same keys and seeds, runs the circuit in the launch configuration the benchmark times, and compares
the digest of every exported ciphertext (canonical form: coefficient domain, residues in [0, q),
[2][limbs][N] little-endian uint64) with the oracle's.  The oracle run takes minutes (full-ring key
switches in plain C), so its results are stored as digests instead of being recomputed per test run.

Cases (Alg. Semi Parallel GWAS with kappa = 3 Newton passes, N = 2^16, L = 26, scale 2^40):

* ``gwas_n245_k4_m10643``: the paper's dataset shape (Results: 245 samples, 4 covariates, 10643 SNPs):
  R = 256, 42 SNP batches of 256 SNPs, the last holding 147.
* ``gwas_n1100_k4_m100``: one job of the batched workload's size range with R = 2048 (32 SNPs per
  ciphertext, 4 batches, the last holding 4 SNPs), whose rotate-and-sums take three (per-batch) and
  four (fixed part) rotation groups.

Keys: the fixed part's rotations and relinearisation are generated at full height, the other keys only
for the few limbs the per-batch part uses (the same entries as the full keys).

Usage: ``python tests/golden/make_circuit_digests.py [case ...]`` (all cases when none is named).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ckks as C  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402
from synth import config_seed, make_gwas_data  # noqa: E402

OUT = os.path.join(HERE, "circuit_digests.json")

CASES = {
    "gwas_n245_k4_m10643": dict(n=245, k=4, m=10643, kappa=3, log_n=16, log2_scale=40,
                                data_seed=config_seed(2), key_seed=7, enc_seed=11),
    "gwas_n1100_k4_m100": dict(n=1100, k=4, m=100, kappa=3, log_n=16, log2_scale=40,
                               data_seed=config_seed(3, 1), key_seed=7, enc_seed=13),
}


def digest(a: np.ndarray) -> str:
    """SHA-256 of an array's canonical bytes (little-endian 64-bit words, C order)."""
    return hashlib.sha256(np.ascontiguousarray(a).astype("<u8", copy=False).tobytes()).hexdigest()


def poly_digest(m: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(m).astype("<i8", copy=False).tobytes()).hexdigest()


def key_limbs(N: int, R: int, L: int, kappa: int):
    """Per-key limb limits: full height for the keys the fixed part uses (relinearisation and the left
    rotations of its rotation groups), the per-batch limb count for every other key."""
    full = {0} | {C.galois_rotate(N, r) for grp in G.rotation_groups(R, G.FIXED_RADIX) for r in grp}
    low = L + 1 - G.snp_depth(kappa)
    return {g: (L + 1 if g in full else low) for g in G.required_galois(N, R)} | {0: L + 1}


def case_inputs(case: dict):
    """Parameters, layout, data and the oracle's encoded plaintexts of a case (deterministic)."""
    p = C.make_params(case["log_n"], G.circuit_depth(case["kappa"]), case["log2_scale"])
    d = make_gwas_data(case["n"], case["k"], case["m"], seed=case["data_seed"])
    lay = G.make_layout(p.N, case["n"], case["k"], case["m"])
    pts = G.encode_inputs(p, d.X, d.y, d.S, case["kappa"])
    return p, lay, d, pts


def run_case(name: str) -> dict:
    case = CASES[name]
    t0 = time.time()
    p, lay, d, pts = case_inputs(case)
    o = C.Oracle(p)
    kl = key_limbs(p.N, lay.R, p.L, case["kappa"])
    o.keygen(case["key_seed"], G.required_galois(p.N, lay.R), key_limbs=kl)
    print("[%s] keys %.1fs" % (name, time.time() - t0), flush=True)
    inp = G.encrypt_inputs(o, pts, case["n"], case["k"], case["m"], case["kappa"], case["enc_seed"])
    t1 = time.time()
    out = G.Circuit(o, lay).run(inp)
    t_circ = time.time() - t1
    print("[%s] circuit %.1fs (%d key switches)" % (name, t_circ, o.n_keyswitch), flush=True)
    rec = dict(case)
    rec.update({
        "cite": "Alg. Semi Parallel GWAS (with Alg. Homomorphic LogReg and Alg. inverseSlots)",
        "R": lay.R, "tau": lay.tau, "n_batches": lay.n_batches,
        "moduli": [int(q) for q in p.q] + [int(q) for q in p.P],
        "galois": [int(g) for g in G.required_galois(p.N, lay.R)],
        "plaintexts": [poly_digest(m) for m in pts.polys],
        "inputs": {"x": [digest(c.data) for c in inp.x], "y": digest(inp.y.data),
                   "A": [digest(inp.A[pr].data) for pr in G.a_pairs(case["k"])],
                   "S": [digest(c.data) for c in inp.S]},
        "outputs": {"beta": [digest(c.data) for c in out.beta], "w": digest(out.w.data),
                    "w_inv": digest(out.w_inv.data), "z_proj": digest(out.z_proj.data), "u": digest(out.u.data),
                    "S_proj": [digest(c.data) for c in out.S_proj], "num": [digest(c.data) for c in out.num],
                    "den_even": [digest(c.data) for c in out.den_even],
                    "den_odd": [digest(c.data) for c in out.den_odd]},
        "depths": {"beta": out.beta[0].depth, "w": out.w.depth, "w_inv": out.w_inv.depth,
                   "z_proj": out.z_proj.depth, "u": out.u.depth, "S_proj": out.S_proj[0].depth,
                   "num": out.num[0].depth, "den": out.den_even[0].depth},
        "oracle_keyswitches": o.n_keyswitch,
        "oracle_circuit_seconds": round(t_circ, 1),
        "oracle_threads": int(C.lib().ref_num_threads()),
    })
    return rec


def main(names) -> None:
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("SHA-256 digests of the CPU oracle's ciphertexts (canonical form) for the encrypted "
                      "GWAS circuit at full sizes; written by tests/golden/make_circuit_digests.py, which "
                      "calls only oracle/ and synth/.")
    for name in names:
        data[name] = run_case(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")
        print("[%s] written to %s" % (name, OUT), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
