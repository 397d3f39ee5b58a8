"""CPU pin of the device's FP64 modular arithmetic (``csrc/fmod64.h``: fmul_mod, fred, fcanon, u2d, d2u).

The kernels use these for every modulus below 2^41 (the rescale primes and the special primes).  The same
header is compiled for the host (hipcc, host pass only) into ``tests/fmod64_check.cpp`` and checked
against 128-bit integer arithmetic on edge and seeded random operands, for every such modulus of the
chains the tests and the benchmark use.
"""
import os
import subprocess

import pytest

import paper_1902_04303_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "fmod64_check.cpp")
HDR = os.path.join(ROOT, "paper_1902_04303_amd", "csrc", "fmod64.h")
OUT = os.path.join(ROOT, "tests", "_build", "fmod64_check")


@pytest.fixture(scope="module")
def checker():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["/opt/rocm/bin/hipcc", "--offload-host-only", "-x", "hip", "-O2", "-std=c++17", SRC, "-o", OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return OUT


def small_moduli(log_n, levels, b, alpha=0):
    q, p, _ = P.chain(log_n, levels, b, alpha)
    return [m for m in q + p if m < (1 << 41)]


@pytest.mark.parametrize("log_n,levels,b", [(16, 26, 40), (13, 26, 30), (10, 26, 30), (16, 19, 40), (16, 12, 40)])
def test_fp64_modular_arithmetic_matches_128_bit_integers(checker, log_n, levels, b):
    mods = small_moduli(log_n, levels, b)
    assert len(mods) >= levels   # every rescale prime and the special primes
    r = subprocess.run([checker, "20000"] + [str(m) for m in mods], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
