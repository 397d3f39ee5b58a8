"""Host-side checks of the HIP library that need no GPU: it loads, exports every
symbol the C header declares, and its prime-chain rule agrees with the oracle's."""
import ctypes
import os
import re

import pytest

import paper_1902_04303_amd as P
from oracle import ckks as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gwas_ckks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:ckks|gwas)_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_symbols()
    assert len(names) > 40
    for name in names:
        assert hasattr(lib, name), name
    assert set(P.exported_symbols()) == set(names)


@pytest.mark.parametrize("log_n,levels,b", [(10, 4, 30), (13, 26, 30), (16, 26, 40), (16, 19, 40)])
def test_prime_chain_matches_oracle(log_n, levels, b):
    q, Pm, scales = P.chain(log_n, levels, b)
    ref = C.make_params(log_n, levels, b)
    assert q == ref.q and Pm == ref.P
    assert scales == ref.scales


@pytest.mark.parametrize("alpha", [2, 3, 5, 8])
def test_special_primes_follow_the_group_size(alpha):
    q, Pm, _ = P.chain(13, 12, 30, alpha)
    ref = C.make_params(13, 12, 30, alpha)
    assert P.ks_alpha(13, 12, 30, alpha) == alpha == len(Pm)
    assert q == ref.q and Pm == ref.P
    assert P.ks_alpha(13, 12, 30) == len(C.make_params(13, 12, 30).P)   # the two defaults agree


@pytest.mark.parametrize("log_n,R", [(10, 2), (10, 8), (10, 64), (13, 256), (16, 256), (16, 2048), (16, 32768)])
def test_galois_elements_match_oracle(log_n, R):
    from oracle import gwas_circuit as G
    assert P.gwas_galois_elements(log_n, R) == G.required_galois(1 << log_n, R)


@pytest.mark.parametrize("radix", [4, 16])
def test_rotation_groups_cover_every_shift_once(radix):
    """The grouped rotate-and-sum adds Rot(a, i) for each i < R exactly once (both implementations'
    group lists generate the same Galois elements, checked above): the sums of one shift per group,
    taken with multiplicity, are 0..R-1 each once."""
    from oracle import gwas_circuit as G
    for R in (2, 4, 8, 16, 32, 64, 128, 256, 2048, 32768):
        sums = [0]
        groups = G.rotation_groups(R, radix)
        for grp in groups:
            assert 1 <= len(grp) <= radix - 1
            sums = [a + b for a in sums for b in [0] + grp]
        assert sorted(sums) == list(range(R)), (R, radix)
        # key switches per rotate-and-sum: ceil(log2 R / log2 radix)
        lr, lk = R.bit_length() - 1, radix.bit_length() - 1
        assert len(groups) == -(-lr // lk), (R, radix)


def test_rotation_groups_radix4_are_the_triples():
    """Radix 4 groups two doubling steps of Alg. colSum: {s, 2s, 3s} for s = 1, 4, 16, .., then {s}."""
    from oracle import gwas_circuit as G
    assert G.rotation_groups(256, 4) == [[1, 2, 3], [4, 8, 12], [16, 32, 48], [64, 128, 192]]
    assert G.rotation_groups(512, 4) == [[1, 2, 3], [4, 8, 12], [16, 32, 48], [64, 128, 192], [256]]
    assert G.rotation_groups(256, 16) == [list(range(1, 16)), list(range(16, 256, 16))]
    assert G.rotation_groups(8, 16) == [list(range(1, 8))]


def test_bad_parameters_are_rejected():
    with pytest.raises(P.CkksError) as e:
        P.chain(9, 4, 30)
    assert e.value.code == -1
    with pytest.raises(P.CkksError):
        P.chain(13, 4, 60)
    for bad in (1, 9, -2):
        with pytest.raises(P.CkksError):
            P.chain(13, 4, 30, bad)
