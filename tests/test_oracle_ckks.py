"""Pins of the CPU oracle's RNS-CKKS (no GPU).

The C oracle is checked against things other than itself: a second, pure-Python
big-integer implementation of every definition (schoolbook products, no NTT, no
residue decomposition), exact identities, and the decode of what it encrypts.
"""
import json
import os

import numpy as np
import pytest

from oracle import bigint_ref as B
from oracle import ckks as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def tiny(logN=4, L=3, b=20):
    p = C.make_params(logN, L, b)
    return p, C.Oracle(p)


def _res(poly, q):
    return [v % q for v in poly]


# ------------------------------------------------------------------ randomness

def test_splitmix_matches_published_definition():
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        i = int(rng.integers(0, 2**40))
        assert int(C.lib().ref_splitmix_out(x, i)) == B.splitmix_out(x, i)


@pytest.mark.parametrize("seed,sid", [(7, 1), (11, 3), (2**63 + 5, 1 << 40)])
def test_samplers_match_bigint(seed, sid):
    N = 256
    t = np.zeros(N, dtype=np.int64)
    C.lib().ref_sample_ternary(seed, sid, N, C._p(t))
    assert t.tolist() == B.sample_ternary(seed, sid, N)
    C.lib().ref_sample_cbd(seed, sid, N, C._p(t))
    assert t.tolist() == B.sample_cbd(seed, sid, N)
    assert abs(t.mean()) < 1.0 and 6.0 < t.var() < 16.0       # variance 10.5
    C.lib().ref_sample_hwt(seed, sid, N, 64, C._p(t))
    assert t.tolist() == B.sample_hwt(seed, sid, N, 64)
    assert np.count_nonzero(t) == 64 and set(np.unique(t)) <= {-1, 0, 1}
    q = 1073754113
    u = np.zeros(N, dtype=np.uint64)
    C.lib().ref_sample_uniform(seed, sid, 3, q, N, C._p(u))
    assert u.tolist() == B.sample_uniform_residues(seed, sid, 3, q, N)


# ------------------------------------------------------------------ arithmetic

@pytest.mark.parametrize("logN", [4, 6, 8])
def test_polymul_matches_schoolbook(logN):
    p, o = tiny(logN=logN, L=2)
    rng = np.random.default_rng(logN)
    for mi, q in enumerate(o.mods):
        a = rng.integers(0, q, size=p.N, dtype=np.uint64)
        b = rng.integers(0, q, size=p.N, dtype=np.uint64)
        out = np.zeros(p.N, dtype=np.uint64)
        C.lib().ref_polymul(o._ctx, mi, C._p(a), C._p(b), C._p(out))
        assert out.tolist() == B.polymul(a.tolist(), b.tolist(), q)


def test_eval_form_roundtrip_and_linearity():
    p, o = tiny(logN=8, L=2)
    rng = np.random.default_rng(1)
    q = o.mods[1]
    a = rng.integers(0, q, size=p.N, dtype=np.uint64)
    b = rng.integers(0, q, size=p.N, dtype=np.uint64)
    fa, fb, fab, back = (np.zeros(p.N, dtype=np.uint64) for _ in range(4))
    C.lib().ref_to_eval(o._ctx, 1, C._p(a), C._p(fa))
    C.lib().ref_from_eval(o._ctx, 1, C._p(fa), C._p(back))
    assert np.array_equal(back, a)
    s = ((a.astype(object) + b.astype(object)) % q).astype(np.uint64)
    C.lib().ref_to_eval(o._ctx, 1, C._p(b), C._p(fb))
    C.lib().ref_to_eval(o._ctx, 1, C._p(s), C._p(fab))
    assert np.array_equal(fab, ((fa.astype(object) + fb.astype(object)) % q).astype(np.uint64))


def test_prime_chain_rule():
    for logN, L, b, alpha in [(4, 3, 20, 2), (4, 3, 20, 4), (13, 26, 30, 3), (16, 26, 40, 2), (16, 26, 40, 4),
                              (16, 26, 40, 8)]:
        p = C.make_params(logN, L, b, alpha)
        N = 1 << logN
        mods = p.q + p.P
        assert len(set(mods)) == len(mods)
        for q in mods:
            assert q % (2 * N) == 1
            # independent primality evidence: no small factor and Fermat witnesses
            assert all(q % d for d in range(3, 2000, 2))
            assert all(pow(a, q - 1, q) == 1 for a in (2, 3, 5, 7, 11, 13, 101))
        assert p.q[0].bit_length() == 60 and all(x.bit_length() == 41 for x in p.P)
        assert len(p.P) == alpha and p.P == sorted(p.P, reverse=True)
        # no prime 1 mod 2N lies between 2^41 and the smallest special prime outside the chain and P
        for c in range(p.P[-1] + 2 * N, 1 << 41, 2 * N):
            if all(pow(a, c - 1, c) == 1 for a in (2, 3, 5, 7)):
                assert c in p.P or c in p.q
        # P exceeds the product of every digit group's moduli (keeps the key-switching noise small)
        groups = C.digit_groups(L + 1, alpha)
        assert sum(len(g) for g in groups) == L + 1 and groups[0][0] == 0
        for g in groups:
            QG = 1
            for i in g:
                QG *= p.q[i]
            assert p.P_prod > QG
        assert all(x.bit_length() == b + (1 if x >= 1 << b else 0) for x in p.q[1:])
        # canonical scales follow Delta_{d+1} = Delta_d^2 / q_{L-d} and stay near 2^b
        for d in range(L):
            assert p.scales[d + 1] == (p.scales[d] * p.scales[d]) / float(p.q[L - d])
        dev = max(abs(s / 2.0 ** b - 1) for s in p.scales)
        assert dev < (1e-4 if logN == 16 else 3e-3)


# ------------------------------------------------------------------ keys / encryption against big integers

@pytest.fixture(scope="module", params=[2, 3, 4])
def tiny_keys(request):
    p = C.make_params(4, 3, 20, request.param)   # alpha 2: {0} {1 2} {3}; 3: {0 1} {2 3}; 4: {0 1 2} {3}
    o = C.Oracle(p)
    g = [C.galois_rotate(p.N, 1), C.galois_conj(p.N), C.galois_rotate(p.N, 2), C.galois_rotate(p.N, 3)]
    o.keygen(5, g)
    bc = B.BigCKKS(p.N, p.q, p.P)
    s = bc.secret(5, C.secret_weight(p.N))
    assert o.sk.tolist() == s
    return p, o, bc, s, g


def test_secret_and_public_key_match_bigint(tiny_keys):
    p, o, bc, _, _ = tiny_keys
    N = 256
    t = np.zeros(N, dtype=np.int64)
    C.lib().ref_sample_hwt(5, C.SID_SECRET, N, C.SECRET_HW, C._p(t))
    assert t.tolist() == B.sample_hwt(5, C.SID_SECRET, N, C.SECRET_HW)
    s = o.sk.tolist()
    b, a = bc.public_key(s, 5)
    QL = bc.Q(p.L + 1)
    for t, q in enumerate(p.q):
        assert o.pk[0, t].tolist() == _res(b, q)
        assert o.pk[1, t].tolist() == _res(a, q)


def test_switching_keys_match_bigint(tiny_keys):
    p, o, bc, _, g = tiny_keys
    s = o.sk.tolist()
    QP = bc.Q(p.L + 1) * bc.P
    s2 = B.polymul(s, s, QP)
    targets = {0: s2, g[0]: B.automorph(s, g[0], QP), g[1]: B.automorph(s, g[1], QP)}
    for K, sp in targets.items():
        keys = bc.switching_key(s, sp, 5, C.ksk_sid_base(K))
        key = o.keys[K]
        assert key.shape[1] == len(keys) == len(C.digit_groups(p.L + 1, p.alpha))
        for j in range(len(keys)):
            for t, q in enumerate(p.q + p.P):
                assert key[0, j, t].tolist() == _res(keys[j][0], q), (K, j, t)
                assert key[1, j, t].tolist() == _res(keys[j][1], q), (K, j, t)


def _ct_big(ct, p, l):
    return tuple(B.crt([ct.data[c, i].tolist() for i in range(l)], p.q[:l]) for c in range(2))


def test_encrypt_tensor_keyswitch_rescale_match_bigint(tiny_keys):
    p, o, bc, _, g = tiny_keys
    s = o.sk.tolist()
    rng = np.random.default_rng(3)
    l = p.L + 1
    m1 = rng.integers(-1000, 1000, size=p.N).astype(np.int64)
    m2 = rng.integers(-1000, 1000, size=p.N).astype(np.int64)
    c1 = o.encrypt(m1, 0, p.scales[0], 21)
    c2 = o.encrypt(m2, 0, p.scales[0], 22)
    pk = (B.crt([o.pk[0, t].tolist() for t in range(l)], p.q), B.crt([o.pk[1, t].tolist() for t in range(l)], p.q))
    b1 = bc.encrypt(pk, m1.tolist(), l, 21)
    assert _ct_big(c1, p, l) == b1
    b2 = _ct_big(c2, p, l)
    # tensor
    d = o.tensor([(c1, c2)])
    bd = bc.tensor(b1, b2, l)
    for c in range(3):
        assert B.crt([d[c, i].tolist() for i in range(l)], p.q[:l]) == bd[c]
    # key switch with the relinearisation key at a reduced level
    lk = l - 1
    QP = bc.Q(p.L + 1) * bc.P
    keys = bc.switching_key(s, B.polymul(s, s, QP), 5, C.ksk_sid_base(0))
    dd = np.ascontiguousarray(d[2, :lk])
    ks = o.keyswitch(dd, 0)
    bks = bc.keyswitch(B.crt([dd[i].tolist() for i in range(lk)], p.q[:lk]), keys, lk)
    for c in range(2):
        assert B.crt([ks[c, i].tolist() for i in range(lk)], p.q[:lk]) == bks[c]
    # rescale
    r = o.rescale(c1)
    br = bc.rescale(b1, l)
    assert _ct_big(r, p, l - 1) == br
    # the product: relinearisation and rescale in one division by P q_{l-1} (mul / mul_sum), at the top
    # level and one level down
    for lev in (l, l - 1):
        a1 = C.Ct(np.ascontiguousarray(c1.data[:, :lev]), p.L + 1 - lev, c1.scale)
        a2 = C.Ct(np.ascontiguousarray(c2.data[:, :lev]), p.L + 1 - lev, c2.scale)
        pr = o.mul(a1, a2)
        assert pr.limbs == lev - 1
        want = bc.mul_rescale(_ct_big(a1, p, lev), _ct_big(a2, p, lev), keys, lev)
        assert _ct_big(pr, p, lev - 1) == want, lev
        # against the two divisions taken one after the other (ModDown by P, then the centred rescale by
        # q_{lev-1}): the one division differs by at most alpha / 2 + 2 per coefficient
        bd = bc.tensor(_ct_big(a1, p, lev), _ct_big(a2, p, lev), lev)
        Ql = bc.Q(lev)
        kd = bc.keyswitch(bd[2], keys, lev)
        seq = bc.rescale(tuple([(x + y) % Ql for x, y in zip(bd[c], kd[c])] for c in range(2)), lev)
        Q1 = Ql // p.q[lev - 1]
        for c in range(2):
            diff = [((w - v + Q1 // 2) % Q1) - Q1 // 2 for w, v in zip(want[c], seq[c])]
            assert max(abs(x) for x in diff) <= o.alpha // 2 + 2, (lev, c)


def test_divisions_by_p_are_unbiased():
    """The centred fast conversions of ModDown and of the product's one division by P q_{l-1}: their
    rounding errors have mean near 0 over a ring of 2^10 coefficients (uncentred conversions would shift
    every coefficient by about alpha / 2 and (alpha + 1) / 2 units, which the slots sum coherently), and
    stay within alpha / 2 + 1 and (alpha + 1) / 2 + 1 of the exactly rounded quotients.  The exact
    quotients come from Python integers on the same x (CRT of the oracle's residues)."""
    p = C.make_params(10, 3, 30, 3)
    alpha = p.alpha
    rng = np.random.default_rng(12)
    l = p.L + 1
    QP = B.BigCKKS(p.N, p.q, p.P)
    Ql = QP.Q(l)
    Pm = QP.P
    mods = list(p.q[:l]) + list(p.P)
    # x: uniform residues on q_0..q_{l-1}, p_1..p_alpha; add: uniform residues on q_0..q_{l-1}
    x = np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in mods])
    add = np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in p.q[:l]])
    xb = B.crt([x[i].tolist() for i in range(len(mods))], mods)
    ab = B.crt([add[i].tolist() for i in range(l)], p.q[:l])
    md = QP.moddown(xb, l)
    exact = [B.centred(v, Ql * Pm) for v in xb]
    # round(v / P) = floor((2 v + P) / (2 P)) (P odd: no ties)
    err = [B.centred(int(m) - (2 * v + Pm) // (2 * Pm), Ql) for m, v in zip(md, exact)]
    assert max(abs(e) for e in err) <= alpha // 2 + 1
    assert abs(np.mean(err)) < 0.1
    ql = p.q[l - 1]
    Bq = Pm * ql
    mr = QP.moddown_rescale(xb, ab, l)
    Q1 = Ql // ql
    xp = [B.centred((v + Pm * a) % (Ql * Pm), Ql * Pm) for v, a in zip(xb, ab)]
    err2 = [B.centred(int(m) - ((2 * v + Bq) // (2 * Bq)), Q1) for m, v in zip(mr, xp)]
    assert max(abs(e) for e in err2) <= (alpha + 1) // 2 + 1
    assert abs(np.mean(err2)) < 0.1


def test_rotation_and_grouped_rotation_sum_match_bigint(tiny_keys):
    """Key switch of an automorphism (digits lifted, then permuted) and the grouped rotate-and-sum
    (three rotations, one division by P) against the big-integer schoolbook implementation."""
    p, o, bc, s, g = tiny_keys
    QP = bc.Q(p.L + 1) * bc.P
    keys = {gg: bc.switching_key(s, B.automorph(s, gg, QP), 5, C.ksk_sid_base(gg)) for gg in g}
    rng = np.random.default_rng(6)
    for l in (p.L + 1, 2):
        ct = C.Ct(np.stack([np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in p.q[:l]])
                            for _ in range(2)]).copy(), p.L + 1 - l, 1.0)
        big = _ct_big(ct, p, l)
        for gg in g[:2]:
            assert _ct_big(o.apply_galois(ct, gg), p, l) == bc.apply_galois(big, gg, keys[gg], l), (l, gg)
        got = o.rotate_sum(ct, [1, 2, 3])
        want = bc.rotate_sum(big, [(gg, keys[gg]) for gg in (g[0], g[2], g[3])], l)
        assert _ct_big(got, p, l) == want, l


def test_automorphism_matches_bigint(tiny_keys):
    p, o, bc, _, g = tiny_keys
    rng = np.random.default_rng(4)
    ct = C.Ct(np.stack([np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in p.q[:2]])] * 2).copy(), 0, 1.0)
    for gg in g + [C.galois_rotate(p.N, -2)]:
        out = o.automorph(ct, gg)
        for c in range(2):
            for i in range(2):
                assert out.data[c, i].tolist() == B.automorph(ct.data[c, i].tolist(), gg, p.q[i])


# ------------------------------------------------------------------ encoding and scheme semantics

def test_encode_decode_roundtrip_and_exact_encodings():
    N = 1 << 10
    rng = np.random.default_rng(5)
    z = rng.standard_normal(N // 2) + 1j * rng.standard_normal(N // 2)
    assert np.max(np.abs(C.decode_poly(C.encode_real_poly(z, N), N) - z)) < 1e-12
    scale = 2.0 ** 30
    m = C.encode(z, N, scale)
    assert np.max(np.abs(C.decode_poly(m.astype(np.float64) / scale, N) - z)) < N * 2.0 ** -30
    # a replicated scalar is the constant polynomial
    c = 0.123456789
    mc = C.encode(np.full(N // 2, c), N, scale)
    assert abs(int(mc[0]) - C.round_half_away(c * scale)) <= 1 and np.max(np.abs(mc[1:])) <= 1
    # block-start mask: closed form with 2R nonzero coefficients, within 1 of the dense encoder
    R = 32
    ind = (np.arange(N // 2) % R == 0).astype(np.complex128)
    dense = C.encode(ind, N, scale)
    mask = C.mask_block_start_poly(N, R, scale)
    assert np.max(np.abs(dense - mask)) <= 1
    assert np.count_nonzero(mask) == 2 * R - 1         # the X^(N/2) coefficient, cos(pi/2) = 0
    nz = np.nonzero(mask)[0]
    assert np.all(nz % (N // (2 * R)) == 0)
    assert int(mask[0]) == C.round_half_away(scale / R)


def test_r_periodic_vectors_live_in_the_subring():
    N, R = 1 << 10, 16
    rng = np.random.default_rng(6)
    v = rng.standard_normal(R)
    z = v[np.arange(N // 2) % R]
    m = C.encode_real_poly(z, N)
    off = np.ones(N, dtype=bool)
    off[:: N // (2 * R)] = False
    assert np.max(np.abs(m[off])) < 1e-12


def test_rotation_conjugation_and_mult_semantics():
    p = C.make_params(10, 3, 30)
    o = C.Oracle(p)
    o.keygen(9, [C.galois_rotate(p.N, 1), C.galois_rotate(p.N, 4), C.galois_rotate(p.N, -4), C.galois_conj(p.N),
                 C.galois_rotate(p.N, -8), C.galois_rotate(p.N, -12)])
    rng = np.random.default_rng(7)
    z = rng.standard_normal(p.slots) + 1j * rng.standard_normal(p.slots)
    w = rng.standard_normal(p.slots)
    ct = o.encrypt(C.encode(z, p.N, p.scales[0]), 0, p.scales[0], 1)
    cw = o.encrypt(C.encode(w, p.N, p.scales[0]), 0, p.scales[0], 2)
    tol = 1e-4
    assert np.max(np.abs(o.decrypt(ct) - z)) < tol
    assert np.max(np.abs(o.decrypt(o.rotate(ct, 1)) - np.roll(z, -1))) < tol
    assert np.max(np.abs(o.decrypt(o.rotate(ct, 4)) - np.roll(z, -4))) < tol
    assert np.max(np.abs(o.decrypt(o.rotate(ct, -4)) - np.roll(z, 4))) < tol
    assert np.max(np.abs(o.decrypt(o.conjugate(ct)) - np.conj(z))) < tol
    pr = o.mul(ct, cw)
    assert pr.depth == 1 and pr.scale == p.scales[1]
    assert np.max(np.abs(o.decrypt(pr) - z * w)) < 10 * tol
    # rotation composition: rot(rot(a, 1), 4) equals rot(a, 5) up to noise
    assert np.max(np.abs(o.decrypt(o.rotate(o.rotate(ct, 1), 4)) - np.roll(z, -5))) < tol
    want = z + np.roll(z, 4) + np.roll(z, 8) + np.roll(z, 12)
    assert np.max(np.abs(o.decrypt(o.rotate_sum(ct, [-4, -8, -12])) - want)) < 4 * tol
    # integer multiply and constants
    assert np.max(np.abs(o.decrypt(o.mul_int(ct, -3)) + 3 * z)) < 10 * tol
    assert np.max(np.abs(o.decrypt(o.add_const(ct, 0.75)) - (z + 0.75))) < tol
    assert np.max(np.abs(o.decrypt(o.mul_const(ct, 0.3)) - 0.3 * z)) < tol
    al = o.align(ct, 2, p.scales[2], 0.125)
    assert al.depth == 2 and np.max(np.abs(o.decrypt(al) - z / 8)) < tol
    mk = o.mul_mask(ct, 8)
    zm = np.where(np.arange(p.slots) % 8 == 0, z, 0)
    assert np.max(np.abs(o.decrypt(mk) - zm)) < tol


def test_mul_i_is_the_exact_monomial_shift():
    """mul_i multiplies by X^(N/2): the decryption polynomial is shifted negacyclically by N/2 with no
    rounding, and every slot (the value at zeta^(5^j), zeta = exp(i pi / N)) is multiplied by i; with
    neg by -i.  The packed denominators' (2 + 2i) S conj(S) + (1 - i) (S^2 + conj(S)^2) is 4 (a^2 + i b^2)."""
    p = C.make_params(10, 2, 30)
    o = C.Oracle(p)
    o.keygen(3, [C.galois_conj(p.N)])
    rng = np.random.default_rng(21)
    z = rng.standard_normal(p.slots) + 1j * rng.standard_normal(p.slots)
    ct = o.encrypt(C.encode(z, p.N, p.scales[0]), 0, p.scales[0], 4)
    h = p.N // 2
    m0 = o.decrypt_poly(ct)
    for neg, unit in ((False, 1j), (True, -1j)):
        r = o.mul_i(ct, neg)
        assert r.depth == ct.depth and r.scale == ct.scale
        m1 = o.decrypt_poly(r)
        sgn = -1 if neg else 1
        # X^(N/2) m(X) mod X^N + 1: coefficient t moves to t + N/2, wrapping with a sign change
        assert all(m1[t + h] == sgn * m0[t] and m1[t] == -sgn * m0[t + h] for t in range(h))
        assert np.max(np.abs(o.decrypt(r) - unit * z)) < 1e-4
    # mul_i twice is the negation, bit for bit
    assert np.array_equal(o.mul_i(o.mul_i(ct)).data, o.neg(ct).data)
    # Gaussian-integer factors: (2 + 2i) and (1 - i) per slot, exactly (2 + 2X^(N/2), 1 - X^(N/2))
    assert np.max(np.abs(o.decrypt(o.mul_gauss(ct, 2, 2)) - (2 + 2j) * z)) < 1e-3
    assert np.array_equal(o.mul_gauss(ct, 1, -1).data, o.sub(ct, o.mul_i(ct)).data)
    # the packing of two real squares into one complex slot:
    # (2 + 2i) S conj(S) + (1 - i) (S^2 + conj(S)^2) = 4 (a^2 + i b^2) for S = a + i b
    a = rng.uniform(-1, 1, p.slots)
    b = rng.uniform(-1, 1, p.slots)
    cs = o.encrypt(C.encode(a + 1j * b, p.N, p.scales[0]), 0, p.scales[0], 5)
    cc = o.conjugate(cs)
    t = o.mul_sum([(o.mul_gauss(cs, 2, 2), cc), (o.mul_gauss(cs, 1, -1), cs), (o.mul_gauss(cc, 1, -1), cc)])
    assert np.max(np.abs(o.decrypt(t) - 4 * (a * a + 1j * b * b))) < 1e-3


# ------------------------------------------------------------------ values printed in the paper

def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        return json.load(f)


def test_power_of_two_rotation_counts():
    for r, count in _golden()["power_of_two_rotations"]["cases"]:
        assert bin(r).count("1") == count


def test_snp_batching_example():
    g = _golden()["snp_batching"]
    N = 1 << g["logN"]
    R = 1
    while R < g["n"]:
        R *= 2
    tau = N // R          # two SNPs per complex slot, N/2 slots, R rows per column
    assert tau == g["tau"]
    assert -(-g["m"] // tau) == g["batches"]
