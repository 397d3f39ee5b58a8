"""Pure-Python big-integer CKKS checker for tiny rings — TEST INFRASTRUCTURE ONLY.

Referee for the C oracle.  Every operation is written directly over the big
integers modulo Q = q_0 ... q_l (times P where the definition needs it), with
schoolbook negacyclic products in Z[X]/(X^N + 1) — no NTT, no residue
decomposition.  Limb residues only appear at the boundary (sampling and
comparison).  Only usable for N <= 2^8 or so.

SplitMix64 is implemented here a second time from its published definition
(Steele, Lea and Flood, OOPSLA 2014): output i of the generator seeded with x
is mix(x + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64).
"""
from __future__ import annotations

from typing import List, Sequence

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def sm_mix(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix_out(x: int, i: int) -> int:
    return sm_mix((x + (i + 1) * GAMMA) & MASK64)


def stream(seed: int, sid: int):
    st = splitmix_out(seed, sid)
    return lambda c: splitmix_out(st, c)


def sample_ternary(seed: int, sid: int, N: int) -> List[int]:
    w = stream(seed, sid)
    return [w(i) % 3 - 1 for i in range(N)]


def sample_hwt(seed: int, sid: int, N: int, h: int) -> List[int]:
    w = stream(seed, sid)
    out = [0] * N
    got, c = 0, 0
    while got < h:
        x = w(c)
        c += 1
        pos = x % N
        if out[pos]:
            continue
        out[pos] = -1 if x >> 63 else 1
        got += 1
    return out


def sample_cbd(seed: int, sid: int, N: int) -> List[int]:
    w = stream(seed, sid)
    out = []
    for i in range(N):
        x = w(i)
        out.append(bin(x & 0x1FFFFF).count("1") - bin((x >> 21) & 0x1FFFFF).count("1"))
    return out


def sample_uniform_residues(seed: int, sid: int, mi: int, q: int, N: int) -> List[int]:
    w = stream(seed, sid)
    return [((w(2 * (mi * N + i)) << 64) | w(2 * (mi * N + i) + 1)) % q for i in range(N)]


# ---------------------------------------------------------------- big-int polynomials

def crt(residues: Sequence[Sequence[int]], mods: Sequence[int]) -> List[int]:
    """Combine limb residues into integers in [0, prod(mods))."""
    Q = 1
    for q in mods:
        Q *= q
    N = len(residues[0])
    out = [0] * N
    for r, q in zip(residues, mods):
        Mi = Q // q
        y = Mi * pow(Mi, -1, q)
        for k in range(N):
            out[k] += r[k] * y
    return [v % Q for v in out]


def to_residues(poly: Sequence[int], mods: Sequence[int]) -> List[List[int]]:
    return [[v % q for v in poly] for q in mods]


def polymul(a: Sequence[int], b: Sequence[int], mod: int) -> List[int]:
    """Schoolbook negacyclic product in Z_mod[X]/(X^N + 1)."""
    N = len(a)
    out = [0] * N
    for i in range(N):
        ai = a[i]
        if ai == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += ai * b[j]
            else:
                out[k - N] -= ai * b[j]
    return [v % mod for v in out]


def polyadd(a, b, mod):
    return [(x + y) % mod for x, y in zip(a, b)]


def centred(v: int, mod: int) -> int:
    v %= mod
    return v - mod if v > mod // 2 else v


def round_div(c: Sequence[int], big: int, d: int, small: int) -> List[int]:
    """round(c / d) for c taken centred mod `big`, reduced mod `small` (= big / d)."""
    out = []
    for v in c:
        cv = centred(v, big)
        # nearest integer to cv / d (d odd, no ties)
        qd, r = divmod(cv, d)
        if 2 * r > d:
            qd += 1
        out.append(qd % small)
    return out


def automorph(a: Sequence[int], g: int, mod: int) -> List[int]:
    N = len(a)
    out = [0] * N
    for i, v in enumerate(a):
        e = (i * g) % (2 * N)
        if e < N:
            out[e] = (out[e] + v) % mod
        else:
            out[e - N] = (out[e - N] - v) % mod
    return out


class BigCKKS:
    """Tiny-ring CKKS over big integers with the same definitions as the oracle."""

    def __init__(self, N: int, q: Sequence[int], P: Sequence[int]):
        self.N = N
        self.q = list(q)     # q_0 .. q_L
        self.p = list(P)     # special primes
        self.P = 1
        for v in self.p:
            self.P *= v
        self.L = len(q) - 1

    def Q(self, l: int) -> int:
        out = 1
        for i in range(l):
            out *= self.q[i]
        return out

    def mods_qp(self) -> List[int]:
        return self.q + self.p

    def groups(self, l: int) -> List[List[int]]:
        """Key-switching digit groups of l limbs, alpha = number of special primes: the first alpha - 1
        limbs, then runs of alpha limbs, cut at l (alpha = 2: {0}, {1, 2}, {3, 4}, ...)."""
        a = len(self.p)
        bounds = [0] + list(range(a - 1, l, a)) + [l]
        return [list(range(lo, hi)) for lo, hi in zip(bounds, bounds[1:]) if hi > lo]

    # ---- keys
    def secret(self, seed: int, h: int) -> List[int]:
        return sample_hwt(seed, 1, self.N, h)

    def uniform_poly_qp(self, seed: int, sid: int) -> List[int]:
        """Uniform element of Z_{QP}[X] whose residue modulo each q_t and p_k (indices 0..L+alpha) is sampled."""
        res = [sample_uniform_residues(seed, sid, t, m, self.N) for t, m in enumerate(self.mods_qp())]
        return crt(res, self.mods_qp())

    def uniform_poly_q(self, seed: int, sid: int) -> List[int]:
        res = [sample_uniform_residues(seed, sid, t, m, self.N) for t, m in enumerate(self.q)]
        return crt(res, self.q)

    def public_key(self, s, seed: int):
        QL = self.Q(self.L + 1)
        a = self.uniform_poly_q(seed, 2)
        e = sample_cbd(seed, 3, self.N)
        b = polyadd([-v for v in polymul(a, s, QL)], e, QL)
        return b, a

    def switching_key(self, s, s_prime, seed: int, sid_base: int):
        """ksk_b = (-a_b s + e_b + P * g_b * s', a_b) mod Q_L P, g_b the CRT idempotent of group b."""
        QL = self.Q(self.L + 1)
        QP = QL * self.P
        keys = []
        for b, grp in enumerate(self.groups(self.L + 1)):
            a = self.uniform_poly_qp(seed, sid_base + 2 * b)
            e = sample_cbd(seed, sid_base + 2 * b + 1, self.N)
            g = 0
            for j in grp:
                Mj = QL // self.q[j]
                g += Mj * pow(Mj, -1, self.q[j])
            t = polymul(a, s, QP)
            kb = [(-t[k] + e[k] + self.P * g * s_prime[k]) % QP for k in range(self.N)]
            keys.append((kb, a))
        return keys

    # ---- encryption
    def encrypt(self, pk, m: Sequence[int], l: int, seed: int):
        Ql = self.Q(l)
        v = sample_ternary(seed, 1, self.N)
        e0 = sample_cbd(seed, 2, self.N)
        e1 = sample_cbd(seed, 3, self.N)
        c0 = [(x + y + z) % Ql for x, y, z in zip(polymul(v, pk[0], Ql), m, e0)]
        c1 = [(x + y) % Ql for x, y in zip(polymul(v, pk[1], Ql), e1)]
        return c0, c1

    def decrypt(self, ct, s, l: int) -> List[int]:
        Ql = self.Q(l)
        m = polyadd(ct[0], polymul(ct[1], s, Ql), Ql)
        return [centred(v, Ql) for v in m]

    # ---- evaluation
    def tensor(self, a, b, l: int):
        Ql = self.Q(l)
        d0 = polymul(a[0], b[0], Ql)
        d1 = polyadd(polymul(a[0], b[1], Ql), polymul(a[1], b[0], Ql), Ql)
        d2 = polymul(a[1], b[1], Ql)
        return d0, d1, d2

    def digits(self, d: Sequence[int], l: int) -> List[List[int]]:
        """D_b = sum_{i in G_b} [d_i (Q_G/q_i)^-1]_{q_i} (Q_G/q_i) for every group of l limbs (integers)."""
        out = []
        for grp in self.groups(l):
            QG = 1
            for i in grp:
                QG *= self.q[i]
            D = [0] * self.N
            for i in grp:
                qi, hat = self.q[i], QG // self.q[i]
                hinv = pow(hat % qi, -1, qi)
                for k, v in enumerate(d):
                    D[k] += ((v % qi) * hinv % qi) * hat
            out.append(D)
        return out

    def moddown(self, x: Sequence[int], l: int) -> List[int]:
        """(x - C) / P mod Q_l for x mod Q_l P, C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k) with each [.]_{p_k}
        the centred representative in (-p_k/2, p_k/2)."""
        Ql = self.Q(l)
        out = []
        for v in x:
            C = 0
            for pk in self.p:
                hat = self.P // pk
                C += centred(v * pow(hat % pk, -1, pk) % pk, pk) * hat
            assert (v - C) % self.P == 0
            # |C| < alpha P / 2: the quotient lies within alpha / 2 of v / P
            assert 2 * abs(C) < len(self.p) * self.P
            out.append(((v - C) // self.P) % Ql)
        return out

    def moddown_rescale(self, x: Sequence[int], add: Sequence[int], l: int) -> List[int]:
        """((x + P add) - C) / B mod Q_{l-1} with B = P q_{l-1}: x mod Q_l P, add mod Q_l, x' = x + P add
        as an integer in [0, Q_l P), C = sum_{b in {p_1..p_alpha, q_{l-1}}} [x' (B/b)^-1]_b (B/b) with each
        [.]_b the centred representative in (-b/2, b/2)."""
        Ql = self.Q(l)
        QP = Ql * self.P
        ql = self.q[l - 1]
        B = self.P * ql
        Q1 = Ql // ql
        out = []
        for v, a in zip(x, add):
            xp = (v + self.P * (a % Ql)) % QP
            C = 0
            for b in self.p + [ql]:
                hat = B // b
                C += centred(xp * pow(hat % b, -1, b) % b, b) * hat
            assert (xp - C) % B == 0
            # |C| < (alpha + 1) B / 2: the quotient lies within (alpha + 1) / 2 of x' / B
            assert 2 * abs(C) < (len(self.p) + 1) * B
            out.append(((xp - C) // B) % Q1)
        return out

    def accumulate(self, d: Sequence[int], key_list, l: int):
        """x = sum_i sum_b sigma_{g_i}(D_b) ksk_{i,b} mod Q_l P (both components), before any division."""
        Ql = self.Q(l)
        QP = Ql * self.P
        D = self.digits(d, l)
        acc0 = [0] * self.N
        acc1 = [0] * self.N
        for g, keys in key_list:
            for b, Db in enumerate(D):
                db = [v % QP for v in Db]
                if g:
                    db = automorph(db, g, QP)
                kb, ka = keys[b]
                acc0 = polyadd(acc0, polymul(db, [v % QP for v in kb], QP), QP)
                acc1 = polyadd(acc1, polymul(db, [v % QP for v in ka], QP), QP)
        return acc0, acc1

    def mul_rescale(self, a, b, rlk, l: int):
        """Product with relinearisation and rescale in one division: tensor (d0, d1, d2), x = the key-switch
        sum of d2 with the s^2 key, out_c = ((x_c + P d_c) - C) / (P q_{l-1}) for c = 0, 1."""
        d0, d1, d2 = self.tensor(a, b, l)
        x0, x1 = self.accumulate(d2, [(0, rlk)], l)
        return self.moddown_rescale(x0, d0, l), self.moddown_rescale(x1, d1, l)

    def keyswitch(self, d: Sequence[int], keys, l: int):
        """Key switch of d (an element of Z_{Q_l}[X]) with the key `keys` (keyswitch_galois, no automorphism)."""
        return self.keyswitch_galois(d, [(0, keys)], l)

    def keyswitch_galois(self, d: Sequence[int], key_list, l: int):
        """(x - C) / P for x = sum_i sum_b sigma_{g_i}(D_b) * ksk_{i,b} mod Q_l P, key_list = [(g_i, keys_i)]:
        each digit D_b (an integer polynomial) is permuted by X -> X^{g_i} (g_i = 0: not permuted)
        before the product; one division by P for the whole sum."""
        Ql = self.Q(l)
        QP = Ql * self.P
        D = self.digits(d, l)
        acc0 = [0] * self.N
        acc1 = [0] * self.N
        for g, keys in key_list:
            for b, Db in enumerate(D):
                db = [v % QP for v in Db]
                if g:
                    db = automorph(db, g, QP)
                kb, ka = keys[b]
                acc0 = polyadd(acc0, polymul(db, [v % QP for v in kb], QP), QP)
                acc1 = polyadd(acc1, polymul(db, [v % QP for v in ka], QP), QP)
        return self.moddown(acc0, l), self.moddown(acc1, l)

    def apply_galois(self, ct, g: int, keys, l: int):
        """(sigma_g(c0), 0) + key switch of sigma_g(c1) from sigma_g(s) back to s."""
        Ql = self.Q(l)
        ks = self.keyswitch_galois(ct[1], [(g, keys)], l)
        return polyadd(automorph(ct[0], g, Ql), ks[0], Ql), ks[1]

    def rotate_sum(self, ct, key_list, l: int):
        """ct + sum_i sigma_{g_i}(ct), the key switches of all g_i sharing one division by P."""
        Ql = self.Q(l)
        ks = self.keyswitch_galois(ct[1], key_list, l)
        c0 = list(ct[0])
        for g, _ in key_list:
            c0 = polyadd(c0, automorph(ct[0], g, Ql), Ql)
        return polyadd(c0, ks[0], Ql), polyadd(ct[1], ks[1], Ql)

    def rescale(self, ct, l: int):
        Ql = self.Q(l)
        ql = self.q[l - 1]
        return tuple(round_div(c, Ql, ql, Ql // ql) for c in ct)
