"""Oracle RNS-CKKS driver — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library.

It wraps the C core (``ckks_ref.c``: coefficient-form polynomial arithmetic)
with the scheme-level logic of the paper's CKKS description (Methods,
"Homomorphic Encryption"): parameters and the RNS prime chain, encoding by the
inverse canonical embedding, key generation, encryption, decryption, and the
evaluation operations with level and scale tracking.

Readings taken where the paper is silent (the paper describes the non-RNS
scheme with power-of-two moduli):

* Prime chain.  q_0 is the largest prime below 2^60 that is 1 mod 2N.  The
  special modulus P = p_1 ... p_alpha is the product of the alpha largest primes
  below 2^41 that are 1 mod 2N and not in the chain, alpha the digit-group size
  of the key switch (P above every digit modulus keeps the key-switching noise
  small).  Rescale primes come from a pool of
  the 4L primes that are 1 mod 2N and nearest to 2^b; for depth d = 0..L-1 the
  unused pool prime nearest to Delta_d^2 / 2^b becomes q_{L-d} (ties to the
  smaller prime), and Delta_{d+1} = (Delta_d * Delta_d) / q_{L-d} in FP64, with
  Delta_0 = 2^b.  This keeps every canonical scale within a few parts in 10^4
  of 2^b (the doubling recursion of scales is otherwise unstable).
* Slot j of a ciphertext is the evaluation at zeta^(5^j mod 2N), zeta = exp(i pi / N).
* Constants: a real c is added at the ciphertext's scale s as the integer
  round_half_away(c * s) in the constant coefficient; a real factor c (and the
  block-start mask) is multiplied encoded at the ciphertext's scale s followed by
  a rescale by q, so the result scale is (s * s) / q, the same canonical
  progression as a ciphertext product.
* Alignment to a deeper (depth, scale): mod-drop to one level above the target,
  multiply by the integer round_half_away(((scale * factor) * q) / s), rescale by
  q and declare the target scale (the residual is below 1 / (2 * integer)).
* Multiplication: tensor product (d0, d1, d2), relinearisation of d2, rescale by
  the last prime q; the result scale is (s_a * s_b) / q in FP64.  The division by
  P that ends the relinearisation's key switch and the rescale's division by q
  are taken as one division by P q of x' = x + P (d0, d1) (x the key switch's
  sum of digit-key products): (x' - C) / (P q) with
  C = sum_b [x' (P q / b)^-1]_b (P q / b), b over q and p_1..p_alpha.  It is the
  same fast conversion as the key switch's own division, with q counted among the
  special primes; each result coefficient lies within alpha + 1 of the exactly
  rounded quotient (relin_rescale).
* Key switching (the paper's non-RNS KeyGen / Mult, in RNS with a hybrid
  decomposition): digit groups of alpha primes, {q_0 .. q_{alpha-2}}, then
  {q_{alpha-1} .. q_{2 alpha-2}}, ... (digit_groups; alpha = 2 gives {q_0},
  {q_1, q_2}, ...);
  a ciphertext with l limbs uses each group's members below l.  Digit b is the
  integer D_b = sum_{i in G_b} [d_i (Q_G/q_i)^-1]_{q_i} (Q_G/q_i) (fast basis
  conversion), key b is (-a_b s + e_b + P e_{G_b} s', a_b) mod Q_L P with e_G the
  CRT idempotent of the group (1 modulo its primes, 0 modulo the other q_i), and
  the sum of digit-key products x is divided by P as (x - C) / P with
  C = sum_k [x (P/p_k)^-1]_{p_k} (P/p_k).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from decimal import Decimal, getcontext
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import build as _build

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)

# --------------------------------------------------------------------------
# C core
# --------------------------------------------------------------------------

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.ref_ctx_new.restype = ctypes.c_void_p
        L.ref_ctx_new.argtypes = [ctypes.c_int, ctypes.c_int, _u64p, _u64p]
        L.ref_ctx_free.argtypes = [ctypes.c_void_p]
        L.ref_splitmix_out.restype = ctypes.c_uint64
        L.ref_splitmix_out.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ref_word.restype = ctypes.c_uint64
        L.ref_word.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.ref_sample_ternary.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _i64p]
        L.ref_sample_hwt.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _i64p]
        L.ref_sample_cbd.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _i64p]
        L.ref_sample_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_int, _u64p]
        L.ref_to_eval.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.ref_from_eval.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.ref_polymul.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p, _u64p]
        L.ref_add.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, _u64p, _u64p]
        L.ref_sub.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, _u64p, _u64p]
        L.ref_mul_int.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_int64, _u64p]
        L.ref_add_const.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_int64]
        L.ref_mul_plain.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, _i64p, _u64p]
        L.ref_tensor.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p, _u64p, ctypes.c_int]
        L.ref_rescale.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, _u64p]
        L.ref_automorph.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_uint64, _u64p]
        L.ref_keyswitch.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_int,
                                    _u64p, ctypes.POINTER(_u64p), ctypes.c_int, _u64p]
        L.ref_keyswitch_rescale.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p,
                                            ctypes.c_int, _u64p, ctypes.POINTER(_u64p), ctypes.c_int, _u64p, _u64p]
        L.ref_gen_ksk.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _i64p, _u64p, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_int, _u64p]
        L.ref_key_to_eval.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p, _u64p]
        L.ref_num_threads.restype = ctypes.c_int
        L.ref_set_threads.argtypes = [ctypes.c_int]
        L.ref_gen_pk.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, _u64p]
        L.ref_encrypt.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_int, _i64p, ctypes.c_uint64,
                                  _u64p]
        L.ref_decrypt.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _i64p, _u64p]
        L.ref_secret_square.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, _u64p]
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    if a.dtype == np.uint64:
        assert a.flags.c_contiguous
        return a.ctypes.data_as(_u64p)
    if a.dtype == np.int64:
        assert a.flags.c_contiguous
        return a.ctypes.data_as(_i64p)
    raise TypeError(a.dtype)


# --------------------------------------------------------------------------
# number theory (plain Python integers)
# --------------------------------------------------------------------------

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (bases: the first twelve primes)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primitive_2n_root(q: int, N: int) -> int:
    """Smallest-generator-derived psi with psi^N = -1 mod q (a primitive 2N-th root)."""
    assert (q - 1) % (2 * N) == 0
    for g in range(2, q):
        psi = pow(g, (q - 1) // (2 * N), q)
        if pow(psi, N, q) == q - 1:
            return psi
    raise ValueError("no primitive root")


def round_half_away(x) -> int:
    """Round a float (exactly, via its rational value) to the nearest integer, halves away from 0."""
    f = Fraction(x)
    a = abs(f)
    n = a.numerator // a.denominator
    if a - n >= Fraction(1, 2):
        n += 1
    return n if f >= 0 else -n


@dataclass
class Params:
    logN: int
    L: int
    b: int                 # log2 of the base scale
    q: List[int]           # q_0 .. q_L
    P: List[int]           # special primes p_1 .. p_alpha (P = their product)
    scales: List[float]    # canonical scale at depth 0..L

    @property
    def alpha(self) -> int:
        """Digit-group size of the key switch (one special prime per group member)."""
        return len(self.P)

    @property
    def N(self) -> int:
        return 1 << self.logN

    @property
    def slots(self) -> int:
        return self.N // 2

    def limbs_at_depth(self, d: int) -> int:
        return self.L + 1 - d

    def q_dropped_at_depth(self, d: int) -> int:
        """Prime removed by the rescale that takes depth d to d+1."""
        return self.q[self.L - d]

    @property
    def P_prod(self) -> int:
        out = 1
        for p in self.P:
            out *= p
        return out


def digit_groups(l: int, alpha: int) -> List[List[int]]:
    """Limb indices of the key-switching digit groups of a ciphertext with l limbs: {0 .. alpha-2},
    then runs of alpha consecutive limbs, cut at l."""
    out = [list(range(0, min(alpha - 1, l)))] if l >= 1 else []
    i = alpha - 1
    while i < l:
        out.append(list(range(i, min(i + alpha, l))))
        i += alpha
    return out


def largest_ntt_prime_below(bits: int, N: int, skip: int = 0) -> int:
    """Largest prime below 2^bits that is 1 mod 2N (skip: how many such primes to pass over)."""
    M = 2 * N
    c = ((1 << bits) - 1) // M * M + 1
    while True:
        if c < (1 << bits) and is_prime(c):
            if skip == 0:
                return c
            skip -= 1
        c -= M


DEFAULT_ALPHA = 3   # digit-group size of the key switch when none is given


def make_params(logN: int, L: int, b: int, alpha: int = DEFAULT_ALPHA) -> Params:
    """The prime-chain rule stated in the module docstring; alpha (2..8) special primes."""
    if not 2 <= alpha <= 8:
        raise ValueError("alpha must be in [2, 8]")
    N = 1 << logN
    M = 2 * N
    q0 = largest_ntt_prime_below(60, N)
    # pool: the 4L primes that are 1 mod 2N nearest to 2^b
    center = 1 << b
    pool: List[int] = []
    lo = (center // M) * M + 1
    if lo > center:
        lo -= M
    hi = lo + M
    while len(pool) < 4 * L:
        # candidates at lo (below or at centre) and hi (above), nearest first
        dl, dh = center - lo, hi - center
        if dl <= dh:
            if lo > 1 and is_prime(lo):
                pool.append(lo)
            lo -= M
        else:
            if is_prime(hi):
                pool.append(hi)
            hi += M
    scales = [float(center)]
    chain = [0] * (L + 1)
    chain[0] = q0
    used = set()
    for d in range(L):
        s = scales[d]
        target = Fraction(s * s / float(center))
        best = None
        for p in sorted(pool):
            if p in used:
                continue
            dist = abs(Fraction(p) - target)
            if best is None or dist < best[0]:
                best = (dist, p)
        p = best[1]
        used.add(p)
        chain[L - d] = p
        scales.append((s * s) / float(p))
    special: List[int] = []
    skip = 0
    while len(special) < alpha:
        p = largest_ntt_prime_below(41, N, skip)
        skip += 1
        if p not in chain:
            special.append(p)
    return Params(logN=logN, L=L, b=b, q=chain, P=special, scales=scales)


# --------------------------------------------------------------------------
# encoding (canonical embedding, FP64)
# --------------------------------------------------------------------------

def slot_exponents(N: int) -> np.ndarray:
    """e_j = 5^j mod 2N for slots j < N/2."""
    e = np.empty(N // 2, dtype=np.int64)
    x = 1
    for j in range(N // 2):
        e[j] = x
        x = x * 5 % (2 * N)
    return e


def encode_real_poly(z: np.ndarray, N: int) -> np.ndarray:
    """Real polynomial m with m(zeta^(5^j)) = z_j, m(zeta^(-5^j)) = conj(z_j) (no scaling, FP64).

    m_i = (1/N) sum over odd e of v_e zeta^(-i e); with e = 2k + 1 this is
    zeta^(-i) * fft(v')_i / N where v'_k = v_(2k+1) (numpy's fft has the minus sign).
    """
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (N // 2,)
    e = slot_exponents(N)
    v = np.zeros(N, dtype=np.complex128)
    v[(e - 1) // 2] = z
    v[(2 * N - e - 1) // 2] = np.conj(z)
    w = np.fft.fft(v) / N
    i = np.arange(N)
    m = w * np.exp(-1j * np.pi * i / N)
    return m.real


def encode(z: np.ndarray, N: int, scale: float) -> np.ndarray:
    """Integer plaintext round(scale * sigma^-1(z)) as int64 coefficients."""
    m = encode_real_poly(np.asarray(z, dtype=np.complex128) * scale, N)
    r = np.rint(m)
    if np.max(np.abs(r)) >= 2.0 ** 62:
        raise OverflowError("plaintext coefficient too large")
    return r.astype(np.int64)


def decode_poly(m: np.ndarray, N: int) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) of a real polynomial m (FP64)."""
    m = np.asarray(m, dtype=np.float64)
    i = np.arange(N)
    t = m * np.exp(1j * np.pi * i / N)
    v = np.fft.ifft(t) * N   # v_k = sum_i m_i zeta^(i (2k+1))
    e = slot_exponents(N)
    return v[(e - 1) // 2]


def _decimal_pi(prec: int) -> Decimal:
    getcontext().prec = prec + 10
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(x: int) -> Decimal:
        x2 = x * x
        term = Decimal(1) / x
        total = term
        k = 1
        eps = Decimal(10) ** (-(prec + 5))
        while abs(term) > eps:
            term /= -x2
            total += term / (2 * k + 1)
            k += 1
        return total
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def _decimal_cos(x: Decimal, prec: int) -> Decimal:
    getcontext().prec = prec + 10
    total = Decimal(1)
    term = Decimal(1)
    k = 0
    eps = Decimal(10) ** (-(prec + 5))
    while abs(term) > eps:
        term *= -x * x / ((2 * k + 1) * (2 * k + 2))
        total += term
        k += 1
    return total


def mask_block_start_poly(N: int, R: int, scale: float) -> np.ndarray:
    """Exact integer encoding of the block-start mask (1 at slots j = 0 mod R).

    The mask is R-periodic, so it lives in the subring spanned by X^(c N / (2R));
    its coefficient at X^(c N/(2R)) is cos(pi c / (2R)) / R (c = 0..2R-1), computed
    here to 50 digits, times the scale, rounded half away from zero.
    """
    out = np.zeros(N, dtype=np.int64)
    stride = N // (2 * R)
    pi = _decimal_pi(50)
    sc = Decimal(Fraction(scale).numerator) / Decimal(Fraction(scale).denominator)
    for c in range(2 * R):
        v = sc * _decimal_cos(pi * c / (2 * R), 50) / R
        a = abs(v)
        n = int(a)
        if a - n >= Decimal("0.5"):
            n += 1
        out[c * stride] = n if v >= 0 else -n
    return out


def automorph_poly(a: np.ndarray, g: int) -> np.ndarray:
    """X -> X^g on a signed integer polynomial: coefficient t moves to t g mod 2N, negated past N."""
    N = len(a)
    out = np.zeros(N, dtype=np.int64)
    idx = (np.arange(N, dtype=np.int64) * g) % (2 * N)
    pos = idx < N
    out[idx[pos]] = a[pos]
    out[idx[~pos] - N] = -a[~pos]
    return out


def slot_class_indicator_poly(N: int, R: int, i: int, scale: float) -> np.ndarray:
    """Exact integer encoding of 1 at the slots j = i mod R: the block-start mask rotated right by i, i.e.
    the automorphism X -> X^(5^-i) of mask_block_start_poly (a signed permutation of its coefficients)."""
    return automorph_poly(mask_block_start_poly(N, R, scale), galois_rotate(N, -i))


# --------------------------------------------------------------------------
# keys and ciphertexts
# --------------------------------------------------------------------------

def galois_rotate(N: int, r: int) -> int:
    """Galois element of a left rotation by r slots: 5^r mod 2N (r may be negative)."""
    M = 2 * N
    if r >= 0:
        return pow(5, r, M)
    return pow(pow(5, -r, M), -1, M)


def galois_conj(N: int) -> int:
    return 2 * N - 1


SID_SECRET = 1
SECRET_HW = 64   # Hamming weight h of the secret (KeyGen samples s from HWT(h); h is not given, 64 here)
SID_PK_A = 2
SID_PK_E = 3


def secret_weight(N: int) -> int:
    """h = min(64, N / 2)."""
    return min(SECRET_HW, N // 2)


def ksk_sid_base(K: int) -> int:
    """Stream base of the switching key with key id K (0: relinearisation, else the Galois element)."""
    return (1 << 40) | (K << 20)


@dataclass
class Ct:
    data: np.ndarray   # uint64 [2][l][N], coefficient form
    depth: int
    scale: float

    @property
    def limbs(self) -> int:
        return self.data.shape[1]

    def copy(self) -> "Ct":
        return Ct(self.data.copy(), self.depth, self.scale)


class Oracle:
    """Scheme-level oracle: keys, encryption and the evaluation operations."""

    def __init__(self, params: Params):
        self.p = params
        N = params.N
        self.mods = list(params.q) + list(params.P)
        self.pidx = params.L + 1          # modulus index of p_1 (the other special primes follow)
        self.alpha = params.alpha
        self.ng = len(digit_groups(params.L + 1, self.alpha))
        qs = np.array(self.mods, dtype=np.uint64)
        psis = np.array([primitive_2n_root(q, N) for q in self.mods], dtype=np.uint64)
        self._ctx = lib().ref_ctx_new(N, len(self.mods), _p(qs), _p(psis))
        self.sk: Optional[np.ndarray] = None
        self.pk: Optional[np.ndarray] = None
        self.keys: Dict[int, np.ndarray] = {}      # coefficient form [2][groups][L+1+alpha][N]
        self._kev: Dict[int, np.ndarray] = {}      # oracle evaluation form
        self.n_keyswitch = 0

    def __del__(self):
        try:
            lib().ref_ctx_free(self._ctx)
        except Exception:
            pass

    # ---------------- key generation ----------------
    def keygen(self, seed: int, galois: Sequence[int], relin: bool = True, max_limbs: Optional[int] = None,
               key_limbs: Optional[Dict[int, int]] = None) -> None:
        """Keys of the scheme.  max_limbs restricts the switching keys to the digits and targets a
        ciphertext of at most that many limbs uses (the entries are the same as in the full key);
        key_limbs overrides that limit per key id (0: relinearisation, else the Galois element)."""
        p = self.p
        self._max_l = p.L + 1 if max_limbs is None else int(max_limbs)
        self._key_l: Dict[int, int] = {}
        self._key_limbs = dict(key_limbs or {})
        N, L = p.N, p.L
        s = np.zeros(N, dtype=np.int64)
        lib().ref_sample_hwt(seed, SID_SECRET, N, secret_weight(N), _p(s))
        self.sk = s
        pk = np.zeros((2, L + 1, N), dtype=np.uint64)
        lib().ref_gen_pk(self._ctx, L, _p(s), seed, SID_PK_A, SID_PK_E, _p(pk))
        self.pk = pk
        self._seed = seed
        if relin:
            sp = np.zeros((L + 1, N), dtype=np.uint64)
            lib().ref_secret_square(self._ctx, L + 1, _p(s), _p(sp))
            self._add_key(0, sp)
        for g in galois:
            self._add_key(int(g), self._secret_residues(self._automorph_signed(s, g)))

    def _secret_residues(self, poly: np.ndarray) -> np.ndarray:
        return np.stack([np.mod(poly, q).astype(np.uint64) for q in self.p.q]).astype(np.uint64)

    def _automorph_signed(self, a: np.ndarray, g: int) -> np.ndarray:
        N = self.p.N
        out = np.zeros(N, dtype=np.int64)
        idx = (np.arange(N, dtype=np.int64) * g) % (2 * N)
        pos = idx < N
        out[idx[pos]] = a[pos]
        out[idx[~pos] - N] = -a[~pos]
        return out

    def _add_key(self, K: int, sp: np.ndarray) -> None:
        p = self.p
        N, L = p.N, p.L
        ml = min(p.L + 1, int(self._key_limbs.get(K, self._max_l)))
        # np.zeros maps untouched pages lazily, so a key restricted to a few limbs holds only those entries
        key = np.zeros((2, self.ng, L + 1 + self.alpha, N), dtype=np.uint64)
        lib().ref_gen_ksk(self._ctx, L, self.alpha, _p(self.sk), _p(np.ascontiguousarray(sp)), self._seed,
                          ksk_sid_base(K), ml, _p(key))
        kev = np.zeros(key.shape, dtype=np.uint64)
        lib().ref_key_to_eval(self._ctx, L, self.alpha, ml, _p(key), _p(kev))
        self.keys[K] = key
        self._kev[K] = kev
        self._key_l[K] = ml

    # ---------------- encryption ----------------
    def encrypt(self, m: np.ndarray, depth: int, scale: float, seed: int) -> Ct:
        p = self.p
        l = p.limbs_at_depth(depth)
        ct = np.zeros((2, l, p.N), dtype=np.uint64)
        m = np.ascontiguousarray(m, dtype=np.int64)
        lib().ref_encrypt(self._ctx, p.L + 1, _p(self.pk), l, _p(m), seed, _p(ct))
        return Ct(ct, depth, scale)

    def decrypt_poly(self, ct: Ct) -> List[int]:
        """Centred integer coefficients of c0 + c1 s mod Q_l (exact CRT with Python integers)."""
        p = self.p
        l = ct.limbs
        m = np.zeros((l, p.N), dtype=np.uint64)
        lib().ref_decrypt(self._ctx, l, _p(np.ascontiguousarray(ct.data)), _p(self.sk), _p(m))
        Q = 1
        for i in range(l):
            Q *= p.q[i]
        res = [0] * p.N
        coeffs = [0] * p.N
        for i in range(l):
            qi = p.q[i]
            Mi = Q // qi
            yi = Mi * pow(Mi, -1, qi) % Q
            col = m[i].tolist()
            for k in range(p.N):
                coeffs[k] += col[k] * yi
        for k in range(p.N):
            v = coeffs[k] % Q
            res[k] = v - Q if v > Q // 2 else v
        return res

    def decrypt(self, ct: Ct) -> np.ndarray:
        m = self.decrypt_poly(ct)
        mf = np.array([float(Fraction(v) / Fraction(ct.scale)) for v in m], dtype=np.float64)
        return decode_poly(mf, self.p.N)

    # ---------------- evaluation ----------------
    def _check_same(self, a: Ct, b: Ct) -> None:
        if a.depth != b.depth or a.scale != b.scale:
            raise ValueError("operands differ in depth (%d, %d) or scale (%r, %r)" % (a.depth, b.depth, a.scale, b.scale))

    def add(self, a: Ct, b: Ct) -> Ct:
        self._check_same(a, b)
        out = np.empty_like(a.data)
        lib().ref_add(self._ctx, 2, a.limbs, _p(a.data), _p(b.data), _p(out))
        return Ct(out, a.depth, a.scale)

    def sub(self, a: Ct, b: Ct) -> Ct:
        self._check_same(a, b)
        out = np.empty_like(a.data)
        lib().ref_sub(self._ctx, 2, a.limbs, _p(a.data), _p(b.data), _p(out))
        return Ct(out, a.depth, a.scale)

    def neg(self, a: Ct) -> Ct:
        return self.mul_int(a, -1)

    def mul_int(self, a: Ct, k: int) -> Ct:
        out = np.empty_like(a.data)
        lib().ref_mul_int(self._ctx, 2, a.limbs, _p(a.data), int(k), _p(out))
        return Ct(out, a.depth, a.scale)

    def add_const(self, a: Ct, c: float) -> Ct:
        out = a.data.copy()
        lib().ref_add_const(self._ctx, a.limbs, _p(out), round_half_away(c * a.scale))
        return Ct(out, a.depth, a.scale)

    def rescale(self, a: Ct) -> Ct:
        l = a.limbs
        out = np.empty((2, l - 1, self.p.N), dtype=np.uint64)
        lib().ref_rescale(self._ctx, 2, l, _p(a.data), _p(out))
        return Ct(out, a.depth + 1, a.scale)

    def mod_drop(self, a: Ct, depth: int) -> Ct:
        l = self.p.limbs_at_depth(depth)
        return Ct(np.ascontiguousarray(a.data[:, :l, :]), depth, a.scale)

    def mul_const(self, a: Ct, c: float) -> Ct:
        """Multiply by the real c encoded at the ciphertext's own scale s: integer
        round_half_away(c * s), then rescale by q; the result scale is (s * s) / q."""
        q = self.p.q_dropped_at_depth(a.depth)
        t = self.mul_int(a, round_half_away(c * a.scale))
        r = self.rescale(t)
        r.scale = (a.scale * a.scale) / float(q)
        return r

    def add_plain(self, a: Ct, pt: np.ndarray) -> Ct:
        """Add a signed integer plaintext polynomial (already at a's scale) to c0."""
        out = a.data.copy()
        for i in range(a.limbs):
            q = int(self.p.q[i])
            out[0, i] = (out[0, i] + np.mod(pt, q).astype(np.uint64)) % np.uint64(q)
        return Ct(out, a.depth, a.scale)

    def mul_mask(self, a: Ct, R: int) -> Ct:
        """Multiply by the block-start mask (1 at slots = 0 mod R) encoded at the ciphertext's
        scale s, then rescale; the result scale is (s * s) / q."""
        q = self.p.q_dropped_at_depth(a.depth)
        pt = mask_block_start_poly(self.p.N, R, a.scale)
        out = np.empty_like(a.data)
        lib().ref_mul_plain(self._ctx, 2, a.limbs, _p(a.data), _p(pt), _p(out))
        r = self.rescale(Ct(out, a.depth, a.scale))
        r.scale = (a.scale * a.scale) / float(q)
        return r

    def mask_sum(self, terms: Sequence[Tuple[Ct, np.ndarray]]) -> Ct:
        """sum_i a_i pt_i for integer plaintext polynomials pt_i (masks already encoded at the operands'
        common scale s), then one rescale by q; the result scale is (s * s) / q, as for mul_mask."""
        a0 = terms[0][0]
        q = self.p.q_dropped_at_depth(a0.depth)
        acc = None
        for a, pt in terms:
            self._check_same(a, a0)
            out = np.empty_like(a.data)
            lib().ref_mul_plain(self._ctx, 2, a.limbs, _p(a.data), _p(np.ascontiguousarray(pt, dtype=np.int64)),
                                _p(out))
            t = Ct(out, a.depth, a.scale)
            acc = t if acc is None else self.add(acc, t)
        r = self.rescale(acc)
        r.scale = (a0.scale * a0.scale) / float(q)
        return r

    def align(self, a: Ct, depth: int, scale: float, factor: float = 1.0) -> Ct:
        """Bring a to (depth, scale), multiplying its value by `factor`: mod-drop to depth-1,
        multiply by the integer round_half_away(((scale * factor) * q) / a.scale), rescale by q,
        and declare the scale."""
        if depth == a.depth and scale == a.scale and factor == 1.0:
            return a
        if depth <= a.depth:
            raise ValueError("align needs a deeper target (%d -> %d)" % (a.depth, depth))
        t = self.mod_drop(a, depth - 1)
        q = self.p.q_dropped_at_depth(depth - 1)
        c = round_half_away(((scale * factor) * float(q)) / a.scale)
        t = self.mul_int(t, c)
        r = self.rescale(t)
        r.scale = scale
        return r

    def set_scale(self, a: Ct, factor: float) -> Ct:
        return Ct(a.data, a.depth, a.scale * factor)

    def mul_gauss(self, a: Ct, re: int, im: int) -> Ct:
        """a times the plaintext re + im X^(N/2), a product with no rounding: slot j is the evaluation at
        zeta^(5^j) (zeta = exp(i pi / N)), where X^(N/2) takes the value zeta^(5^j N/2) = i because
        5^j = 1 mod 4, so every slot is multiplied by the Gaussian integer re + im i.  Same depth and scale."""
        N = self.p.N
        pt = np.zeros(N, dtype=np.int64)
        pt[0] = re
        pt[N // 2] = im
        out = np.empty_like(a.data)
        lib().ref_mul_plain(self._ctx, 2, a.limbs, _p(a.data), _p(pt), _p(out))
        return Ct(out, a.depth, a.scale)

    def mul_i(self, a: Ct, neg: bool = False) -> Ct:
        """a times X^(N/2) (or -X^(N/2)): every slot times i (or -i), exactly (see mul_gauss)."""
        return self.mul_gauss(a, 0, -1 if neg else 1)

    def keyswitch(self, d: np.ndarray, K: int) -> np.ndarray:
        """Key switch of d ([l][N], coefficient form) with the key of id K (keyswitch_galois, no automorphism)."""
        return self.keyswitch_galois(d, [(0, K)])

    def keyswitch_galois(self, d: np.ndarray, pairs: Sequence[Tuple[int, int]]) -> np.ndarray:
        """(x - C) / P for x = sum_i sum_b sigma_{g_i}(D_b) * ksk_{K_i, b}, pairs (g_i, K_i); d is [l][N].

        One decomposition of d (the digits D_b of the module docstring) serves every key: each digit
        is taken modulo the target moduli first and then permuted by its automorphism (g = 0: none),
        and all products are summed before the single division by P."""
        l = d.shape[0]
        for _, K in pairs:
            if l > self._key_l[K]:
                raise ValueError("key %d was generated for at most %d limbs" % (K, self._key_l[K]))
        p = self.p
        out = np.zeros((2, l, p.N), dtype=np.uint64)
        gal = np.array([g for g, _ in pairs], dtype=np.uint64)
        kevs = (_u64p * len(pairs))(*[_p(self._kev[K]) for _, K in pairs])
        lib().ref_keyswitch(self._ctx, p.L, self.alpha, l, _p(np.ascontiguousarray(d)), len(pairs), _p(gal), kevs,
                            self.ng,
                            _p(out))
        self.n_keyswitch += 1
        return out

    def tensor(self, pairs: Sequence[Tuple[Ct, Ct]]) -> np.ndarray:
        a0, b0 = pairs[0]
        l = a0.limbs
        out = np.zeros((3, l, self.p.N), dtype=np.uint64)
        for i, (a, b) in enumerate(pairs):
            if a.depth != a0.depth or b.depth != a0.depth:
                raise ValueError("tensor operands at different depths")
            lib().ref_tensor(self._ctx, l, _p(a.data), _p(b.data), _p(out), 1 if i else 0)
        return out

    def relinearize(self, d: np.ndarray, depth: int, scale: float) -> Ct:
        ks = self.keyswitch(d[2], 0)
        out = np.empty((2, d.shape[1], self.p.N), dtype=np.uint64)
        lib().ref_add(self._ctx, 2, d.shape[1], _p(np.ascontiguousarray(d[:2])), _p(ks), _p(out))
        return Ct(out, depth, scale)

    def relin_rescale(self, d: np.ndarray, depth: int) -> Ct:
        """(d0, d1) + KS(d2) with the relinearisation key, rescaled by q_{l-1} in the same division: one
        division of x + P (d0, d1) by P q_{l-1} (ref_keyswitch_rescale).  The result is one level deeper;
        the caller sets its scale."""
        l = d.shape[1]
        if l > self._key_l[0]:
            raise ValueError("relinearisation key was generated for at most %d limbs" % self._key_l[0])
        if l < 2:
            raise ValueError("no limb left to rescale")
        p = self.p
        out = np.zeros((2, l - 1, p.N), dtype=np.uint64)
        gal = np.zeros(1, dtype=np.uint64)
        kevs = (_u64p * 1)(_p(self._kev[0]))
        lib().ref_keyswitch_rescale(self._ctx, p.L, self.alpha, l, _p(np.ascontiguousarray(d[2])), 1, _p(gal), kevs,
                                    self.ng, _p(np.ascontiguousarray(d[:2])), _p(out))
        self.n_keyswitch += 1
        return Ct(out, depth + 1, 0.0)

    def mul_sum(self, pairs: Sequence[Tuple[Ct, Ct]]) -> Ct:
        """sum_i a_i * b_i: the tensors summed, then one relinearisation and rescale in a single division by
        P q_{l-1} (relin_rescale); all pairs share depth and product scale."""
        a0, b0 = pairs[0]
        s = a0.scale * b0.scale
        for a, b in pairs:
            if a.scale * b.scale != s:
                raise ValueError("lazy sum of products with different scales")
        d = self.tensor(pairs)
        r = self.relin_rescale(d, a0.depth)
        q = self.p.q_dropped_at_depth(a0.depth)
        r.scale = (a0.scale * b0.scale) / float(q)
        return r

    def mul(self, a: Ct, b: Ct) -> Ct:
        return self.mul_sum([(a, b)])

    def automorph(self, a: Ct, g: int) -> Ct:
        out = np.empty_like(a.data)
        lib().ref_automorph(self._ctx, 2, a.limbs, _p(a.data), g, _p(out))
        return Ct(out, a.depth, a.scale)

    def apply_galois(self, a: Ct, g: int) -> Ct:
        """The automorphism X -> X^g switched back to s (Rotate / conjugate): c0 is permuted, and the
        key switch of sigma_g(c1) permutes the lifted digits of c1 (keyswitch_galois)."""
        c0 = self.automorph(a, g).data[0]
        ks = self.keyswitch_galois(a.data[1], [(g, g)])
        out = np.empty((1, a.limbs, self.p.N), dtype=np.uint64)
        lib().ref_add(self._ctx, 1, a.limbs, _p(np.ascontiguousarray(c0)), _p(np.ascontiguousarray(ks[0])), _p(out))
        return Ct(np.ascontiguousarray(np.stack([out[0], ks[1]])), a.depth, a.scale)

    def rotate_sum(self, a: Ct, rots: Sequence[int]) -> Ct:
        """a + sum_i Rot(a, r_i) with one key switch: the rotations share the decomposition of c1 and
        the division by P (keyswitch_galois over all of them)."""
        N, l = self.p.N, a.limbs
        gs = [galois_rotate(N, r) for r in rots]
        ks = self.keyswitch_galois(a.data[1], [(g, g) for g in gs])
        c0 = np.ascontiguousarray(a.data[0:1])
        for g in gs:
            t = self.automorph(a, g)
            nxt = np.empty_like(c0)
            lib().ref_add(self._ctx, 1, l, _p(c0), _p(np.ascontiguousarray(t.data[0:1])), _p(nxt))
            c0 = nxt
        out = np.empty((2, l, N), dtype=np.uint64)
        lib().ref_add(self._ctx, 1, l, _p(c0), _p(np.ascontiguousarray(ks[0:1])), _p(out[0:1]))
        o1 = np.empty((1, l, N), dtype=np.uint64)
        lib().ref_add(self._ctx, 1, l, _p(np.ascontiguousarray(a.data[1:2])), _p(np.ascontiguousarray(ks[1:2])), _p(o1))
        out[1] = o1[0]
        return Ct(out, a.depth, a.scale)

    def rotate(self, a: Ct, r: int) -> Ct:
        """Slot j of the result holds slot j + r of a."""
        return self.apply_galois(a, galois_rotate(self.p.N, r))

    def conjugate(self, a: Ct) -> Ct:
        return self.apply_galois(a, galois_conj(self.p.N))
