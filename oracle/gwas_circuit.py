"""Encrypted modified semi-parallel GWAS on the CPU oracle — TEST INFRASTRUCTURE ONLY.

Follows Alg. "Semi Parallel GWAS" (with Alg. "Homomorphic LogReg" and
Alg. "inverseSlots") step by step on oracle ciphertexts.  Layouts:

* R = PO2(n) rows per block, B = N / (2R) blocks per ciphertext (N/2 slots).
* Per-sample vectors (covariate columns x_j, y) are R-periodic: slot s holds
  v[s mod R] when s mod R < n, else 0 — a CP column (Methods, "Column-Packed
  Matrices") already duplicated into every block (Alg. Duplicate done by the
  client).  On such data the rotate-and-sum of Alg. DotProd leaves the full dot
  product in every slot.  The rotate-and-sum adds Rot(a, i) for every i < R; it
  is taken as groups a <- a + sum_{0 < j < m} Rot(a, j s) with one shared key
  switch per group (Oracle.rotate_sum), m = min(radix, R / s) and the next group
  starting at shift m s (rotation_groups): radix 8 in the fixed part ({1..7},
  {8, 16, .., 56}, {64, 128, 192} for R = 256) and radix 16 per SNP batch
  ({1..15}, {16, 32, .., 240}).  This sums the same rotations as the log2(R)
  doubling steps of Alg. colSum with fewer key switches.
* Entries of A = (X^T X)^-1 are replicated scalars (the same value in every slot).
* A SNP batch is a CCP matrix (Methods, "Column-Compact-Packed Matrices") with
  two SNPs per complex slot (Methods, "Complex Space of CKKS ciphertext"):
  slot c R + r holds S[r, 2c] + i S[r, 2c+1] of that batch, tau = N / R SNPs per
  ciphertext (eq. numSNPinBatch read as 2 (N/2) / R).

The projection M S = S - X (A (X^T S)) is evaluated through associativity
(eqs. M, Sprime) as S' = S - sum_j x_j (.) bcast(mask (.) colSum(r_j (.) S)) with
r_j = sum_l A_jl x_l, so that M is never materialised.

Depth plan (kappa >= 2; D_p = 7 (kappa - 1)): beta^(1) at 2, each further
Newton pass adds 7 levels (eta, 4 for sigma7, g, beta); w at D_p + 1,
w^-1 at D_p + 5, z at D_p + 6, z' at D_p + 9, u = w z' at D_p + 10; SNP batches
are encrypted at D_S = D_p + 7, S' at D_S + 3, num at D_S + 4 and the two
denominators at D_S + 5 = 7 kappa + 5 = L.

kappa = 1 (Discussion: the SEAL run reduces kappa to 1): the only Newton pass
starts from beta = 0, so the p it leaves for the weights is sigma7(0) = 1/2 and
w = 1/4 and w^-1 = inverseSlots(1/4) = 4 - 2^-14 are public constants.  beta^(1)
at 2, z = X beta + w^-1 (y - 1/2) at 3 (the constant folded into the alignment
of y - 1/2), z' at 6, u = z' / 4 at 7 (the 1/4 folded into an alignment); SNP
batches at D_S = 4, S' at 7, and num and both denominators at 8 = L (the
denominators square S' directly and take w = 1/4 into their tracked scale).
No w or w^-1 ciphertext exists.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import ckks as C
from .gwas_fp64 import (DIV_GUESS, DIV_ITERS, SIGMA7_C1, SIGMA7_C3, SIGMA7_C5, SIGMA7_C7, inverse_slots,
                        snp_normalisers, xtx_inverse)

# kappa = 1: the weights of the only Newton pass are public, w = sigma7(0) (1 - sigma7(0)) = 1/4
W_KAPPA1 = 0.25
W_INV_KAPPA1 = float(inverse_slots(np.array(W_KAPPA1)))   # Alg. inverseSlots at w = 1/4: 4 - 2^-14


def circuit_depth(kappa: int) -> int:
    """Number of rescales (L) the circuit consumes for kappa Newton passes."""
    if kappa < 1:
        raise ValueError("kappa >= 1 Newton passes")
    return 8 if kappa == 1 else 7 * kappa + 5


def snp_depth(kappa: int) -> int:
    """Depth at which the SNP batches are encrypted."""
    if kappa < 1:
        raise ValueError("kappa >= 1 Newton passes")
    return 4 if kappa == 1 else 7 * (kappa - 1) + 7


@dataclass
class Layout:
    N: int
    n: int
    k: int
    m: int
    R: int

    @property
    def blocks(self) -> int:
        return self.N // (2 * self.R)

    @property
    def tau(self) -> int:
        return 2 * self.blocks

    @property
    def n_batches(self) -> int:
        return -(-self.m // self.tau)

    @property
    def log_r(self) -> int:
        return self.R.bit_length() - 1


def make_layout(N: int, n: int, k: int, m: int) -> Layout:
    R = 1
    while R < n:
        R *= 2
    if 2 * R > N:
        raise ValueError("n too large for the ring: need PO2(n) <= N/2")
    return Layout(N=N, n=n, k=k, m=m, R=R)


def periodic_slots(v: np.ndarray, lay: Layout) -> np.ndarray:
    z = np.zeros(lay.N // 2, dtype=np.complex128)
    s = np.arange(lay.N // 2)
    r = s % lay.R
    ok = r < lay.n
    z[ok] = v[r[ok]]
    return z


def snp_batch_slots(S: np.ndarray, lay: Layout, b: int) -> np.ndarray:
    z = np.zeros(lay.N // 2, dtype=np.complex128)
    for c in range(lay.blocks):
        j0 = b * lay.tau + 2 * c
        base = c * lay.R
        if j0 < lay.m:
            z[base:base + lay.n] += S[:, j0].astype(np.float64)
        if j0 + 1 < lay.m:
            z[base:base + lay.n] += 1j * S[:, j0 + 1].astype(np.float64)
    return z


def a_pairs(k: int):
    return [(j, l) for j in range(k) for l in range(j, k)]


def constant_poly(c: float, N: int, scale: float) -> np.ndarray:
    """Exact encoding of a replicated real scalar: round_half_away(c * scale) at X^0."""
    m = np.zeros(N, dtype=np.int64)
    m[0] = C.round_half_away(c * scale)
    return m


@dataclass
class EncInput:
    lay: Layout
    kappa: int
    x: List[C.Ct]
    y: C.Ct
    A: Dict[tuple, C.Ct]
    S: List[C.Ct]

    def a(self, j: int, l: int) -> C.Ct:
        return self.A[(j, l) if j <= l else (l, j)]


@dataclass
class Plaintexts:
    """Integer plaintext polynomials of every input ciphertext, in encryption order."""
    polys: List[np.ndarray]
    depths: List[int]


def encode_inputs(params: C.Params, X: np.ndarray, y: np.ndarray, S: np.ndarray, kappa: int) -> Plaintexts:
    """Client-side encoding (oracle encoder, FP64) of x_j, y, A_jl and the SNP batches."""
    n, k = X.shape
    lay = make_layout(params.N, n, k, S.shape[1])
    A = xtx_inverse(X)
    polys, depths = [], []
    for j in range(k):
        polys.append(C.encode(periodic_slots(X[:, j], lay), params.N, params.scales[0]))
        depths.append(0)
    polys.append(C.encode(periodic_slots(y, lay), params.N, params.scales[0]))
    depths.append(0)
    for (j, l) in a_pairs(k):
        polys.append(constant_poly(A[j, l], params.N, a_scale(params, lay)))
        depths.append(0)
    ds = snp_depth(kappa)
    for b in range(lay.n_batches):
        polys.append(C.encode(snp_batch_slots(S, lay, b), params.N, params.scales[ds]))
        depths.append(ds)
    return Plaintexts(polys=polys, depths=depths)


def a_scale(params: C.Params, lay: Layout) -> float:
    """Entries of (X^T X)^-1 are O(1/n); they are encrypted at depth 0 with scale R * Delta_0 so that
    their integer content stays well above the noise, and reach the canonical scale by alignment."""
    return params.scales[0] * float(lay.R)


def input_seed(enc_seed: int, i: int) -> int:
    """Encryption seed of input ciphertext i: output number i of SplitMix64 seeded with enc_seed."""
    return int(C.lib().ref_splitmix_out(enc_seed, i))


def encrypt_inputs(o: C.Oracle, pts: Plaintexts, n: int, k: int, m: int, kappa: int, enc_seed: int) -> EncInput:
    p = o.p
    lay = make_layout(p.N, n, k, m)
    scales = [p.scales[d] for d in pts.depths]
    for i in range(k + 1, k + 1 + len(a_pairs(k))):
        scales[i] = a_scale(p, lay)
    cts = [o.encrypt(pt, d, s, input_seed(enc_seed, i)) for i, (pt, d, s) in enumerate(zip(pts.polys, pts.depths, scales))]
    x = cts[:k]
    yc = cts[k]
    pairs = a_pairs(k)
    A = {pr: cts[k + 1 + i] for i, pr in enumerate(pairs)}
    S = cts[k + 1 + len(pairs):]
    return EncInput(lay=lay, kappa=kappa, x=x, y=yc, A=A, S=S)


# Rotations per shared key switch: up to FIXED_RADIX - 1 in the fixed part (one to a few ciphertexts per
# call) and up to BATCH_RADIX - 1 in the per-SNP-batch part.
FIXED_RADIX = 8
BATCH_RADIX = 16


def rotation_groups(R: int, radix: int = FIXED_RADIX) -> List[List[int]]:
    """The left rotations of a rotate-and-sum over R = 2^r slots, grouped by shared key switch.

    Alg. colSum doubles its partial sums: a <- a + Rot(a, s) for s = 1, 2, 4, .., R/2.  A group merges
    log2(m) consecutive doublings starting at shift s into one step a <- a + sum_{0 < j < m} Rot(a, j s),
    since (1 + X^s)(1 + X^2s)..(1 + X^(m/2) s) = sum_{j < m} X^(j s); here m = min(radix, R / s) and the
    next group starts at shift m s.  Radix 4 gives {s, 2s, 3s} for s = 1, 4, 16, .. and a last {s} when
    r is odd."""
    out = []
    s = 1
    while s < R:
        m = min(radix, R // s)
        out.append([j * s for j in range(1, m)])
        s *= m
    return out


def diag_width(lay: Layout) -> int:
    """K of the packed projection (reading 21), or 0 where it does not apply: K is the smallest power of two
    >= k for k >= 2; it must divide m = min(BATCH_RADIX, R), the size of the first rotation group, and
    n + K - 1 <= R must hold, so that the rows which the products and the stride sums wrap onto are padding
    rows (zero in x_j, r_j and S)."""
    k, R = lay.k, lay.R
    if k < 2:
        return 0
    K = 1
    while K < k:
        K *= 2
    m = min(BATCH_RADIX, R)
    if K > m or m % K or lay.n + K - 1 > R:
        return 0
    return K


def stride_groups(R: int, K: int, radix: int = BATCH_RADIX) -> List[List[int]]:
    """The left rotations of sum_{u < R/K} Rot(a, K u), grouped by shared key switch: the multiples of K in
    the first group of rotation_groups(R, radix) (dropped when there are none), then its other groups
    unchanged.  Since sum_{j < m} X^j factors into the groups of rotation_groups, keeping only the multiples
    of K in the first factor (K divides its size m) leaves the sum over the multiples of K below R.  Every
    rotation is one of rotation_groups(R, radix), so no other key is needed."""
    g = rotation_groups(R, radix)
    head = [r for r in g[0] if r % K == 0]
    return ([head] if head else []) + g[1:]


def required_galois(N: int, R: int) -> List[int]:
    """Galois elements of the left and right rotations of rotation_groups(R, FIXED_RADIX) and
    rotation_groups(R, BATCH_RADIX), each once in first-seen order, then conjugation."""
    out: List[int] = []
    for radix in (FIXED_RADIX, BATCH_RADIX):
        for grp in rotation_groups(R, radix):
            for r in grp:
                for e in (C.galois_rotate(N, r), C.galois_rotate(N, -r)):
                    if e not in out:
                        out.append(e)
    e = C.galois_conj(N)
    if e not in out:
        out.append(e)
    return out


@dataclass
class FixedPart:
    """What the per-batch part needs from the fixed part: x_j, r_j = (X A)_{:, j}, w and u = w z'
    (w is None when it is the public 1/4 of kappa = 1); for the packed projection (reading 21) the
    diagonals Rot(Z_t, -t) at the SNP depth and X_t at the SNP depth + 2, t < K (else None)."""
    x: List[C.Ct]
    rr: List[C.Ct]
    w: Optional[C.Ct]
    u: C.Ct
    zt: Optional[List[C.Ct]] = None
    xt: Optional[List[C.Ct]] = None


@dataclass
class EncOutput:
    beta: List[C.Ct]
    w: Optional[C.Ct]        # None for kappa = 1 (public)
    w_inv: Optional[C.Ct]    # None for kappa = 1 (public)
    z_proj: C.Ct
    u: C.Ct
    S_proj: List[C.Ct]
    num: List[C.Ct]
    den_even: List[C.Ct]
    den_odd: List[C.Ct]
    m_cols: Optional[List[C.Ct]] = None   # M-materialised layout: Dup(M_i), i < n


class Circuit:
    def __init__(self, o: C.Oracle, lay: Layout, m_in: Optional["MInput"] = None):
        """m_in: the client's inputs of the M-materialised layout (then S' = M S by CP-REP-MatMult and the
        CCP SNP batches of the input are not used)."""
        self.o = o
        self.lay = lay
        self.sc = o.p.scales
        self.m_in = m_in

    # canonical-scale helpers
    def at(self, a: C.Ct, d: int, factor: float = 1.0) -> C.Ct:
        """a brought to depth d at the canonical scale; factor scales the value (exact powers of two)."""
        if d == a.depth and factor == 1.0:
            return a
        return self.o.align(a, d, self.sc[d], factor)

    def rot_sum(self, a: C.Ct, radix: int = FIXED_RADIX) -> C.Ct:
        """sum_{i < R} Rot(a, i) (Alg. colSum / Alg. DotProd), by the groups of rotation_groups(R, radix)."""
        for grp in rotation_groups(self.lay.R, radix):
            a = self.o.rotate_sum(a, grp)
        return a

    def bcast(self, a: C.Ct, radix: int = FIXED_RADIX) -> C.Ct:
        """sum_{i < R} Rot(a, -i): copies each block's first slot over its block."""
        for grp in rotation_groups(self.lay.R, radix):
            a = self.o.rotate_sum(a, [-r for r in grp])
        return a

    def sigma7(self, u: C.Ct) -> C.Ct:
        """sigma7 for u = eta / 8 at canonical scale; 4 levels (eq. sigma7, sign-corrected)."""
        o = self.o
        d = u.depth
        u2 = o.mul(u, u)
        a1 = o.add_const(o.mul_const(u2, -SIGMA7_C3), SIGMA7_C1)
        a2 = o.add_const(o.mul_const(u2, -SIGMA7_C7), SIGMA7_C5)
        u4 = o.mul(u2, u2)
        b = o.mul(u4, a2)
        cc = o.add(self.at(a1, d + 3), b)
        return o.add_const(o.mul(self.at(u, d + 3), cc), 0.5)

    def diagonals(self, inp: EncInput, rr: List[C.Ct], ds: int, K: int):
        """The packed projection's diagonals (reading 21): with comb_c the mask of the slots s = c mod K,
        Z_t = sum_j comb_{(j - t) mod K} r_j and X_t = sum_j comb_{(j - t) mod K} x_j (slot s of block row r
        holds r_{(r + t) mod K}[r], or 0 where (r + t) mod K >= k), each one mask_sum of the r_j brought to
        depth ds - 1 and of the x_j brought to ds + 1, so that Z_t lands at the SNP depth ds and X_t at ds + 2
        with their canonical scales (the mask product's s^2 / q is the next depth's canonical scale); Z_t is
        then rotated right by t."""
        o = self.o
        N = self.lay.N
        k = self.lay.k
        ra = [self.at(rr[j], ds - 1) for j in range(k)]
        xa = [self.at(inp.x[j], ds + 1) for j in range(k)]
        zt, xt = [], []
        for t in range(K):
            z = o.mask_sum([(ra[j], C.slot_class_indicator_poly(N, K, (j - t) % K, ra[j].scale)) for j in range(k)])
            assert z.depth == ds and z.scale == self.sc[ds]
            zt.append(o.rotate(z, -t) if t else z)
            xm = o.mask_sum([(xa[j], C.slot_class_indicator_poly(N, K, (j - t) % K, xa[j].scale)) for j in range(k)])
            assert xm.depth == ds + 2 and xm.scale == self.sc[ds + 2]
            xt.append(xm)
        return zt, xt

    def project_diag(self, S: C.Ct, fx: "FixedPart") -> C.Ct:
        """S' = S - sum_j x_j (.) E_j by the packed projection (reading 21):
        D = sum_t Rot(Z_t, -t) (.) Rot(S, -t) = sum_t Rot(Z_t (.) S, -t) (one lazily summed product),
        W = sum_{u < R/K} Rot(D, K u), whose slot j < k of each block is C_j = colSum(r_j (.) S),
        Mk = W times the mask of the first k slots of each block,
        V = sum_{u < R/K} Rot(Mk, -K u), which holds C_{r mod K} at block row r,
        x E = sum_t X_t (.) Rot(V, t) (one lazily summed product)."""
        o = self.o
        lay = self.lay
        K = len(fx.zt)
        pairs = [(fx.zt[0], S)] + [(fx.zt[t], o.rotate(S, -t)) for t in range(1, K)]
        w = o.mul_sum(pairs)
        for grp in stride_groups(lay.R, K):
            w = o.rotate_sum(w, grp)
        mk = o.mask_sum([(w, sum(C.slot_class_indicator_poly(lay.N, lay.R, j, w.scale) for j in range(lay.k)))])
        v = mk
        for grp in stride_groups(lay.R, K):
            v = o.rotate_sum(v, [-r for r in grp])
        xe = o.mul_sum([(fx.xt[0], v)] + [(fx.xt[t], o.rotate(v, t)) for t in range(1, K)])
        return o.sub(self.at(S, xe.depth), xe)

    def run_batch(self, S: C.Ct, fx: "FixedPart"):
        """Per-batch part (Alg. Semi Parallel GWAS, batch loop): S' = M S, num, denEven, denOdd."""
        if fx.zt is not None:
            sp = self.project_diag(S, fx)
            return (sp,) + self.num_den(sp, fx)
        o = self.o
        k = self.lay.k
        ds = S.depth
        cs = []
        for j in range(k):
            pj = o.mul(self.at(fx.rr[j], ds), S)
            cj = self.rot_sum(pj, BATCH_RADIX)    # column sums at block starts (Alg. colSum)
            cj = o.mul_mask(cj, self.lay.R)       # keep block starts only
            cs.append(self.bcast(cj, BATCH_RADIX))   # (A X^T S)_{j, c} over block c
        dc = cs[0].depth
        xe = o.mul_sum([(self.at(fx.x[j], dc), cs[j]) for j in range(k)])
        sp = o.sub(self.at(S, xe.depth), xe)
        return (sp,) + self.num_den(sp, fx)

    def num_den(self, sp: C.Ct, fx: "FixedPart"):
        """numerator and both denominators of a projected batch S' (Alg. Semi Parallel GWAS).  With
        S' = a + i b per slot (the even SNP in a, the odd one in b) the denominators are sum w a^2 and
        sum w b^2.  Both come from one rotate-and-sum of W = 4 w (a^2 + i b^2) = w T with
        T = (2 + 2i) S' conj(S') + (1 - i) (S'^2 + conj(S')^2) (one lazily summed product, the Gaussian
        integer factors as exact products with re + im X^(N/2)); den_even = sum W / 4 and
        den_odd = -i sum W / 4, whose real parts are the two denominators (reading 20)."""
        o = self.o
        dsp = sp.depth
        num = self.rot_sum(o.mul(self.at(fx.u, dsp), sp), BATCH_RADIX)
        sc = o.conjugate(sp)
        t = o.mul_sum([(o.mul_gauss(sp, 2, 2), sc), (o.mul_gauss(sp, 1, -1), sp), (o.mul_gauss(sc, 1, -1), sc)])
        if fx.w is None:
            w4 = t                        # public w = 1/4, in the tracked scale
            factor = 4.0 / W_KAPPA1
        else:
            w4 = o.mul(self.at(fx.w, t.depth), t)
            factor = 4.0
        de = self.rot_sum(o.set_scale(w4, factor), BATCH_RADIX)
        do = o.mul_i(de, neg=True)
        return num, de, do

    # ---- the M-materialised layout (paper: Alg. CP-REP-MatMult; the walk-through of Alg. Semi Parallel
    #      GWAS: M as a CP matrix, S' = M S_i by CP-REP-MatMult with S_i in REP form)
    def m_columns(self, inp: EncInput, rr: List[C.Ct], m_in: "MInput") -> List[C.Ct]:
        """Dup(M_i) = Dup(e_i) - sum_j r_j X_ij for every sample i: column i of M = I - X A X^T duplicated
        over the ciphertext (CP), by CP-REP-MatMult of X A (columns r_j) with X^T in REP form (entry X_ij
        replicated over every slot); the identity column is the exact indicator of the slots = i mod R."""
        o = self.o
        k = self.lay.k
        dx = m_in.Xrep[0][0].depth
        rx = [self.at(r, dx) for r in rr]          # r_j brought to the REP X^T's depth once
        out = []
        for i in range(self.lay.n):
            g = o.mul_sum([(rx[j], m_in.Xrep[i][j]) for j in range(k)])
            e = C.slot_class_indicator_poly(self.lay.N, self.lay.R, i, g.scale)
            out.append(o.add_plain(o.neg(g), e))
        return out

    def project_m(self, cols: List[C.Ct], S_rep: List[C.Ct]) -> C.Ct:
        """S' = M S_b = sum_i Dup(M_i) (.) S_rep(i) (Alg. CP-REP-MatMult): n products in one lazy sum."""
        return self.o.mul_sum([(self.at(cols[i], S_rep[i].depth), S_rep[i]) for i in range(self.lay.n)])

    def _project_z(self, inp: EncInput, z: C.Ct) -> C.Ct:
        """z' = M z = z - X (A (X^T z))."""
        o = self.o
        k = self.lay.k
        x = inp.x
        h = [self.rot_sum(o.mul(self.at(x[j], z.depth), z)) for j in range(k)]
        dh = h[0].depth
        v = [o.mul_sum([(self.at(inp.a(j, l), dh), h[l]) for l in range(k)]) for j in range(k)]
        dv = v[0].depth
        xv = o.mul_sum([(self.at(x[j], dv), v[j]) for j in range(k)])
        return o.sub(self.at(z, xv.depth), xv)

    def _fixed(self, inp: EncInput, w: Optional[C.Ct], u: C.Ct) -> FixedPart:
        rr = self._xa(inp)
        fx = FixedPart(x=inp.x, rr=rr, w=w, u=u)
        K = diag_width(self.lay)
        if K and self.m_in is None:
            fx.zt, fx.xt = self.diagonals(inp, rr, snp_depth(inp.kappa), K)
        return fx

    def _xa(self, inp: EncInput) -> List[C.Ct]:
        """r_j = (X A)_{:, j} = sum_l A_jl x_l for the projection of the SNP batches, from A and x brought to
        the SNP depth - 2 first (r_j is used no higher than the SNP depth - 1), so that the products run on
        the few limbs left there."""
        k = self.lay.k
        d = snp_depth(inp.kappa) - 2
        return [self.o.mul_sum([(self.at(inp.a(j, l), d), self.at(inp.x[l], d)) for l in range(k)])
                for j in range(k)]

    def _batches(self, inp: EncInput, fixed: FixedPart, beta, w, w_inv, z_proj, u) -> EncOutput:
        S_proj, nums, dens_e, dens_o = [], [], [], []
        cols = None
        if self.m_in is not None:
            cols = self.m_columns(inp, fixed.rr, self.m_in)
            ds = snp_depth(inp.kappa) + 2
            cols_al = [self.at(c, ds) for c in cols]
            for Sr in self.m_in.S_rep:
                sp = self.project_m(cols_al, Sr)
                num, de, do = self.num_den(sp, fixed)
                S_proj.append(sp)
                nums.append(num)
                dens_e.append(de)
                dens_o.append(do)
        else:
            for S in inp.S:
                sp, num, de, do = self.run_batch(S, fixed)
                S_proj.append(sp)
                nums.append(num)
                dens_e.append(de)
                dens_o.append(do)
        return EncOutput(beta=beta, w=w, w_inv=w_inv, z_proj=z_proj, u=u, S_proj=S_proj,
                         num=nums, den_even=dens_e, den_odd=dens_o, m_cols=cols)

    def _run_kappa1(self, inp: EncInput, r: C.Ct, beta: List[C.Ct]) -> EncOutput:
        """kappa = 1: p = 1/2, w = 1/4 and w^-1 public; z = X beta^(1) + w^-1 (y - 1/2), z' = M z, u = z'/4."""
        o = self.o
        k = self.lay.k
        db = beta[0].depth
        xb = o.mul_sum([(self.at(inp.x[j], db), beta[j]) for j in range(k)])
        z = o.add(xb, self.at(r, xb.depth, W_INV_KAPPA1))
        z_proj = self._project_z(inp, z)
        u = self.at(z_proj, snp_depth(1) + 3, W_KAPPA1)
        fixed = self._fixed(inp, None, u)
        return self._batches(inp, fixed, beta, None, None, z_proj, u)

    def run(self, inp: EncInput) -> EncOutput:
        o = self.o
        lay = self.lay
        k = lay.k
        x, y = inp.x, inp.y
        # ---- Alg. Homomorphic LogReg, pass 1: beta = 0 so p = sigma7(0) = 1/2 is public
        r = o.add_const(y, -0.5)
        g = [self.rot_sum(o.mul(x[j], r)) for j in range(k)]
        beta = [o.mul_int(o.mul_sum([(self.at(inp.a(j, l), 1), g[l]) for l in range(k)]), 4) for j in range(k)]
        if inp.kappa == 1:
            return self._run_kappa1(inp, r, beta)
        p = None
        for _t in range(1, inp.kappa):
            d = beta[0].depth
            # u = X beta / 8: the 1/8 of sigma7's argument is folded into the alignment of x_j
            u = o.mul_sum([(self.at(x[j], d, 0.125), beta[j]) for j in range(k)])
            p = self.sigma7(u)
            dp = p.depth
            r = o.sub(self.at(y, dp), p)
            g = [self.rot_sum(o.mul(self.at(x[j], dp), r)) for j in range(k)]
            dg = g[0].depth
            inc = [o.mul_int(o.mul_sum([(self.at(inp.a(j, l), dg), g[l]) for l in range(k)]), 4) for j in range(k)]
            beta = [o.add(self.at(beta[j], inc[j].depth), inc[j]) for j in range(k)]
        # ---- w = p (1 - p) and Alg. inverseSlots (guess 3, three Newton steps; the first is 6 - 9 w)
        dp = p.depth
        w = o.mul(p, o.add_const(o.neg(p), 1.0))
        gi = o.add_const(o.mul_int(w, -9), 6.0)
        for _ in range(2):
            wg = o.mul(self.at(w, gi.depth), gi)
            h = o.add_const(o.neg(wg), 2.0)
            gi = o.mul(self.at(gi, h.depth), h)
        w_inv = gi
        # ---- z = X beta^(kappa) + w^-1 (y - p^(kappa-1))
        db = beta[0].depth
        xb = o.mul_sum([(self.at(x[j], db), beta[j]) for j in range(k)])
        t = o.mul(self.at(r, w_inv.depth), w_inv)
        z = o.add(self.at(xb, t.depth), t)
        # ---- z' = M z = z - X (A (X^T z)), u = w z'
        z_proj = self._project_z(inp, z)
        u = o.mul(self.at(w, z_proj.depth), z_proj)
        fixed = self._fixed(inp, w, u)
        return self._batches(inp, fixed, beta, w, w_inv, z_proj, u)


# ---- the M-materialised layout's client inputs: X^T in REP form (X_ij in every slot, depth snp_depth + 1,
#      so that the columns of M land at the REP rows' depth with few limbs) and every SNP batch in REP form
#      (row i of the batch, each entry over its block of R slots, two SNPs per complex slot, depth
#      snp_depth + 2, so that S' lands at the depth of the CCP layout's S')
M_SEED_BASE = 2 << 20    # encryption seeds: input_seed(enc_seed, base + i)


@dataclass
class MInput:
    Xrep: List[List[C.Ct]]    # [i][j], i < n, j < k
    S_rep: List[List[C.Ct]]   # [b][i]: batch b, row i


def m_depths(kappa: int):
    return snp_depth(kappa) + 1, snp_depth(kappa) + 2


def snp_rep_slots(S: np.ndarray, lay: Layout, b: int, i: int) -> np.ndarray:
    """Row i of SNP batch b in REP form: slot c R + r (every r < R) holds S[i, b tau + 2c] + i S[i, b tau + 2c + 1]."""
    z = np.zeros(lay.N // 2, dtype=np.complex128)
    for c in range(lay.blocks):
        j0 = b * lay.tau + 2 * c
        v = 0j
        if j0 < lay.m:
            v += float(S[i, j0])
        if j0 + 1 < lay.m:
            v += 1j * float(S[i, j0 + 1])
        z[c * lay.R:(c + 1) * lay.R] = v
    return z


def encode_inputs_m(params: C.Params, X: np.ndarray, S: np.ndarray, kappa: int) -> Plaintexts:
    """Client-side encoding of the M layout's inputs: X_ij replicated (exact constant polynomials, i-major),
    then the REP rows of every SNP batch (batch-major)."""
    n, k = X.shape
    lay = make_layout(params.N, n, k, S.shape[1])
    dx, dsr = m_depths(kappa)
    polys, depths = [], []
    for i in range(n):
        for j in range(k):
            polys.append(constant_poly(X[i, j], params.N, params.scales[dx]))
            depths.append(dx)
    for b in range(lay.n_batches):
        for i in range(n):
            polys.append(C.encode(snp_rep_slots(S, lay, b, i), params.N, params.scales[dsr]))
            depths.append(dsr)
    return Plaintexts(polys=polys, depths=depths)


def encrypt_inputs_m(o: C.Oracle, pts: Plaintexts, n: int, k: int, enc_seed: int) -> MInput:
    cts = [o.encrypt(pt, d, o.p.scales[d], input_seed(enc_seed, M_SEED_BASE + i))
           for i, (pt, d) in enumerate(zip(pts.polys, pts.depths))]
    Xrep = [cts[i * k:(i + 1) * k] for i in range(n)]
    rest = cts[n * k:]
    S_rep = [rest[b * n:(b + 1) * n] for b in range(len(rest) // n)]
    return MInput(Xrep=Xrep, S_rep=S_rep)


# ---- homomorphic division (an extension beyond the paper, which divides on the client): b' and err' as
#      ciphertexts through a Newton reciprocal of den normalised by the public bound d_j of each SNP
DIV_LEVELS = 3 + 2 * (DIV_ITERS - 1)    # x = den v, the Newton steps after the first, err' = g v, b' = num err'
DIV_SEED_BASE = 1 << 20                 # encryption seeds of the normalisers: input_seed(enc_seed, base + i)
assert DIV_GUESS == 1.0                 # the first Newton step is then 2 - x, with no product


def den_scale_factor(kappa: int) -> float:
    """The factor by which a denominator's tracked scale exceeds the canonical scale of its depth."""
    return 4.0 / W_KAPPA1 if kappa == 1 else 4.0


def normaliser_scale(params: C.Params, kappa: int) -> float:
    """Scale of the normalisers: Delta_L / (2 f), so that Re(den) v = ((den + conj(den)) / 2) v is canonical
    (f = den_scale_factor; the real part doubles the tracked scale once more)."""
    return params.scales[circuit_depth(kappa)] / (2.0 * den_scale_factor(kappa))


def normaliser_slots(S: np.ndarray, lay: Layout, b: int, parity: int) -> np.ndarray:
    """1 / d_j at the block start of SNP j = b tau + 2c + parity (c = 0 .. B-1), 0 elsewhere and for SNPs
    beyond m or with d_j = 0."""
    d = snp_normalisers(S)
    z = np.zeros(lay.N // 2, dtype=np.complex128)
    for c in range(lay.blocks):
        j = b * lay.tau + 2 * c + parity
        if j < lay.m and d[j] > 0:
            z[c * lay.R] = 1.0 / d[j]
    return z


def encode_normalisers(params: C.Params, S: np.ndarray, lay: Layout, kappa: int) -> Plaintexts:
    """Client side: the normalisers of every SNP batch, even SNPs of all batches then odd SNPs, at the
    denominators' depth and at normaliser_scale."""
    d = circuit_depth(kappa)
    sc = normaliser_scale(params, kappa)
    polys = [C.encode(normaliser_slots(S, lay, b, par), params.N, sc)
             for par in (0, 1) for b in range(lay.n_batches)]
    return Plaintexts(polys=polys, depths=[d] * len(polys))


def encrypt_normalisers(o: C.Oracle, pts: Plaintexts, kappa: int, enc_seed: int) -> List[C.Ct]:
    sc = normaliser_scale(o.p, kappa)
    return [o.encrypt(pt, dd, sc, input_seed(enc_seed, DIV_SEED_BASE + i))
            for i, (pt, dd) in enumerate(zip(pts.polys, pts.depths))]


@dataclass
class DivOutput:
    b_even: List[C.Ct]     # per batch: real part at block start c = b' of SNP b tau + 2c
    b_odd: List[C.Ct]      # per batch: imaginary part at block start c = b' of SNP b tau + 2c + 1
    inv_even: List[C.Ct]   # per batch: err' = 1 / den of the even SNPs (real part at block starts)
    inv_odd: List[C.Ct]


def divide(o: C.Oracle, num: C.Ct, den: C.Ct, v: C.Ct):
    """Encrypted b' and err' of one batch and parity.  The denominator's slots are complex (its imaginary
    parts are cross terms of the packing), so its real part (den + conj(den)) / 2 is taken first; then
    x = Re(den) v (canonical), g_1 = 2 - x (guess 1), g <- g (2 - x g) (Alg. inverseSlots' pattern),
    err' = g v (real) and b' = num err' (real part: the even SNP's b', imaginary part: the odd one's)."""
    sc = o.p.scales
    at = lambda a, d: a if d == a.depth else o.align(a, d, sc[d])  # noqa: E731
    x = o.mul(o.set_scale(o.add(den, o.conjugate(den)), 2.0), v)
    g = o.add_const(o.neg(x), 2.0)     # g_1 = g_0 (2 - x g_0) with g_0 = DIV_GUESS = 1
    for _ in range(DIV_ITERS - 1):
        h = o.mul(at(x, g.depth), g)
        e = o.add_const(o.neg(h), 2.0)
        g = o.mul(at(g, e.depth), e)
    inv = o.mul(g, at(v, g.depth))
    b = o.mul(at(num, inv.depth), inv)
    return b, inv


def divide_all(o: C.Oracle, out: EncOutput, v: List[C.Ct]) -> DivOutput:
    """divide() for the even and the odd SNPs of every batch (v: even normalisers, then odd)."""
    nb = len(out.num)
    be, bo, ie, io = [], [], [], []
    for b in range(nb):
        x, y = divide(o, out.num[b], out.den_even[b], v[b])
        be.append(x)
        ie.append(y)
        x, y = divide(o, out.num[b], out.den_odd[b], v[nb + b])
        bo.append(x)
        io.append(y)
    return DivOutput(b_even=be, b_odd=bo, inv_even=ie, inv_odd=io)


def finalize_divided(o: C.Oracle, lay: Layout, dv: DivOutput):
    """Client side for the divided outputs: b' and err' decrypted directly (no division), se = sqrt(err')."""
    b = np.zeros(lay.n_batches * lay.tau)
    err = np.zeros(lay.n_batches * lay.tau)
    starts = np.arange(lay.blocks) * lay.R
    for bi in range(lay.n_batches):
        base = bi * lay.tau
        b[base:base + lay.tau:2] = o.decrypt(dv.b_even[bi])[starts].real
        b[base + 1:base + lay.tau:2] = o.decrypt(dv.b_odd[bi])[starts].imag
        err[base:base + lay.tau:2] = o.decrypt(dv.inv_even[bi])[starts].real
        err[base + 1:base + lay.tau:2] = o.decrypt(dv.inv_odd[bi])[starts].real
    b, err = b[:lay.m], err[:lay.m]
    return b, err, np.sqrt(np.maximum(err, 0.0))


def finalize(o: C.Oracle, lay: Layout, out: EncOutput):
    """Client side: decrypt num / den separately, b' = num / den, err' = 1 / den (Alg. Semi Parallel GWAS)."""
    num = np.zeros(lay.n_batches * lay.tau)
    den = np.zeros(lay.n_batches * lay.tau)
    starts = np.arange(lay.blocks) * lay.R
    for b in range(lay.n_batches):
        zn = o.decrypt(out.num[b])[starts]
        ze = o.decrypt(out.den_even[b])[starts]
        zo = o.decrypt(out.den_odd[b])[starts]
        base = b * lay.tau
        num[base:base + lay.tau:2] = zn.real
        num[base + 1:base + lay.tau:2] = zn.imag
        den[base:base + lay.tau:2] = ze.real
        den[base + 1:base + lay.tau:2] = zo.real
    num, den = num[:lay.m], den[:lay.m]
    with np.errstate(divide="ignore", invalid="ignore"):
        b = num / den
        err = 1.0 / den
    return num, den, b, err, np.sqrt(err)
