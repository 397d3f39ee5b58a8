"""FP64 plaintext semi-parallel GWAS — TEST INFRASTRUCTURE ONLY.

``modified_gwas`` is the result the encrypted circuit approximates: the paper's
modified semi-parallel GWAS with the paper's own approximations (fixed Hessian,
degree-7 sigmoid, Newton reciprocal of the weights), computed in FP64 from
(X, y, S).  ``sikorska_gwas`` (exact semi-parallel GWAS with IRLS) and
``per_snp_logreg`` (one logistic regression per SNP) are secondary references
used only for information.

Readings (where the paper's printed formulas are garbled or silent):

* Degree-7 sigmoid (Methods, "Sigmoid Function Approximation"): the printed
  polynomial is decreasing, i.e. it equals sigma(-x); the signs of the odd
  terms are flipped here so that it approximates sigma(x).
* Newton step (Methods, eq. updateBeta and Alg. "Homomorphic LogReg"): with
  g = X^T (y - p) the ascent step is beta + H~^-1 g with H~^-1 = 4 (X^T X)^-1.
  The printed minus sign combined with the printed (decreasing) sigmoid gives
  -beta with the same probabilities; the projected z' does not depend on that
  sign because M X = 0.
* z uses beta^(kappa) and the p of the last Newton pass, p^(kappa-1)
  (Alg. "Semi Parallel GWAS").
* The numerator weight is w (Alg. "Semi Parallel GWAS" and eq. estSNPeffect),
  not w^-1 as in one sentence of the walk-through.
* err' = 1 / colSum(W S'^2) (eq. estSNPerror) is a variance; se = sqrt(err').
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# magnitudes of the degree-7 sigmoid coefficients in powers of x/8 (Methods, eq. sigma7)
SIGMA7_C1 = 1.73496
SIGMA7_C3 = 4.19407
SIGMA7_C5 = 5.43402
SIGMA7_C7 = 2.50739

INVERSE_GUESS = 3.0   # Alg. inverseSlots: initial guess
INVERSE_ITERS = 3     # Alg. inverseSlots: number of Newton iterations


def sigma7(x: np.ndarray) -> np.ndarray:
    """0.5 + 1.73496 u - 4.19407 u^3 + 5.43402 u^5 - 2.50739 u^7, u = x / 8 (sign-corrected)."""
    u = np.asarray(x, dtype=np.float64) / 8.0
    return 0.5 + SIGMA7_C1 * u - SIGMA7_C3 * u ** 3 + SIGMA7_C5 * u ** 5 - SIGMA7_C7 * u ** 7


def sigma7_printed(x: np.ndarray) -> np.ndarray:
    """The polynomial with the signs exactly as printed (decreasing in x)."""
    u = np.asarray(x, dtype=np.float64) / 8.0
    return 0.5 - SIGMA7_C1 * u + SIGMA7_C3 * u ** 3 - SIGMA7_C5 * u ** 5 + SIGMA7_C7 * u ** 7


def inverse_slots(w: np.ndarray, iters: int = INVERSE_ITERS, guess: float = INVERSE_GUESS) -> np.ndarray:
    """Newton reciprocal g <- g (2 - w g) from g = guess (Alg. inverseSlots)."""
    g = np.full_like(np.asarray(w, dtype=np.float64), guess)
    for _ in range(iters):
        g = g * (2.0 - w * g)
    return g


def xtx_inverse(X: np.ndarray) -> np.ndarray:
    """(X^T X)^-1 through a Cholesky factorisation (the client's preprocessing)."""
    G = X.T @ X
    Lc = np.linalg.cholesky(G)
    Li = np.linalg.solve(Lc, np.eye(G.shape[0]))
    return Li.T @ Li


@dataclass
class GwasResult:
    beta: np.ndarray      # covariate coefficients beta^(kappa)
    p: np.ndarray         # p^(kappa-1)
    w: np.ndarray
    w_inv: np.ndarray
    z: np.ndarray
    z_proj: np.ndarray    # z'
    S_proj: np.ndarray    # S'
    num: np.ndarray
    den: np.ndarray
    b: np.ndarray         # b' = num / den
    err: np.ndarray       # err' = 1 / den
    se: np.ndarray        # sqrt(err')


def homomorphic_logreg_plain(X: np.ndarray, y: np.ndarray, A: np.ndarray, kappa: int, sig=None):
    """Alg. Homomorphic LogReg in FP64: kappa fixed-Hessian Newton steps from beta = 0.

    sig is the sigmoid (default: the degree-7 approximation sigma7).  Returns (beta^(kappa), p^(kappa-1)).
    """
    sig = sigma7 if sig is None else sig
    beta = np.zeros(X.shape[1])
    p = None
    for _ in range(kappa):
        p = sig(X @ beta)
        g = X.T @ (y - p)
        beta = beta + 4.0 * (A @ g)
    return beta, p


def modified_gwas(X: np.ndarray, y: np.ndarray, S: np.ndarray, kappa: int = 3) -> GwasResult:
    """The modified semi-parallel GWAS (Alg. Semi Parallel GWAS; eqs. M, Sprime, zprime, estSNPeffect)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Sf = np.asarray(S, dtype=np.float64)
    A = xtx_inverse(X)
    beta, p = homomorphic_logreg_plain(X, y, A, kappa)
    w = p * (1.0 - p)
    w_inv = inverse_slots(w)
    z = X @ beta + w_inv * (y - p)
    z_proj = z - X @ (A @ (X.T @ z))
    S_proj = Sf - X @ (A @ (X.T @ Sf))
    num = (w * z_proj) @ S_proj
    den = (w[:, None] * S_proj ** 2).sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        b = num / den
        err = 1.0 / den
    return GwasResult(beta=beta, p=p, w=w, w_inv=w_inv, z=z, z_proj=z_proj, S_proj=S_proj,
                      num=num, den=den, b=b, err=err, se=np.sqrt(err))


def packed_num_den(w: np.ndarray, z_proj: np.ndarray, S_proj: np.ndarray):
    """num / den through the complex packing of two SNPs per slot (eqs. z-square .. S-odd).

    Pairs SNP 2c (real part) and 2c+1 (imaginary part); an odd count is padded with a zero SNP.
    Returns (num, den) for the original SNP order.
    """
    n, m = S_proj.shape
    if m % 2:
        S_proj = np.concatenate([S_proj, np.zeros((n, 1))], axis=1)
    Z = S_proj[:, 0::2] + 1j * S_proj[:, 1::2]
    num_c = (w * z_proj) @ Z
    WZ = w[:, None] * Z
    WSS = (WZ * Z).sum(axis=0)
    WSC = (WZ * np.conj(Z)).sum(axis=0)
    den_even = 0.5 * (WSC + WSS)
    den_odd = 0.5 * (WSC - WSS)
    num = np.empty(S_proj.shape[1])
    den = np.empty(S_proj.shape[1])
    num[0::2], num[1::2] = num_c.real, num_c.imag
    den[0::2], den[1::2] = den_even.real, den_odd.real
    return num[:m], den[:m]


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def irls_logreg(X: np.ndarray, y: np.ndarray, tol: float = 1e-12, max_iter: int = 100) -> np.ndarray:
    """Maximum-likelihood logistic regression by Newton-Raphson / IRLS (eqs. updateBeta, grad, hessian)."""
    beta = np.zeros(X.shape[1])
    for _ in range(max_iter):
        p = sigmoid(X @ beta)
        g = X.T @ (y - p)
        H = X.T @ ((p * (1 - p))[:, None] * X)
        step = np.linalg.solve(H, g)
        beta = beta + step
        if np.max(np.abs(g)) < tol:
            break
    return beta


def sikorska_gwas(X: np.ndarray, y: np.ndarray, S: np.ndarray):
    """Exact semi-parallel GWAS (eqs. z, Str, ztr, SNPeffect, SNPerror) with the exact sigmoid.

    Returns (b, err) with err = 1 / colsum(W S*^2).
    """
    X = np.asarray(X, dtype=np.float64)
    Sf = np.asarray(S, dtype=np.float64)
    beta = irls_logreg(X, y)
    p = sigmoid(X @ beta)
    w = p * (1 - p)
    z = X @ beta + (y - p) / w
    G = np.linalg.inv(X.T @ (w[:, None] * X))
    S_star = Sf - X @ (G @ (X.T @ (w[:, None] * Sf)))
    z_star = z - X @ (G @ (X.T @ (w * z)))
    den = (w[:, None] * S_star ** 2).sum(axis=0)
    b = ((w * z_star) @ S_star) / den
    return b, 1.0 / den


def per_snp_logreg(X: np.ndarray, y: np.ndarray, S: np.ndarray):
    """Brute force: one maximum-likelihood fit of [X, s_j] per SNP; returns (b_j, se_j)."""
    X = np.asarray(X, dtype=np.float64)
    b = np.empty(S.shape[1])
    se = np.empty(S.shape[1])
    for j in range(S.shape[1]):
        Xj = np.concatenate([X, S[:, j:j + 1].astype(np.float64)], axis=1)
        beta = irls_logreg(Xj, y)
        p = sigmoid(Xj @ beta)
        H = Xj.T @ ((p * (1 - p))[:, None] * Xj)
        b[j] = beta[-1]
        se[j] = np.sqrt(np.linalg.inv(H)[-1, -1])
    return b, se


def accuracy_counts(b_ref: np.ndarray, b_test: np.ndarray, errs=(0.1, 0.01, 0.005)):
    """The paper's first accuracy method (Results, HEAAN/SEAL accuracy tables):
    number and percentage of entries with |b_ref - b_test| > e."""
    out = {}
    for e in errs:
        bad = int(np.sum(np.abs(b_ref - b_test) > e))
        out[e] = (bad, 100.0 * (1 - bad / len(b_ref)))
    return out


def fit_line(b_ref: np.ndarray, b_test: np.ndarray):
    """The paper's second accuracy method: least-squares line b_test ~ slope * b_ref + intercept."""
    slope, intercept = np.polyfit(b_ref, b_test, 1)
    return float(slope), float(intercept)


# ---- homomorphic division of num by den (an extension: the paper decrypts num and den separately and
#      divides on the client, Methods, walk-through of Alg. Semi Parallel GWAS)
DIV_GUESS = 1.0   # initial guess of the Newton reciprocal of x = den / d (x in (0, 1])
DIV_ITERS = 5     # Newton steps; the first, g = 2 - x, needs no product


def snp_normalisers(S: np.ndarray) -> np.ndarray:
    """d_j = 1/4 ||S_j - mean(S_j)||^2: an upper bound of den_j = sum_i w_i S'_ij^2 known to the holder of S.

    w_i = p_i (1 - p_i) <= 1/4 for every real p_i, and S'_j = M S_j is the shortest residual of S_j after
    projecting out the columns of X, which include the intercept, so ||S'_j|| <= ||S_j - mean(S_j)||.
    A monomorphic SNP has d_j = 0 (no estimate)."""
    Sf = np.asarray(S, dtype=np.float64)
    return 0.25 * ((Sf - Sf.mean(axis=0)) ** 2).sum(axis=0)


def reciprocal_newton(x: np.ndarray, iters: int = DIV_ITERS, guess: float = DIV_GUESS) -> np.ndarray:
    """g <- g (2 - x g) from g = guess (the pattern of Alg. inverseSlots); 1 - x g_t = (1 - guess x)^(2^t)."""
    g = np.full_like(np.asarray(x, dtype=np.float64), guess)
    for _ in range(iters):
        g = g * (2.0 - x * g)
    return g


def divide_plain(num: np.ndarray, den: np.ndarray, d: np.ndarray, iters: int = DIV_ITERS,
                 guess: float = DIV_GUESS):
    """FP64 counterpart of the encrypted division: x = den / d, g = Newton reciprocal of x,
    err' = g / d (about 1 / den) and b' = num err'.  SNPs with d = 0 give 0."""
    v = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    x = den * v
    inv = reciprocal_newton(x, iters, guess) * v
    return num * inv, inv
