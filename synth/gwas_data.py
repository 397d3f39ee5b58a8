"""Synthetic GWAS workloads with the shapes of the paper's evaluation data.

The paper evaluates on n=245 samples, 4 covariates and 10643 SNPs (Results
section).  That dataset is not available, so every workload here is drawn from
a seeded generator with these distributions:

* X: column 0 is the intercept (all ones), columns 1..k-1 are iid N(0, 1).
* b: iid N(0, 0.5) (variance 0.5), the covariate effects of the phenotype model.
* y_i ~ Bernoulli(sigmoid(x_i . b)), the binary response.
* MAF_j ~ U[0.05, 0.5] and S_ij ~ Binomial(2, MAF_j), independent of y (null SNPs),
  optionally with a planted logit effect on a fraction of the SNPs (acting on the centred genotype
  S_ij - 2 MAF_j).

The draws are made in this fixed order from ``numpy.random.default_rng(seed)``
(PCG64): X, b, MAF, S, then y.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GwasData:
    X: np.ndarray   # (n, k) float64, column 0 = 1
    y: np.ndarray   # (n,) float64 in {0, 1}
    S: np.ndarray   # (n, m) uint8 in {0, 1, 2}
    b: np.ndarray   # (k,) float64 generating covariate effects
    maf: np.ndarray  # (m,) float64
    planted: np.ndarray  # (m,) float64 planted SNP logit effects (zeros for null SNPs)
    seed: int

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def k(self) -> int:
        return self.X.shape[1]

    @property
    def m(self) -> int:
        return self.S.shape[1]


def config_seed(config: int, job: int = 0) -> int:
    """Data seed of workload ``config`` (1-based) and job ``job``."""
    return 1000 + 100 * config + job


def padded_rows(n: int) -> int:
    """Smallest power of two >= n (the paper's PO2 rounding of the column size)."""
    r = 1
    while r < n:
        r *= 2
    return r


def make_gwas_data(n: int, k: int, m: int, seed: int, planted_frac: float = 0.0,
                   planted_effect: float = 0.5) -> GwasData:
    if n < 2 or k < 1 or m < 1:
        raise ValueError("need n >= 2, k >= 1, m >= 1")
    rng = np.random.default_rng(seed)
    X = np.empty((n, k), dtype=np.float64)
    X[:, 0] = 1.0
    if k > 1:
        X[:, 1:] = rng.standard_normal((n, k - 1))
    b = rng.normal(0.0, np.sqrt(0.5), size=k)
    maf = rng.uniform(0.05, 0.5, size=m)
    S = rng.binomial(2, maf[None, :], size=(n, m)).astype(np.uint8)
    planted = np.zeros(m, dtype=np.float64)
    if planted_frac > 0.0:
        n_pl = max(1, int(round(planted_frac * m)))
        idx = rng.choice(m, size=n_pl, replace=False)
        planted[idx] = planted_effect
    # planted effects act on centred genotypes (S - 2 MAF), so that many planted SNPs shift the spread of
    # the logit rather than its mean (the phenotype stays a mix of both classes)
    logit = X @ b + (S.astype(np.float64) - 2.0 * maf[None, :]) @ planted
    p = 1.0 / (1.0 + np.exp(-logit))
    y = (rng.uniform(size=n) < p).astype(np.float64)
    return GwasData(X=X, y=y, S=S, b=b, maf=maf, planted=planted, seed=seed)


def job_mix(count: int, seed: int, m_scale: float = 1.0):
    """Sizes of a mix of GWAS jobs: n ~ U{100..2000}, k = 4, m = round(exp(U[ln 1e3, ln 5e4]) * m_scale).

    Returns a list of (n, k, m, data_seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.integers(100, 2001))
        m = max(1, int(round(np.exp(rng.uniform(np.log(1e3), np.log(5e4))) * m_scale)))
        out.append((n, 4, m, seed * 1000 + j))
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
