"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the method itself: it only draws the
covariates, phenotypes and genotypes that both the CPU oracle and the HIP path
consume, so that the two are fed the same bytes.
"""
from .gwas_data import GwasData, config_seed, job_mix, make_gwas_data, padded_rows, poisson_arrivals  # noqa: F401
