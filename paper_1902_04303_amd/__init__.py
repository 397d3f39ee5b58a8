"""MI355X-native RNS-CKKS evaluator and encrypted semi-parallel GWAS.

The computation lives in the HIP library ``_build/libgwasckks.so`` behind the C
ABI of ``include/gwas_ckks.h``; this package is a thin ctypes binding with the
same names.  Importing it does not need a GPU; creating a context does.
"""
from ._binding import (  # noqa: F401
    Ciphertext,
    CkksError,
    Context,
    GwasInput,
    GwasOutput,
    GwasServer,
    LIB_PATH,
    chain,
    exported_symbols,
    gwas_div_levels,
    gwas_galois_elements,
    ks_alpha,
    lib,
)
