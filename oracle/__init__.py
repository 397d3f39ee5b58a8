"""CPU oracle for the encrypted semi-parallel GWAS hot path — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  The
product library (``paper_1902_04303_amd``) never does, and the two share no
code: the only module both sides consume is the seeded input generator in
``synth/``.

Contents:
  ckks_ref.c     plain C RNS-CKKS in coefficient form (unsigned __int128)
  ckks.py        scheme-level driver (params, encode/decode, keys, ops)
  gwas_circuit.py  the encrypted modified semi-parallel GWAS on the oracle
  gwas_fp64.py   the plaintext FP64 GWAS it approximates
  bigint_ref.py  pure-Python big-integer schoolbook checker for tiny rings
"""
