"""ctypes binding of ``include/gwas_ckks.h`` — argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays to pointers and error codes to exceptions.  PyTorch supplies the
device memory (through the allocator callbacks) and the HIP stream.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libgwasckks.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p
_szp = ctypes.POINTER(ctypes.c_size_t)


class CkksParams(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int), ("levels", ctypes.c_int), ("log2_scale", ctypes.c_int),
                ("ks_alpha", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class CkksAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


ERRORS = {-1: "INVALID_ARG", -2: "PARAM_MISMATCH", -3: "LEVEL", -4: "KEY_MISSING", -5: "NOMEM", -6: "HIP",
          -7: "CANCELLED", -8: "NOT_READY"}


class CkksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


_LIB = None
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    """Destroy live contexts before the interpreter (and torch's allocator) shuts down."""
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:
            pass

# (name, restype, argtypes)
_SIGS = [
    ("ckks_last_error", ctypes.c_char_p, []),
    ("ckks_params_ks_alpha", ctypes.c_int, [ctypes.POINTER(CkksParams)]),
    ("ckks_chain", ctypes.c_int, [ctypes.POINTER(CkksParams), _u64p, _dp]),
    ("ckks_ctx_create", ctypes.c_int, [ctypes.POINTER(CkksParams), ctypes.POINTER(CkksAllocator), _vp, ctypes.c_size_t,
                                       ctypes.POINTER(_vp)]),
    ("ckks_ctx_destroy", None, [_vp]),
    ("ckks_ctx_moduli", ctypes.c_int, [_vp, _u64p, ctypes.c_int]),
    ("ckks_ctx_scales", ctypes.c_int, [_vp, _dp, ctypes.c_int]),
    ("ckks_ctx_pool_stats", ctypes.c_int, [_vp, _szp, _szp, _szp, _szp]),
    ("ckks_ctx_pool_trim", ctypes.c_int, [_vp]),
    ("ckks_ctx_kernel_timing", ctypes.c_int, [_vp, ctypes.c_int]),
    ("ckks_ctx_kernel_report", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    ("ckks_ctx_kernel_timing_only", ctypes.c_int, [_vp, ctypes.c_char_p]),
    ("ckks_ctx_set_streams", ctypes.c_int, [_vp, ctypes.c_int]),
    ("ckks_ctx_set_stack", ctypes.c_int, [_vp, ctypes.c_int]),
    ("ckks_ctx_counters", ctypes.c_int, [_vp, _u64p, _u64p, _u64p]),
    ("ckks_ctx_keyswitch_ciphertexts", ctypes.c_int, [_vp, _u64p]),
    ("ckks_keygen", ctypes.c_int, [_vp, ctypes.c_uint64, _u64p, ctypes.c_int]),
    ("ckks_galois_rotate", ctypes.c_uint64, [_vp, ctypes.c_int64]),
    ("ckks_galois_conj", ctypes.c_uint64, [_vp]),
    ("ckks_export_switching_key", ctypes.c_int, [_vp, ctypes.c_uint64, _u64p, ctypes.c_size_t]),
    ("ckks_export_secret", ctypes.c_int, [_vp, _i64p, ctypes.c_size_t]),
    ("ckks_export_public_key", ctypes.c_int, [_vp, _u64p, ctypes.c_size_t]),
    ("ckks_import_public_key", ctypes.c_int, [_vp, _u64p, ctypes.c_size_t]),
    ("ckks_import_switching_key", ctypes.c_int, [_vp, ctypes.c_uint64, _u64p, ctypes.c_size_t]),
    ("ckks_ctx_has_secret", ctypes.c_int, [_vp]),
    ("ckks_encode", ctypes.c_int, [_vp, _dp, _dp, ctypes.c_size_t, ctypes.c_double, _i64p]),
    ("ckks_decode", ctypes.c_int, [_vp, _dp, _dp, _dp]),
    ("ckks_encrypt", ctypes.c_int, [_vp, _i64p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    ("ckks_decrypt", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _dp]),
    ("ckks_decrypt_poly", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp]),
    ("ckks_ct_info", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), _dp]),
    ("ckks_ct_export", ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_size_t]),
    ("ckks_ct_import", ctypes.c_int, [_vp, _u64p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp)]),
    ("ckks_ct_free", None, [_vp]),
    ("ckks_add", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    ("ckks_sub", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    ("ckks_mul", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    ("ckks_mul_noalloc", ctypes.c_int, [_vp, _vp, _vp, _vp]),
    ("ckks_mul_int", ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.POINTER(_vp)]),
    ("ckks_add_const", ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.POINTER(_vp)]),
    ("ckks_mul_const", ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.POINTER(_vp)]),
    ("ckks_rescale", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    ("ckks_align", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_vp)]),
    ("ckks_rotate", ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.POINTER(_vp)]),
    ("ckks_rotate_sum", ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_galois_elements", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int)]),
    ("ckks_conjugate", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    ("ckks_mul_mask", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("ckks_ntt_device", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    ("gwas_layout", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("gwas_pack_encrypt", ctypes.c_int, [_vp, _dp, _dp, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint64, ctypes.POINTER(_vp)]),
    ("gwas_input_from_cts", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(_vp), _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_input_free", None, [_vp]),
    ("gwas_input_ct", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_output_from_cts", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int,
                                            ctypes.POINTER(_vp)]),
    ("gwas_semiparallel", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    ("gwas_semiparallel_chunked", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_output_ct", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_output_batches", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("gwas_output_free", None, [_vp]),
    ("gwas_finalize", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]),
    ("gwas_div_levels", ctypes.c_int, []),
    ("gwas_tune", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 _dp, _dp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("ckks_ctx_use_tuned", ctypes.c_int, [_vp, ctypes.c_int]),
    ("gwas_keep_projected", ctypes.c_int, [_vp, ctypes.c_int]),
    ("gwas_graph_create", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_graph_set_input", ctypes.c_int, [_vp, _vp]),
    ("gwas_graph_launch", ctypes.c_int, [_vp]),
    ("gwas_graph_output", ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    ("gwas_graph_destroy", None, [_vp]),
    ("gwas_input_attach_m", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                           ctypes.c_int]),
    ("gwas_pack_encrypt_m", ctypes.c_int, [_vp, _vp, _dp, _u8p, ctypes.c_uint64]),
    ("gwas_pack_normalisers", ctypes.c_int, [_vp, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                             ctypes.POINTER(_vp)]),
    ("gwas_divide", ctypes.c_int, [_vp, _vp, _vp]),
    ("gwas_finalize_divided", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _dp, _dp]),
    ("ckks_ct_stack", ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_semiparallel_multi", ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(_vp)]),
    ("gwas_input_footprint", ctypes.c_int, [_vp, _szp]),
    ("gwas_input_spill", ctypes.c_int, [_vp, _vp]),
    ("gwas_server_create", ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_server_submit", ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    ("gwas_server_poll", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("gwas_server_cancel", ctypes.c_int, [_vp, ctypes.c_uint64]),
    ("gwas_server_stats", ctypes.c_int, [_vp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_int)]),
    ("gwas_server_destroy", None, [_vp]),
]


def lib():
    """Load the built library; raises if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library not built: %s is missing (run paper_1902_04303_amd/build.py)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols() -> List[str]:
    return [s[0] for s in _SIGS]


def _check(rc: int):
    if rc != 0:
        raise CkksError(rc, lib().ckks_last_error().decode())


def _u64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(_u64p)


def _i64(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_i64p)


def _f64(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def gwas_div_levels() -> int:
    """Levels the homomorphic division takes after the denominators."""
    return int(lib().gwas_div_levels())


def ks_alpha(log_n: int, levels: int, log2_scale: int, alpha: int = 0) -> int:
    """Digit-group size of key switching that the parameters select (alpha = 0: the library default)."""
    a = lib().ckks_params_ks_alpha(ctypes.byref(CkksParams(log_n, levels, log2_scale, alpha)))
    if a < 0:
        _check(a)
    return int(a)


def chain(log_n: int, levels: int, log2_scale: int, alpha: int = 0):
    """(q_0..q_L, [p_1..p_alpha], canonical scales): the moduli and scales of the parameters (host only)."""
    p = CkksParams(log_n, levels, log2_scale, alpha)
    q = np.zeros(levels + 1 + ks_alpha(log_n, levels, log2_scale, alpha), dtype=np.uint64)
    s = np.zeros(levels + 1, dtype=np.float64)
    _check(lib().ckks_chain(ctypes.byref(p), _u64(q), _f64(s)))
    return [int(v) for v in q[:levels + 1]], [int(v) for v in q[levels + 1:]], [float(v) for v in s]


def gwas_galois_elements(log_n: int, R: int) -> List[int]:
    """Galois elements whose switching keys the GWAS circuit needs for block size R (host computation)."""
    cnt = ctypes.c_int()
    _check(lib().gwas_galois_elements(log_n, R, None, 0, ctypes.byref(cnt)))
    out = (ctypes.c_uint64 * cnt.value)()
    _check(lib().gwas_galois_elements(log_n, R, out, cnt.value, ctypes.byref(cnt)))
    return [int(v) for v in out]


class Ciphertext:
    """A batch of ciphertexts owned by the library (freed on garbage collection)."""

    def __init__(self, ctx: "Context", handle: int, owned: bool = True):
        self.ctx = ctx
        self.h = _vp(handle)
        self.owned = owned

    def __del__(self):
        if getattr(self, "owned", False) and self.h and self.ctx is not None and self.ctx.h:
            lib().ckks_ct_free(self.h)
            self.h = None

    def info(self):
        c, d, l, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().ckks_ct_info(self.h, ctypes.byref(c), ctypes.byref(d), ctypes.byref(l), ctypes.byref(s)))
        return c.value, d.value, l.value, s.value

    @property
    def count(self):
        return self.info()[0]

    @property
    def depth(self):
        return self.info()[1]

    @property
    def limbs(self):
        return self.info()[2]

    @property
    def scale(self):
        return self.info()[3]


class Context:
    def __init__(self, log_n: int, levels: int, log2_scale: int, use_torch: bool = True, pool_budget: int = 0,
                 stream: Optional[int] = None, alpha: int = 0):
        self.h = None
        p = CkksParams(log_n, levels, log2_scale, alpha)
        self.alpha = ks_alpha(log_n, levels, log2_scale, alpha)   # digit-group size of key switching
        self._keep = []
        alloc = None
        if use_torch:
            import torch
            dev = torch.cuda.current_device()
            st = torch.cuda.current_stream() if stream is None else None
            s_handle = st.cuda_stream if st is not None else stream

            t_alloc = torch.cuda.caching_allocator_alloc
            t_free = torch.cuda.caching_allocator_delete

            def _alloc(nbytes, user):
                try:
                    return int(t_alloc(int(nbytes), dev, s_handle))
                except Exception:
                    return None

            def _free(ptr, nbytes, user):
                try:
                    t_free(int(ptr))
                except Exception:
                    pass

            fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep += [fa, ff]
            alloc = CkksAllocator(fa, ff, None)
            stream_handle = s_handle
        else:
            stream_handle = stream
        out = _vp()
        _check(lib().ckks_ctx_create(ctypes.byref(p), ctypes.byref(alloc) if alloc else None,
                                     _vp(stream_handle) if stream_handle else None, pool_budget, ctypes.byref(out)))
        self.h = out
        _LIVE.add(self)
        self.log_n, self.levels, self.log2_scale = log_n, levels, log2_scale
        self.N = 1 << log_n

    def close(self):
        if self.h:
            lib().ckks_ctx_destroy(self.h)
            self.h = None
        _LIVE.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- parameters
    def moduli(self) -> List[int]:
        a = np.zeros(self.levels + 1 + self.alpha, dtype=np.uint64)
        _check(lib().ckks_ctx_moduli(self.h, _u64(a), len(a)))
        return [int(v) for v in a]

    def scales(self) -> List[float]:
        a = np.zeros(self.levels + 1, dtype=np.float64)
        _check(lib().ckks_ctx_scales(self.h, _f64(a), len(a)))
        return [float(v) for v in a]

    def pool_stats(self):
        v = [ctypes.c_size_t() for _ in range(4)]
        _check(lib().ckks_ctx_pool_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("in_use", "cached", "peak", "n_alloc"), [x.value for x in v]))

    def pool_trim(self):
        _check(lib().ckks_ctx_pool_trim(self.h))

    def counters(self):
        v = [ctypes.c_uint64() for _ in range(3)]
        _check(lib().ckks_ctx_counters(self.h, *[ctypes.byref(x) for x in v]))
        n = ctypes.c_uint64()
        _check(lib().ckks_ctx_keyswitch_ciphertexts(self.h, ctypes.byref(n)))
        return dict(zip(("keyswitches", "limb_ntts", "launches", "keyswitch_ciphertexts"),
                        [x.value for x in v] + [n.value]))

    def kernel_timing(self, enable: bool):
        _check(lib().ckks_ctx_kernel_timing(self.h, 1 if enable else 0))

    def kernel_timing_only(self, name: Optional[str]):
        _check(lib().ckks_ctx_kernel_timing_only(self.h, name.encode() if name else None))

    def set_streams(self, n: int):
        """1: the GWAS circuit runs in order on one stream; 2 (default): the logistic-regression part
        overlaps the independent per-batch work on a second stream."""
        _check(lib().ckks_ctx_set_streams(self.h, int(n)))

    def set_stack(self, n: int):
        """Ciphertexts up to which the per-batch part stacks its covariates' products (0: one at a time)."""
        _check(lib().ckks_ctx_set_stack(self.h, int(n)))

    def kernel_report(self):
        """{kernel: (launches, total_ms, algorithmic_bytes, algorithmic_fp64_ops, pass_bytes)} from the
        HIP-event timing ("keyswitch": whole key switches, when selected with kernel_timing_only)."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().ckks_ctx_kernel_report(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms, by, fl, pb = line.rsplit(None, 5)   # kernel names may contain spaces
            out[name] = (int(cnt), float(ms), float(by), float(fl), float(pb))
        return out

    # ---- keys
    def keygen(self, seed: int, galois: Sequence[int] = ()):
        g = np.array(list(galois), dtype=np.uint64)
        _check(lib().ckks_keygen(self.h, seed, _u64(g) if len(g) else None, len(g)))

    def galois_rotate(self, r: int) -> int:
        return int(lib().ckks_galois_rotate(self.h, r))

    def galois_conj(self) -> int:
        return int(lib().ckks_galois_conj(self.h))

    def export_switching_key(self, key_id: int) -> np.ndarray:
        L = self.levels
        a = np.zeros((2, 1 + (L + 1) // self.alpha, L + 1 + self.alpha, self.N), dtype=np.uint64)
        _check(lib().ckks_export_switching_key(self.h, key_id, _u64(a), a.size))
        return a

    def export_secret(self) -> np.ndarray:
        a = np.zeros(self.N, dtype=np.int64)
        _check(lib().ckks_export_secret(self.h, _i64(a), a.size))
        return a

    def export_public_key(self) -> np.ndarray:
        a = np.zeros((2, self.levels + 1, self.N), dtype=np.uint64)
        _check(lib().ckks_export_public_key(self.h, _u64(a), a.size))
        return a

    def import_public_key(self, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        _check(lib().ckks_import_public_key(self.h, _u64(a), a.size))

    def import_switching_key(self, key_id: int, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        _check(lib().ckks_import_switching_key(self.h, key_id, _u64(a), a.size))

    def has_secret(self) -> bool:
        return bool(lib().ckks_ctx_has_secret(self.h))

    # ---- encode / encrypt / decrypt
    def encode(self, z: np.ndarray, scale: float) -> np.ndarray:
        z = np.asarray(z, dtype=np.complex128)
        re = np.ascontiguousarray(z.real)
        im = np.ascontiguousarray(z.imag)
        out = np.zeros(self.N, dtype=np.int64)
        _check(lib().ckks_encode(self.h, _f64(re), _f64(im), len(z), scale, _i64(out)))
        return out

    def encrypt(self, m: np.ndarray, depth: int, scale: float, seed: int) -> Ciphertext:
        m = np.ascontiguousarray(m, dtype=np.int64)
        out = _vp()
        _check(lib().ckks_encrypt(self.h, _i64(m), depth, scale, seed, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def decrypt(self, ct: Ciphertext, index: int = 0) -> np.ndarray:
        re = np.zeros(self.N // 2)
        im = np.zeros(self.N // 2)
        _check(lib().ckks_decrypt(self.h, ct.h, index, _f64(re), _f64(im)))
        return re + 1j * im

    def decrypt_poly(self, ct: Ciphertext, index: int = 0) -> np.ndarray:
        out = np.zeros(self.N)
        _check(lib().ckks_decrypt_poly(self.h, ct.h, index, _f64(out)))
        return out

    def export(self, ct: Ciphertext, index: int = 0) -> np.ndarray:
        _, _, l, _ = ct.info()
        a = np.zeros((2, l, self.N), dtype=np.uint64)
        _check(lib().ckks_ct_export(self.h, ct.h, index, _u64(a), a.size))
        return a

    def import_ct(self, data: np.ndarray, depth: int, scale: float) -> Ciphertext:
        data = np.ascontiguousarray(data, dtype=np.uint64)
        out = _vp()
        _check(lib().ckks_ct_import(self.h, _u64(data), depth, scale, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    # ---- evaluation
    def _op(self, fn, *args) -> Ciphertext:
        out = _vp()
        _check(fn(self.h, *args, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def add(self, a, b):
        return self._op(lib().ckks_add, a.h, b.h)

    def sub(self, a, b):
        return self._op(lib().ckks_sub, a.h, b.h)

    def mul(self, a, b):
        return self._op(lib().ckks_mul, a.h, b.h)

    def mul_noalloc(self, a, b, out: Ciphertext) -> Ciphertext:
        """a * b (as mul) written into the existing ciphertext `out` without any device allocation."""
        _check(lib().ckks_mul_noalloc(self.h, a.h, b.h, out.h))
        return out

    def mul_int(self, a, k: int):
        return self._op(lib().ckks_mul_int, a.h, int(k))

    def add_const(self, a, c: float):
        return self._op(lib().ckks_add_const, a.h, float(c))

    def mul_const(self, a, c: float):
        return self._op(lib().ckks_mul_const, a.h, float(c))

    def rescale(self, a):
        return self._op(lib().ckks_rescale, a.h)

    def align(self, a, depth: int, scale: float, factor: float = 1.0):
        return self._op(lib().ckks_align, a.h, depth, scale, factor)

    def rotate(self, a, r: int):
        return self._op(lib().ckks_rotate, a.h, int(r))

    def rotate_sum(self, a, rots: Sequence[int]):
        """a + sum_i rotate(a, rots[i]) with one shared key switch (1 to 16 rotations)."""
        arr = (ctypes.c_int64 * len(rots))(*[int(r) for r in rots])
        return self._op(lib().ckks_rotate_sum, a.h, arr, len(rots))

    def conjugate(self, a):
        return self._op(lib().ckks_conjugate, a.h)

    def mul_mask(self, a, R: int):
        return self._op(lib().ckks_mul_mask, a.h, int(R))

    def ntt_device(self, dev_ptr: int, count: int, moduli_index: Sequence[int], direction: int):
        idx = (ctypes.c_int * count)(*moduli_index)
        _check(lib().ckks_ntt_device(self.h, _vp(dev_ptr), count, idx, direction))

    # ---- GWAS
    def gwas_layout(self, n: int, k: int, m: int, kappa: int):
        v = [ctypes.c_int() for _ in range(4)]
        _check(lib().gwas_layout(self.h, n, k, m, kappa, *[ctypes.byref(x) for x in v]))
        return dict(zip(("R", "tau", "n_batches", "levels_needed"), [x.value for x in v]))

    def gwas_pack_encrypt(self, X: np.ndarray, y: np.ndarray, S: np.ndarray, kappa: int, enc_seed: int) -> "GwasInput":
        X = np.ascontiguousarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.uint8)
        n, k = X.shape
        m = S.shape[1]
        out = _vp()
        _check(lib().gwas_pack_encrypt(self.h, _f64(X), _f64(y), S.ctypes.data_as(_u8p), n, k, m, kappa, enc_seed,
                                       ctypes.byref(out)))
        return GwasInput(self, out.value, n, k, m, kappa)

    def gwas_input_from_cts(self, n, k, m, kappa, x: Sequence[Ciphertext], y: Ciphertext, A: Sequence[Ciphertext],
                            S: Sequence[Ciphertext]) -> "GwasInput":
        xa = (_vp * len(x))(*[c.h for c in x])
        aa = (_vp * len(A))(*[c.h for c in A])
        sa = (_vp * len(S))(*[c.h for c in S])
        out = _vp()
        _check(lib().gwas_input_from_cts(self.h, n, k, m, kappa, xa, y.h, aa, sa, len(S), ctypes.byref(out)))
        return GwasInput(self, out.value, n, k, m, kappa)

    def gwas_output_from_cts(self, n, k, m, num: Sequence[Ciphertext], den_even: Sequence[Ciphertext],
                             den_odd: Sequence[Ciphertext]) -> "GwasOutput":
        arr = lambda v: (_vp * len(v))(*[c.h for c in v])  # noqa: E731
        out = _vp()
        _check(lib().gwas_output_from_cts(self.h, n, k, m, arr(num), arr(den_even), arr(den_odd), len(num),
                                          ctypes.byref(out)))
        return GwasOutput(self, out.value, m)

    def gwas_semiparallel(self, inp: "GwasInput", chunk: Optional[int] = None) -> "GwasOutput":
        out = _vp()
        if chunk is None:
            _check(lib().gwas_semiparallel(self.h, inp.h, ctypes.byref(out)))
        else:
            _check(lib().gwas_semiparallel_chunked(self.h, inp.h, chunk, ctypes.byref(out)))
        return GwasOutput(self, out.value, inp.m)

    def gwas_semiparallel_multi(self, inputs: Sequence["GwasInput"], chunk: int = 64) -> List["GwasOutput"]:
        arr = (_vp * len(inputs))(*[i.h for i in inputs])
        outs = (_vp * len(inputs))()
        _check(lib().gwas_semiparallel_multi(self.h, arr, len(inputs), chunk, outs))
        return [GwasOutput(self, outs[i], inputs[i].m) for i in range(len(inputs))]

    def gwas_server(self, hbm_budget: int = 0, max_jobs: int = 64, chunk: int = 64) -> "GwasServer":
        return GwasServer(self, hbm_budget, max_jobs, chunk)

    def gwas_tune(self, inp: "GwasInput", reps: int = 2):
        """Time the bit-identical schedules (chunk, streams, stack) on inp and record the fastest for its shape."""
        ch, st, cand, stk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ms, ms0 = ctypes.c_double(), ctypes.c_double()
        _check(lib().gwas_tune(self.h, inp.h, reps, ctypes.byref(ch), ctypes.byref(st), ctypes.byref(ms),
                               ctypes.byref(ms0), ctypes.byref(cand), ctypes.byref(stk)))
        return dict(chunk=ch.value, streams=st.value, stack=stk.value, ms=ms.value, ms_default=ms0.value,
                    candidates=cand.value)

    def keep_projected(self, keep: bool):
        """Whether outputs keep S' of every SNP batch (default True)."""
        _check(lib().gwas_keep_projected(self.h, 1 if keep else 0))

    def use_tuned(self, enable: bool = True):
        _check(lib().ckks_ctx_use_tuned(self.h, 1 if enable else 0))

    def gwas_graph(self, inp: "GwasInput", chunk: int = 0) -> "GwasGraph":
        """gwas_semiparallel of inp's shape captured as a HIP graph (replayed by GwasGraph.launch)."""
        return GwasGraph(self, inp, chunk)

    def stack(self, parts: Sequence[Ciphertext]) -> Ciphertext:
        """One batch holding the ciphertexts of every part, in order (copied)."""
        arr = (_vp * len(parts))(*[p.h for p in parts])
        out = _vp()
        _check(lib().ckks_ct_stack(self.h, arr, len(parts), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def gwas_input_attach_m(self, inp: "GwasInput", xrep: Sequence[Ciphertext], srep: Sequence[Ciphertext]):
        """M-materialised layout: attach the REP X^T (n k, sample-major) and REP SNP rows (n per batch)."""
        xa = (_vp * len(xrep))(*[c.h for c in xrep])
        sa = (_vp * len(srep))(*[c.h for c in srep])
        _check(lib().gwas_input_attach_m(self.h, inp.h, xa, len(xrep), sa, len(srep)))
        return inp

    def gwas_pack_encrypt_m(self, inp: "GwasInput", X: np.ndarray, S: np.ndarray, enc_seed: int):
        """Client side: encrypt and attach the REP inputs of the M-materialised layout."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.uint8)
        _check(lib().gwas_pack_encrypt_m(self.h, inp.h, _f64(X), S.ctypes.data_as(_u8p), enc_seed))
        return inp

    def gwas_pack_normalisers(self, S: np.ndarray, kappa: int, enc_seed: int) -> Ciphertext:
        """Client side: the division's normalisers 1 / d_j (2 per SNP batch: even SNPs, then odd)."""
        S = np.ascontiguousarray(S, dtype=np.uint8)
        n, m = S.shape
        out = _vp()
        _check(lib().gwas_pack_normalisers(self.h, S.ctypes.data_as(_u8p), n, m, kappa, enc_seed,
                                           ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def gwas_divide(self, out: "GwasOutput", v: Ciphertext) -> "GwasOutput":
        """Encrypted b' and err' (Newton reciprocal of the normalised denominators), stored in out."""
        _check(lib().gwas_divide(self.h, out.h, v.h))
        return out

    def gwas_finalize_divided(self, out: "GwasOutput"):
        m = out.m
        b, err, se = (np.zeros(m) for _ in range(3))
        _check(lib().gwas_finalize_divided(self.h, out.h, m, _f64(b), _f64(err), _f64(se)))
        return dict(b=b, err=err, se=se)

    def gwas_finalize(self, out: "GwasOutput"):
        m = out.m
        b, err, se, num, den = (np.zeros(m) for _ in range(5))
        _check(lib().gwas_finalize(self.h, out.h, m, _f64(b), _f64(err), _f64(se), _f64(num), _f64(den)))
        return dict(b=b, err=err, se=se, num=num, den=den)


class GwasGraph:
    def __init__(self, ctx: Context, inp: "GwasInput", chunk: int):
        self.ctx, self.m, self.h = ctx, inp.m, None
        h = _vp()
        _check(lib().gwas_graph_create(ctx.h, inp.h, chunk, ctypes.byref(h)))
        self.h = h
        o = _vp()
        _check(lib().gwas_graph_output(self.h, ctypes.byref(o)))
        self.out = GwasOutput(ctx, o.value, inp.m, owned=False)
        self.out._parent = self

    def set_input(self, inp: "GwasInput"):
        _check(lib().gwas_graph_set_input(self.h, inp.h))

    def launch(self) -> "GwasOutput":
        """Replay the graph on the context's stream; returns the (graph-owned) output."""
        _check(lib().gwas_graph_launch(self.h))
        return self.out

    def close(self):
        if self.h and self.ctx is not None and self.ctx.h:
            lib().gwas_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()


class GwasInput:
    def __init__(self, ctx: Context, handle: int, n, k, m, kappa):
        self.ctx, self.h = ctx, _vp(handle)
        self.n, self.k, self.m, self.kappa = n, k, m, kappa

    def __del__(self):
        if self.h and self.ctx is not None and self.ctx.h:
            lib().gwas_input_free(self.h)
            self.h = None

    X, Y, A, S = range(4)

    def ct(self, which: int, index: int = 0) -> Ciphertext:
        out = _vp()
        _check(lib().gwas_input_ct(self.h, which, index, ctypes.byref(out)))
        ct = Ciphertext(self.ctx, out.value, owned=False)
        ct._parent = self   # the handle belongs to this input
        return ct

    def footprint(self) -> int:
        v = ctypes.c_size_t()
        _check(lib().gwas_input_footprint(self.h, ctypes.byref(v)))
        return v.value

    def spill(self):
        _check(lib().gwas_input_spill(self.ctx.h, self.h))


class GwasServer:
    """Serving loop of the library (a native worker thread); submit() hands the input over."""

    def __init__(self, ctx: Context, hbm_budget: int, max_jobs: int, chunk: int):
        self.ctx, self.h = ctx, None
        out = _vp()
        _check(lib().gwas_server_create(ctx.h, hbm_budget, max_jobs, chunk, ctypes.byref(out)))
        self.h = out

    def submit(self, inp: GwasInput) -> int:
        jid = ctypes.c_uint64()
        _check(lib().gwas_server_submit(self.h, inp.h, ctypes.byref(jid)))
        inp.h = None          # owned by the server now (a failed submit leaves it with the caller)
        return jid.value

    def poll(self, job_id: int, m: int, wait: bool = False) -> Optional["GwasOutput"]:
        out = _vp()
        rc = lib().gwas_server_poll(self.h, job_id, 1 if wait else 0, ctypes.byref(out))
        if rc == -8:
            return None
        _check(rc)
        return GwasOutput(self.ctx, out.value, m)

    def cancel(self, job_id: int):
        _check(lib().gwas_server_cancel(self.h, job_id))

    def stats(self):
        p50, p99, tput = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n, peak = ctypes.c_uint64(), ctypes.c_int()
        _check(lib().gwas_server_stats(self.h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(tput),
                                       ctypes.byref(n), ctypes.byref(peak)))
        return dict(p50_ms=p50.value, p99_ms=p99.value, jobs_per_s=tput.value, completed=n.value,
                    peak_jobs_in_flight=peak.value)

    def close(self):
        if self.h:
            lib().gwas_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GwasOutput:
    NUM, DEN_EVEN, DEN_ODD, S_PROJ, BETA, W, W_INV, Z_PROJ, U, DIV_B, DIV_ERR, M_COLS = range(12)

    def __init__(self, ctx: Context, handle: int, m: int, owned: bool = True):
        self.ctx, self.h, self.m, self.owned = ctx, _vp(handle), m, owned

    def __del__(self):
        if self.owned and self.h and self.ctx is not None and self.ctx.h:
            lib().gwas_output_free(self.h)
        self.h = None

    def ct(self, which: int, index: int = 0) -> Ciphertext:
        out = _vp()
        _check(lib().gwas_output_ct(self.h, which, index, ctypes.byref(out)))
        ct = Ciphertext(self.ctx, out.value, owned=False)
        ct._parent = self   # the handle belongs to this output: keep it alive while the ciphertext is used
        return ct
