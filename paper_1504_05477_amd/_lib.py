"""ctypes view of libbk.so (include/bk.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbk.so")

# bk_dtype
F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
# bk_status
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ENOCONV, ERANK = range(7)
PHASES = ("pi", "ax", "aty", "proj", "cholqr", "m", "eig", "z", "refine",
          "prep", "center", "long")


class Options(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("refine", C.c_int32),
        ("center_rows", C.c_int32),
        ("max_jacobi_sweeps", C.c_int32),
        ("jacobi_tol", C.c_double),
        ("breakdown_tol", C.c_double),
        ("pi", C.c_void_p),
        ("timing", C.c_int32),
        ("save_for_backward", C.c_int32),
        ("jacobi_block", C.c_int32),
        ("block_size", C.c_int32),
        ("method", C.c_int32),
        ("timing_phases", C.c_int32),
        ("reserved", C.c_int32 * 2),
        ("residuals", C.c_void_p),
        ("a_transposed", C.c_void_p),
        ("ld_at", C.c_int64),
        ("at_scales", C.c_void_p),
        ("fp32_products", C.c_int32),
        ("csr_gather", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("q_eff", C.c_int32),
        ("jacobi_sweeps", C.c_int32),
        ("jacobi_offdiag", C.c_double),
        ("ms", C.c_float * len(PHASES)),
        ("launches", C.c_int32 * len(PHASES)),
        ("workspace_bytes", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "q_eff": self.q_eff,
            "jacobi_sweeps": self.jacobi_sweeps,
            "jacobi_offdiag": self.jacobi_offdiag,
            "ms": {p: float(self.ms[i]) for i, p in enumerate(PHASES)},
            "launches": {p: int(self.launches[i]) for i, p in enumerate(PHASES)},
            "workspace_bytes": int(self.workspace_bytes),
        }


class Metrics(C.Structure):
    _fields_ = [(f, C.c_double) for f in (
        "fro2", "captured_fro2", "resid_fro", "resid_spec", "fro_ratio", "spec_ratio",
        "per_vector")]

    def as_dict(self) -> dict:
        return {f: float(getattr(self, f)) for f, _ in self._fields_}


class BKError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


class RankDeficient(BKError):
    pass


_lib = None

# (name, restype, argtypes)
_P, _I64, _I32, _U64, _D, _SZ = (C.c_void_p, C.c_int64, C.c_int32, C.c_uint64,
                                 C.c_double, C.c_size_t)
_SIGS = [
    ("bk_status_string", C.c_char_p, [C.c_int]),
    ("bk_version", C.c_char_p, []),
    ("bk_svd_dense_workspace", _SZ, [_I64, _I64, _I32, _I32, _I32, _P]),
    ("bk_svd_dense", C.c_int, [_P, _I64, _I32, _P, _P, _I64, _I64, _I64, _I32, _I32, _U64,
                               _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    ("bk_svd_dense_noalloc", C.c_int, [_P, _I64, _I32, _P, _P, _I64, _I64, _I64, _I32, _I32,
                                       _U64, _P, _P, _I64, _P, _P, _P]),
    ("bk_svd_csr_workspace", _SZ, [_I64, _I64, _I64, _I32, _I32, _P]),
    ("bk_svd_csr", C.c_int, [_P, _P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _I32, _U64,
                             _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    ("bk_error_metrics_dense_workspace", _SZ, [_I64, _I64, _I32, _I32, _I32]),
    ("bk_error_metrics_dense", C.c_int, [_P, _I64, _I32, _I64, _I64, _P, _I64, _I32, _I32,
                                         _U64, _P, _I64, _P, _P, _P, _SZ, _P]),
    ("bk_error_metrics_csr_workspace", _SZ, [_I64, _I64, _I64, _I32, _I32]),
    ("bk_error_metrics_csr", C.c_int, [_P, _P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _P,
                                       _I64, _I32, _I32, _U64, _P, _I64, _P, _P, _P, _SZ,
                                       _P]),
    ("bk_svd_dense_backward_workspace", _SZ, [_I64, _I64, _I32, _I32, _I32]),
    ("bk_svd_dense_backward", C.c_int, [_P, _I64, _I32, _I64, _I64, _I32, _I32, _P, _I64, _P,
                                        _P, _P, _P, _I64, _P, _SZ, _P, _SZ, _P]),
    ("bk_gaussian", C.c_int, [_U64, _I64, _I64, _I64, _I32, _P, _P]),
    ("bk_philox4x32_10", C.c_int, [_P, _I64, _P, _P]),
    ("bk_quantize_dense", C.c_int, [_P, _I64, _I64, _I64, _I32, _P, _P, _P]),
    ("bk_quantize_dense_transposed", C.c_int, [_P, _I64, _I64, _I64, _I32, _P, _P, _P]),
    ("bk_dense_product_workspace", _SZ, [_I32, _I64, _I64, _I32, _I32]),
    ("bk_dense_product", C.c_int, [_I32, _P, _I64, _I32, _P, _I64, _I64, _P, _I64, _I32, _P,
                                   _I64, _P, _SZ, _P]),
    ("bk_csr_product", C.c_int, [_P, _P, _P, _I64, _I64, _I64, _P, _I64, _I32, _P, _I64, _P]),
    ("bk_csr_transpose_workspace", _SZ, [_I64, _I64, _I64]),
    ("bk_csr_transpose", C.c_int, [_P, _P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _SZ, _P]),
    ("bk_eigh_psd_workspace", _SZ, [_I64]),
    ("bk_eigh_psd", C.c_int, [_P, _I64, _I64, _P, _P, _I64, _I32, _D, _P, _P, _SZ, _P]),
]

EXPORTS = tuple(name for name, _, _ in _SIGS)


def load(path: str | None = None):
    """Load libbk.so (or the build named by BK_LIBRARY, e.g. the host-
    sanitized one); raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or os.environ.get("BK_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(
            f"{p} is missing: build the HIP library first "
            "(python -m paper_1504_05477_amd.build); there is no CPU fallback")
    lib = C.CDLL(p)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().bk_status_string(status).decode()
    except ImportError:
        return "library not loaded"


def check(status: int, what: str) -> None:
    if status == OK:
        return
    if status == ERANK:
        raise RankDeficient(status, what)
    raise BKError(status, what)
