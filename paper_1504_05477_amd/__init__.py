"""Randomized Block Krylov Iteration (Musco & Musco, Algorithm 2) on the AMD
MI355X (gfx950): a HIP library (libbk.so, C ABI in include/bk.h) and this thin
torch binding.  Build the library with ``python -m paper_1504_05477_amd.build``.
"""
from ._lib import (BKError, RankDeficient, EXPORTS, LIB_PATH, load,
                   status_string)
from .api import (BKSVD, Metrics, SVDResult, csr_product, svd_dense_backward, csr_transpose,
                  dense_product, eigh_psd, error_metrics_csr, error_metrics_dense, gaussian,
                  philox, quantize, svd_csr, svd_dense)

__all__ = [
    "BKError", "RankDeficient", "EXPORTS", "LIB_PATH", "load", "status_string",
    "BKSVD", "Metrics", "SVDResult", "error_metrics_csr", "error_metrics_dense", "svd_dense_backward", "csr_product", "csr_transpose", "dense_product", "eigh_psd",
    "gaussian", "philox", "quantize", "svd_csr", "svd_dense",
]
