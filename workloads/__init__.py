"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs (matrices with planted spectra, term-document
CSR matrices, explicit Gaussian sketches for the explicit-Pi option).  It holds
none of the Block Krylov arithmetic: both the CPU oracle and the GPU library
consume what it produces, and neither is imported here.

Workload recipes (the paper's datasets -- SNAP/amazon0302, SNAP/email-Enron,
20 Newsgroups, Section 7 -- are not available; these stand in for them):

* ``dense1``  2000 x 1000, sigma_i = i^-1/2, k=10, q=8, FP64.  The gap
  sigma_10/sigma_11 - 1 = .049 is close to email-Enron's .042 (Section 7).
* ``csr2``    11000 x 130000 term-document CSR, ~1.5M nonzeros, row lengths
  log-normal (median 90, mean 136.4), column ids Zipf(1.1) through a seeded
  permutation, values log(1+tf)*idf, implicit row centering; k=20, q=10.  Shape
  of the 20 Newsgroups matrix the paper times (Section 7, k = 20).
* ``dense3``  65536 x 16384, sigma_i = exp(-i/200) + 1e-3, + 1e-4 N(0,1) noise,
  k=100, q=12, FP32 master + BF16 copy.  Gap .0050 (amazon0302: .004).
* ``dense4``  8192 x 4096, sigma_i = 1/i, k=32, q=10 (differentiation).
* ``dense5``  131072 x 32768, sigma_i = i^-0.8, k=256, q=8, FP8 copy + FP32
  master.

Seeds: matrix ``100 + cfg``, sketch ``200 + cfg``, noise ``300 + cfg``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "spectrum", "planted_dense", "planted_dense_torch",
    "term_document_csr", "gaussian_sketch", "low_rank_dense", "scaled",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int
    n: int
    d: int
    k: int
    q: int
    kind: str            # "dense" or "csr"
    spectrum: str        # key into spectrum()
    dtype: str           # storage/compute type of the plain path
    noise: float = 0.0   # iid N(0, noise^2) added after planting
    center: bool = False

    @property
    def m(self) -> int:
        return (self.q + 1) * self.k

    @property
    def seed_matrix(self) -> int:
        return 100 + self.cfg

    @property
    def seed_sketch(self) -> int:
        return 200 + self.cfg

    @property
    def seed_noise(self) -> int:
        return 300 + self.cfg


WORKLOADS = {
    "dense1": Workload("dense1", 1, 2000, 1000, 10, 8, "dense", "inv_sqrt", "f64"),
    "csr2": Workload("csr2", 2, 11000, 130000, 20, 10, "csr", "termdoc", "f32",
                     center=True),
    "dense3": Workload("dense3", 3, 65536, 16384, 100, 12, "dense", "exp200",
                       "f32", noise=1e-4),
    "dense4": Workload("dense4", 4, 8192, 4096, 32, 10, "dense", "inv", "f32"),
    "dense5": Workload("dense5", 5, 131072, 32768, 256, 8, "dense", "pow08",
                       "f32"),
}


def scaled(w: Workload, n: int, d: int, k: int | None = None,
           q: int | None = None) -> Workload:
    """Same recipe at a smaller shape (for tests the oracle finishes quickly)."""
    return dataclasses.replace(w, n=n, d=d, k=w.k if k is None else k,
                               q=w.q if q is None else q)


def spectrum(kind: str, r: int) -> np.ndarray:
    """Planted singular values sigma_1 >= ... >= sigma_r (float64)."""
    i = np.arange(1, r + 1, dtype=np.float64)
    if kind == "inv_sqrt":
        return i ** -0.5
    if kind == "inv":
        return 1.0 / i
    if kind == "exp200":
        return np.exp(-i / 200.0) + 1e-3
    if kind == "pow08":
        return i ** -0.8
    raise ValueError(f"unknown spectrum {kind!r}")


def _orthonormal_np(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    g = rng.standard_normal((rows, cols))
    qm, rm = np.linalg.qr(g)
    # make the factor unique (positive diagonal of R) so it is a fixed function of the seed
    s = np.sign(np.diag(rm))
    s[s == 0] = 1.0
    return qm * s


def planted_dense(n: int, d: int, sigma: np.ndarray, seed: int,
                  noise: float = 0.0, noise_seed: int | None = None) -> np.ndarray:
    """A = U diag(sigma) V^T in float64 on the host.

    U (n x r) and V (d x r), r = min(n, d), are the Q factors of seeded N(0,1)
    matrices.  ``sigma`` may be shorter than r (rank-deficient A)."""
    r = min(n, d)
    sig = np.zeros(r)
    sig[: len(sigma)] = sigma[:r]
    rng = np.random.default_rng(seed)
    u = _orthonormal_np(rng, n, r)
    v = _orthonormal_np(rng, d, r)
    a = (u * sig) @ v.T
    if noise:
        nr = np.random.default_rng(noise_seed if noise_seed is not None else seed + 200)
        a += noise * nr.standard_normal((n, d))
    return a


def low_rank_dense(n: int, d: int, rank: int, seed: int) -> np.ndarray:
    """Exactly rank-``rank`` planted matrix with sigma_i = 1/i (float64)."""
    return planted_dense(n, d, 1.0 / np.arange(1, rank + 1), seed)


# Factors of at least 2^31 entries are not handed to one library QR (its
# 32-bit indexing does not reach them); they are built row block by row
# block instead.
_BIG = 1 << 31
_ROWBLK = 8192


def _gaussian_rows(rows, cols, g, device, rowblk=None):
    """rows x cols N(0,1) FP64 drawn from generator g in row blocks."""
    import torch

    rb = rowblk or _ROWBLK
    x = torch.empty(rows, cols, dtype=torch.float64, device=device)
    for r0 in range(0, rows, rb):
        r1 = min(rows, r0 + rb)
        x[r0:r1] = torch.randn(r1 - r0, cols, generator=g, device=device,
                               dtype=torch.float64)
    return x


def _cholqr2_rows(x, rowblk=None):
    """In place: x <- its Q factor (positive diagonal of R) by CholeskyQR2 in
    FP64: with G = X^T X = R^T R (Cholesky), Q = X R^-1, repeated once on
    Q.  In exact arithmetic this is the Householder Q made unique by
    diag(R) > 0; a Gaussian matrix with rows >= 2 cols is well conditioned,
    so two passes reach FP64 orthogonality.  Every library call sees at most
    rowblk x cols entries (Grams accumulated over row blocks)."""
    import torch

    rb = rowblk or _ROWBLK
    rows, cols = x.shape
    for _ in range(2):
        gram = torch.zeros(cols, cols, dtype=torch.float64, device=x.device)
        for r0 in range(0, rows, rb):
            blk = x[r0:min(rows, r0 + rb)]
            gram += blk.t() @ blk
        rfac = torch.linalg.cholesky(gram, upper=True)
        del gram
        for r0 in range(0, rows, rb):
            r1 = min(rows, r0 + rb)
            x[r0:r1] = torch.linalg.solve_triangular(rfac, x[r0:r1], upper=True, left=False)
        del rfac
    return x


def _orth_blocked(rows, cols, g, device):
    """Q factor of a seeded N(0,1) rows x cols matrix for factors too large
    for one library QR: drawn in row blocks, orthonormalized by CholeskyQR2."""
    return _cholqr2_rows(_gaussian_rows(rows, cols, g, device))


def planted_dense_torch(n: int, d: int, sigma, seed: int, device="cuda",
                        out_dtype=None, noise: float = 0.0,
                        noise_seed: int | None = None, return_factors=False,
                        stats: dict | None = None):
    """A = U diag(sigma) V^T built with torch on ``device`` (for large shapes).

    U and V are Q factors of seeded N(0,1) matrices (FP64 QR, made unique by a
    positive diagonal of R); the product is formed in FP64 row block by row
    block and stored as ``out_dtype`` (default float32).  Returns A, and also
    (U, sigma, V) in FP64 when ``return_factors``.  ``stats``, when given,
    receives "storage_rounding_fro": ||A_stored - A_FP64||_F, the Frobenius
    norm of what storing the FP64 product (noise included) in ``out_dtype``
    changed (a bound on how far the stored matrix's singular values are from
    the planted ones, Weyl)."""
    import torch

    out_dtype = torch.float32 if out_dtype is None else out_dtype
    r = min(n, d)
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def orth(rows, cols):
        if rows * cols < _BIG:
            x = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float64)
            qm, rm = torch.linalg.qr(x)
            s = torch.sign(torch.diagonal(rm))
            s[s == 0] = 1
            del rm, x
            return qm * s
        return _orth_blocked(rows, cols, g, device)

    u = orth(n, r)
    v = orth(d, r)
    sig = torch.zeros(r, dtype=torch.float64, device=device)
    sv = torch.as_tensor(np.asarray(sigma, dtype=np.float64)[:r], device=device)
    sig[: sv.numel()] = sv
    a = torch.empty(n, d, dtype=out_dtype, device=device)
    vt = v.t().contiguous()
    gn = None
    if noise:
        gn = torch.Generator(device=device)
        gn.manual_seed(noise_seed if noise_seed is not None else seed + 200)
    rb = 8192
    rnd2 = 0.0
    for r0 in range(0, n, rb):
        r1 = min(n, r0 + rb)
        blk = (u[r0:r1] * sig) @ vt
        if noise:
            blk += noise * torch.randn(r1 - r0, d, generator=gn, device=device,
                                       dtype=torch.float64)
        a[r0:r1] = blk.to(out_dtype)
        if stats is not None:
            rnd2 += float(((a[r0:r1].to(torch.float64) - blk) ** 2).sum())
        del blk
    if stats is not None:
        stats["storage_rounding_fro"] = math.sqrt(rnd2)
    if return_factors:
        return a, (u, sig, v)
    del u, v, vt
    return a


def term_document_csr(n: int, d: int, seed: int, median_len: float = 90.0,
                      ln_sigma: float = 0.912, zipf_s: float = 1.1,
                      tf_p: float = 0.6):
    """Term-document-like CSR matrix (rows = documents, columns = terms).

    * row length L_r = clamp(round(LogNormal(ln median, ln_sigma)), 1, d);
    * L_r distinct term ranks drawn from Zipf(zipf_s) truncated to 1..d, mapped
      to column ids through a seeded permutation (hot terms are scattered);
    * tf ~ Geometric(tf_p) on {1, 2, ...}, df_j = #rows containing term j,
      value = ln(1 + tf) * ln(n / df_j) in float32 (zeros, when df_j = n, are
      kept as stored entries).

    Returns (row_ptr int32[n+1], col_idx int32[nnz], vals float32[nnz]); the
    column ids are sorted ascending within each row."""
    rng = np.random.default_rng(seed)
    lens = np.rint(rng.lognormal(math.log(median_len), ln_sigma, size=n))
    lens = np.clip(lens, 1, d).astype(np.int64)
    ranks = np.arange(1, d + 1, dtype=np.float64)
    pmf = ranks ** -zipf_s
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    perm = rng.permutation(d).astype(np.int64)
    cols = []
    for r in range(n):
        want = int(lens[r])
        got = np.empty(0, dtype=np.int64)
        draw = max(2 * want, 16)
        while True:
            u = rng.random(draw)
            cand = np.minimum(np.searchsorted(cdf, u, side="right"), d - 1)
            allc = np.concatenate([got, cand])
            uniq, first = np.unique(allc, return_index=True)
            if len(uniq) >= want:
                order = np.argsort(first, kind="stable")[:want]
                got = uniq[order]
                break
            got = uniq[np.argsort(first, kind="stable")]
            draw *= 2
        cols.append(np.sort(perm[got]))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(lens)
    col_idx = np.concatenate(cols)
    tf = rng.geometric(tf_p, size=col_idx.size).astype(np.float64)
    df = np.bincount(col_idx, minlength=d).astype(np.float64)
    idf = np.zeros(d)
    nzc = df > 0
    idf[nzc] = np.log(n / df[nzc])
    vals = (np.log1p(tf) * idf[col_idx]).astype(np.float32)
    return row_ptr.astype(np.int32), col_idx.astype(np.int32), vals


def gaussian_sketch(d: int, k: int, seed: int) -> np.ndarray:
    """An explicit d x k N(0,1) sketch from NumPy's PCG64 (float64).

    Used for the explicit-sketch option, where the same matrix is handed to
    both the oracle and the GPU library instead of each drawing it from the
    seed with its own counter-based generator."""
    return np.random.default_rng(seed).standard_normal((d, k))
