"""Python binding of the Block Krylov library (torch tensors in, torch tensors
out).  Every function only marshals arguments to libbk.so; all arithmetic
runs in the HIP kernels.  torch provides device memory and the stream."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU (device 'cuda')")


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return L.F64
    if t.dtype == torch.float32:
        return L.F32
    if t.dtype == torch.bfloat16:
        return L.BF16
    if t.dtype == torch.uint8 or str(t.dtype).startswith("torch.float8_e4m3fn"):
        return L.FP8_E4M3
    raise TypeError(f"unsupported matrix dtype {t.dtype}")


_METHODS = {"bki": 0, "block_krylov": 0, "si": 1, "simultaneous": 1, "lanczos": 2,
            "block_lanczos": 2}


def _options(*, refine=0, center=False, max_sweeps=0, jacobi_tol=0.0,
             breakdown_tol=0.0, pi=None, timing=False, save=False,
             jacobi_block=0, block_size=0, method="bki", residuals=None,
             A_t=None, at_scales=None, fp32_products="limbs",
             csr_gather="default") -> L.Options:
    """timing: False, True (every phase) or an iterable of phase names from
    _lib.PHASES (only those get events; launch counts are kept for all)."""
    o = L.Options()
    o.struct_size = C.sizeof(L.Options)
    o.refine = int(refine)
    o.center_rows = int(bool(center))
    o.max_jacobi_sweeps = int(max_sweeps)
    o.jacobi_tol = float(jacobi_tol)
    o.breakdown_tol = float(breakdown_tol)
    o.pi = _ptr(pi)
    if timing is True or timing is False or timing is None:
        o.timing = int(bool(timing))
        o.timing_phases = 0
    else:
        names = list(timing)
        bad = [p for p in names if p not in L.PHASES]
        if bad:
            raise ValueError(f"unknown phases {bad}; known: {L.PHASES}")
        o.timing = 1
        o.timing_phases = sum(1 << L.PHASES.index(p) for p in set(names))
    o.save_for_backward = int(bool(save))
    o.jacobi_block = int(jacobi_block)
    o.block_size = int(block_size or 0)
    if method not in _METHODS:
        raise ValueError(f"method must be one of {sorted(_METHODS)}")
    o.method = _METHODS[method]
    o.residuals = _ptr(residuals)
    o.a_transposed = _ptr(A_t)
    o.ld_at = 0 if A_t is None else A_t.stride(0)
    o.at_scales = _ptr(at_scales)
    if fp32_products not in ("limbs", "cores"):
        raise ValueError("fp32_products must be 'limbs' or 'cores'")
    o.fp32_products = 1 if fp32_products == "cores" else 0
    gathers = {"default": 0, "inplace": 1, "staged": 2}
    if csr_gather not in gathers:
        raise ValueError(f"csr_gather must be one of {sorted(gathers)}")
    o.csr_gather = gathers[csr_gather]
    return o


@dataclass
class SVDResult:
    Z: torch.Tensor          # n x k orthonormal Ritz vectors
    sigma: torch.Tensor      # k Ritz values (FP64), descending
    info: dict
    workspace: torch.Tensor | None = None   # forward state (save_for_backward)
    residuals: torch.Tensor | None = None   # k FP64 ||A A^T z_i - sigma_i^2 z_i||


def svd_dense(A: torch.Tensor, k: int, q: int, seed: int = 0, *, a_scales=None,
              A_master=None, refine: int = 0, pi=None, timing=False,
              save_for_backward=False, max_sweeps=0, jacobi_tol=0.0,
              breakdown_tol=0.0, jacobi_block=0, block_size=0, method="bki",
              residuals=False, A_t=None, at_scales=None, fp32_products="limbs",
              stream=None) -> SVDResult:
    """Block Krylov Iteration on a dense A (n x d row-major on the GPU).

    A's dtype selects the path: float64 / float32 (plain), bfloat16, or uint8
    holding OCP e4m3 codes with ``a_scales`` (FP8).  Returns Z (n x k, FP64 for
    the FP64 path, FP32 otherwise) and the Ritz values (FP64).
    ``block_size`` = p >= k oversamples the sketch (0: p = k);
    ``method`` = "si" runs Simultaneous Iteration instead.
    ``residuals`` also returns ||A A^T z_i - sigma_i^2 z_i|| per Ritz pair
    (A: the FP32 master after the correction pass).
    ``A_t`` (with ``at_scales`` for FP8): the BF16 / FP8 copy stored
    transposed (``quantize(..., transposed=True)``); the A^T Y products then
    read it row by row.  ``fp32_products``: "limbs" (FP32 operands as three
    BF16 limbs on the BF16 matrix cores) or "cores" (the FP32 matrix
    cores)."""
    lib = L.load()
    _need_cuda(A, a_scales, A_master, pi, A_t, at_scales)
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    n, d = A.shape
    code = _dtype_code(A)
    if A_t is not None:
        if (tuple(A_t.shape) != (d, n) or A_t.stride(1) != 1
                or A_t.element_size() != A.element_size()):
            raise ValueError("A_t must be the row-major d x n transposed copy in A's dtype")
    if code == L.FP8_E4M3 and A.dtype != torch.uint8:
        A = A.view(torch.uint8)
    zdt = torch.float64 if code == L.F64 else torch.float32
    if pi is not None:
        pi = pi.to(zdt).contiguous()
    if A_master is not None and (A_master.dtype != torch.float32 or A_master.stride(1) != 1):
        raise ValueError("A_master must be a row-major float32 tensor")
    res_t = torch.empty(k, dtype=torch.float64, device=A.device) if residuals else None
    opt = _options(refine=refine, pi=pi, timing=timing, save=save_for_backward,
                   max_sweeps=max_sweeps, jacobi_tol=jacobi_tol,
                   breakdown_tol=breakdown_tol, jacobi_block=jacobi_block,
                   block_size=block_size, method=method, residuals=res_t,
                   A_t=A_t, at_scales=at_scales, fp32_products=fp32_products)
    nbytes = lib.bk_svd_dense_workspace(n, d, k, q, code, C.byref(opt))
    if nbytes == 0:
        raise ValueError(f"invalid shape/rank: n={n} d={d} k={k} q={q}")
    ws = _ws(nbytes, A.device)
    Z = torch.empty(n, k, dtype=zdt, device=A.device)
    sig = torch.empty(k, dtype=torch.float64, device=A.device)
    info = L.Info()
    st = lib.bk_svd_dense(_ptr(A), A.stride(0), code, _ptr(a_scales), _ptr(A_master),
                          0 if A_master is None else A_master.stride(0), n, d, k, q,
                          int(seed) & (2**64 - 1), C.byref(opt), _ptr(Z), Z.stride(0),
                          _ptr(sig), C.byref(info), _ptr(ws), nbytes, _stream(stream))
    L.check(st, "bk_svd_dense")
    return SVDResult(Z, sig, info.as_dict(), ws if save_for_backward else None, res_t)


def svd_dense_backward(A: torch.Tensor, k: int, q: int, fwd: SVDResult, Z_bar=None,
                       sigma_bar=None, stream=None) -> torch.Tensor:
    """Gradient of a loss L(Z, sigma) with respect to A (FP32 / FP64 plain
    paths), for a forward run with ``save_for_backward=True``.  The loss must
    be unchanged by rotations inside span(Z) (e.g. sum of the Ritz values,
    ||Z Z^T A||_F^2 through Z)."""
    lib = L.load()
    if fwd.workspace is None:
        raise ValueError("the forward must be run with save_for_backward=True")
    code = _dtype_code(A)
    if code not in (L.F64, L.F32):
        raise ValueError("the adjoint covers the FP32 and FP64 paths")
    n, d = A.shape
    zdt = torch.float64 if code == L.F64 else torch.float32
    if Z_bar is not None:
        Z_bar = Z_bar.to(zdt).contiguous()
        _need_cuda(Z_bar)
    if sigma_bar is not None:
        sigma_bar = sigma_bar.to(torch.float64).contiguous()
        _need_cuda(sigma_bar)
    A_bar = torch.empty(n, d, dtype=A.dtype, device=A.device)
    nbytes = lib.bk_svd_dense_backward_workspace(n, d, k, q, code)
    ws = _ws(nbytes, A.device)
    st = lib.bk_svd_dense_backward(_ptr(A), A.stride(0), code, n, d, k, q, _ptr(fwd.Z), k,
                                   _ptr(fwd.sigma), _ptr(Z_bar), _ptr(sigma_bar), _ptr(A_bar),
                                   A_bar.stride(0), _ptr(fwd.workspace),
                                   fwd.workspace.numel(), _ptr(ws), nbytes, _stream(stream))
    L.check(st, "bk_svd_dense_backward")
    return A_bar


class BKSVD(torch.autograd.Function):
    """(Z, sigma) = BKSVD.apply(A, k, q, seed): differentiable Block Krylov
    Iteration on a dense FP32 / FP64 A.  The backward is the library's adjoint
    (Krylov blocks recomputed from the saved orthonormal blocks); it is exact
    for losses invariant under rotations inside span(Z)."""

    @staticmethod
    def forward(ctx, A, k: int, q: int, seed: int = 0):
        A = A.contiguous()
        res = svd_dense(A, k, q, seed, save_for_backward=True)
        # The outputs go through save_for_backward (version-checked: an
        # in-place change to Z or sigma before backward raises), and ctx
        # holds only the forward workspace, not the outputs, so there is no
        # output -> grad_fn -> ctx -> output cycle keeping the workspace alive.
        ctx.save_for_backward(A, res.Z, res.sigma)
        ctx.workspace = res.workspace
        ctx.info = res.info
        ctx.kq = (k, q)
        return res.Z, res.sigma

    @staticmethod
    def backward(ctx, Z_bar, sigma_bar):
        A, Z, sigma = ctx.saved_tensors
        k, q = ctx.kq
        fwd = SVDResult(Z, sigma, ctx.info, ctx.workspace)
        A_bar = svd_dense_backward(A, k, q, fwd, Z_bar, sigma_bar)
        ctx.workspace = None
        return A_bar, None, None, None


def svd_csr(row_ptr, col_idx, vals, n: int, d: int, k: int, q: int, seed: int = 0, *,
            transpose=None, center=False, pi=None, timing=False, max_sweeps=0,
            jacobi_tol=0.0, breakdown_tol=0.0, jacobi_block=0, block_size=0,
            method="bki", residuals=False, csr_gather="default",
            stream=None) -> SVDResult:
    """Block Krylov Iteration on a CSR A (int32 row_ptr / col_idx, float32
    values, on the GPU).  ``transpose`` = (t_row_ptr, t_col_idx, t_vals) of A^T
    is optional; ``center`` applies implicit row centring; ``residuals`` as
    svd_dense (of the centred matrix with ``center``; needs block_size k);
    ``csr_gather``: "inplace" (gathers from the Krylov block), "staged" (from
    a copy with 128-byte-aligned rows) or "default"."""
    lib = L.load()
    _need_cuda(row_ptr, col_idx, vals, pi)
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (vals, torch.float32)):
        if t.dtype != dt or not t.is_contiguous():
            raise ValueError("CSR arrays must be contiguous int32/int32/float32")
    nnz = col_idx.numel()
    tr = transpose or (None, None, None)
    if pi is not None:
        pi = pi.to(torch.float32).contiguous()
    res_t = (torch.empty(k, dtype=torch.float64, device=row_ptr.device) if residuals
             else None)
    opt = _options(center=center, pi=pi, timing=timing, max_sweeps=max_sweeps,
                   jacobi_tol=jacobi_tol, breakdown_tol=breakdown_tol,
                   jacobi_block=jacobi_block, block_size=block_size, method=method,
                   residuals=res_t, csr_gather=csr_gather)
    nbytes = lib.bk_svd_csr_workspace(n, d, nnz, k, q, C.byref(opt))
    if nbytes == 0:
        raise ValueError(f"invalid shape/rank: n={n} d={d} k={k} q={q}")
    ws = _ws(nbytes, row_ptr.device)
    Z = torch.empty(n, k, dtype=torch.float32, device=row_ptr.device)
    sig = torch.empty(k, dtype=torch.float64, device=row_ptr.device)
    info = L.Info()
    st = lib.bk_svd_csr(_ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(tr[0]), _ptr(tr[1]),
                        _ptr(tr[2]), n, d, nnz, k, q, int(seed) & (2**64 - 1), C.byref(opt),
                        _ptr(Z), Z.stride(0), _ptr(sig), C.byref(info), _ptr(ws), nbytes,
                        _stream(stream))
    L.check(st, "bk_svd_csr")
    return SVDResult(Z, sig, info.as_dict(), None, res_t)


@dataclass
class Metrics:
    """Error measures of a basis Z (Section 3): the raw norms and, with the
    true singular values, the ratios of eqs. (1)-(3)."""
    values: dict
    captured: torch.Tensor  # k FP64 (CPU): z_i^T Abar Abar^T z_i
    status: int


def _sigma_host(sigma_true):
    if sigma_true is None:
        return None, 0, None
    s = torch.as_tensor(sigma_true, dtype=torch.float64).detach().cpu().contiguous()
    return s, s.numel(), C.cast(s.data_ptr(), C.c_void_p)


def _finish_metrics(st, what, m, cap) -> Metrics:
    if st not in (L.OK, L.ERANK):
        L.check(st, what)
    return Metrics(m.as_dict(), cap, st)


def error_metrics_dense(A: torch.Tensor, Z: torch.Tensor, sigma_true=None, q_spec: int = 4,
                        seed: int = 0, stream=None) -> Metrics:
    """Error measures of Z (n x k, orthonormal columns, A's dtype) against a
    dense FP32 / FP64 A on the GPU; ``sigma_true`` (k+1 or more values,
    descending) enables the ratios."""
    lib = L.load()
    _need_cuda(A, Z)
    if A.dim() != 2 or A.stride(1) != 1 or Z.dim() != 2 or Z.stride(1) != 1:
        raise ValueError("A and Z must be row-major 2-D tensors")
    if Z.dtype != A.dtype:
        raise TypeError("Z must have A's dtype")
    n, d = A.shape
    k = Z.shape[1]
    code = _dtype_code(A)
    nbytes = lib.bk_error_metrics_dense_workspace(n, d, k, q_spec, code)
    if nbytes == 0:
        raise ValueError(f"invalid shape/type: n={n} d={d} k={k} q_spec={q_spec} {A.dtype}")
    ws = _ws(nbytes, A.device)
    sig, ns, sp = _sigma_host(sigma_true)
    cap = torch.empty(k, dtype=torch.float64)
    m = L.Metrics()
    st = lib.bk_error_metrics_dense(_ptr(A), A.stride(0), code, n, d, _ptr(Z), Z.stride(0), k,
                                    q_spec, int(seed) & (2**64 - 1), sp, ns,
                                    C.cast(cap.data_ptr(), C.c_void_p), C.byref(m), _ptr(ws),
                                    nbytes, _stream(stream))
    return _finish_metrics(st, "bk_error_metrics_dense", m, cap)


def error_metrics_csr(row_ptr, col_idx, vals, n: int, d: int, Z: torch.Tensor,
                      sigma_true=None, q_spec: int = 4, seed: int = 0, *, center=False,
                      transpose=None, stream=None) -> Metrics:
    """Error measures of an FP32 Z (n x k) against a CSR A (or its row-centred
    form with ``center``) on the GPU."""
    lib = L.load()
    _need_cuda(row_ptr, col_idx, vals, Z)
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (vals, torch.float32)):
        if t.dtype != dt or not t.is_contiguous():
            raise ValueError("CSR arrays must be contiguous int32/int32/float32")
    if Z.dtype != torch.float32 or Z.dim() != 2 or Z.stride(1) != 1:
        raise ValueError("Z must be a row-major float32 n x k tensor")
    nnz = col_idx.numel()
    k = Z.shape[1]
    tr = transpose or (None, None, None)
    nbytes = lib.bk_error_metrics_csr_workspace(n, d, nnz, k, q_spec)
    if nbytes == 0:
        raise ValueError(f"invalid shape: n={n} d={d} k={k} q_spec={q_spec}")
    ws = _ws(nbytes, row_ptr.device)
    sig, ns, sp = _sigma_host(sigma_true)
    cap = torch.empty(k, dtype=torch.float64)
    m = L.Metrics()
    st = lib.bk_error_metrics_csr(_ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(tr[0]),
                                  _ptr(tr[1]), _ptr(tr[2]), n, d, nnz, 1 if center else 0,
                                  _ptr(Z), Z.stride(0), k, q_spec, int(seed) & (2**64 - 1), sp,
                                  ns, C.cast(cap.data_ptr(), C.c_void_p), C.byref(m), _ptr(ws),
                                  nbytes, _stream(stream))
    return _finish_metrics(st, "bk_error_metrics_csr", m, cap)


def gaussian(seed: int, rows: int, cols: int, dtype=torch.float32, device="cuda",
             stream=None) -> torch.Tensor:
    """The Philox4x32-10 / Box-Muller sketch (see bk_gaussian)."""
    lib = L.load()
    out = torch.empty(rows, cols, dtype=dtype, device=device)
    code = L.F64 if dtype == torch.float64 else L.F32
    L.check(lib.bk_gaussian(int(seed) & (2**64 - 1), rows, cols, cols, code, _ptr(out),
                            _stream(stream)), "bk_gaussian")
    return out


def philox(ctr_key: torch.Tensor, stream=None) -> torch.Tensor:
    """Raw Philox4x32-10 words: ctr_key int32/uint32 (count x 6) -> (count x 4)."""
    lib = L.load()
    _need_cuda(ctr_key)
    x = ctr_key.contiguous()
    out = torch.empty(x.shape[0], 4, dtype=x.dtype, device=x.device)
    L.check(lib.bk_philox4x32_10(_ptr(x), x.shape[0], _ptr(out), _stream(stream)),
            "bk_philox4x32_10")
    return out


def quantize(A: torch.Tensor, to: str, stream=None, transposed: bool = False):
    """A float32 (n x d) -> ("bf16": bfloat16 copy) or ("fp8": (uint8 e4m3
    codes, float32 tile scales ceil(n/128) x ceil(d/128))).  ``transposed``
    returns the same codes stored as A^T (d x n; FP8 scales ceil(d/128) x
    ceil(n/128)), for ``svd_dense(..., A_t=...)``."""
    lib = L.load()
    _need_cuda(A)
    if A.dtype != torch.float32 or A.stride(1) != 1:
        raise ValueError("A must be a row-major float32 tensor")
    n, d = A.shape
    fn = lib.bk_quantize_dense_transposed if transposed else lib.bk_quantize_dense
    name = "bk_quantize_dense_transposed" if transposed else "bk_quantize_dense"
    rows, cols = (d, n) if transposed else (n, d)
    if to == "bf16":
        out = torch.empty(rows, cols, dtype=torch.bfloat16, device=A.device)
        L.check(fn(_ptr(A), n, d, A.stride(0), L.BF16, _ptr(out), None, _stream(stream)), name)
        return out
    if to == "fp8":
        out = torch.empty(rows, cols, dtype=torch.uint8, device=A.device)
        sc = torch.empty((rows + 127) // 128, (cols + 127) // 128, dtype=torch.float32,
                         device=A.device)
        L.check(fn(_ptr(A), n, d, A.stride(0), L.FP8_E4M3, _ptr(out), _ptr(sc),
                   _stream(stream)), name)
        return out, sc
    raise ValueError("to must be 'bf16' or 'fp8'")


def dense_product(A: torch.Tensor, X: torch.Tensor, trans: bool = False, a_scales=None,
                  stream=None) -> torch.Tensor:
    """Y = A X (trans False) or A^T X (trans True) with the library's kernels."""
    lib = L.load()
    _need_cuda(A, X, a_scales)
    code = _dtype_code(A)
    if code == L.FP8_E4M3 and A.dtype != torch.uint8:
        A = A.view(torch.uint8)
    n, d = A.shape
    k = X.shape[1]
    wdt = torch.float64 if code == L.F64 else torch.float32
    X = X.to(wdt)
    if X.stride(1) != 1:
        X = X.contiguous()
    Y = torch.empty(d if trans else n, k, dtype=wdt, device=A.device)
    nbytes = lib.bk_dense_product_workspace(int(trans), n, d, k, code)
    ws = _ws(nbytes, A.device)
    L.check(lib.bk_dense_product(int(trans), _ptr(A), A.stride(0), code, _ptr(a_scales), n,
                                 d, _ptr(X), X.stride(0), k, _ptr(Y), Y.stride(0), _ptr(ws),
                                 nbytes, _stream(stream)), "bk_dense_product")
    return Y


def csr_product(row_ptr, col_idx, vals, cols: int, X: torch.Tensor, stream=None):
    """Y = A X for a CSR A (rows = row_ptr.numel() - 1)."""
    lib = L.load()
    rows = row_ptr.numel() - 1
    X = X.to(torch.float32).contiguous()
    k = X.shape[1]
    Y = torch.empty(rows, k, dtype=torch.float32, device=X.device)
    L.check(lib.bk_csr_product(_ptr(row_ptr), _ptr(col_idx), _ptr(vals), rows, cols,
                               col_idx.numel(), _ptr(X), k, k, _ptr(Y), k, _stream(stream)),
            "bk_csr_product")
    return Y


def csr_transpose(row_ptr, col_idx, vals, cols: int, stream=None):
    """CSR of A^T (column ids ascending within rows)."""
    lib = L.load()
    rows = row_ptr.numel() - 1
    nnz = col_idx.numel()
    dev = row_ptr.device
    trp = torch.empty(cols + 1, dtype=torch.int32, device=dev)
    tci = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
    tv = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)[:nnz]
    nbytes = lib.bk_csr_transpose_workspace(rows, cols, nnz)
    ws = _ws(nbytes, dev)
    L.check(lib.bk_csr_transpose(_ptr(row_ptr), _ptr(col_idx), _ptr(vals), rows, cols, nnz,
                                 _ptr(trp), _ptr(tci), _ptr(tv), _ptr(ws), nbytes,
                                 _stream(stream)), "bk_csr_transpose")
    return trp, tci, tv


def eigh_psd(M: torch.Tensor, max_sweeps: int = 0, tol: float = 0.0, stream=None):
    """theta (descending), V of a symmetric PSD float64 matrix, and the sweep
    count (one-sided block Jacobi)."""
    lib = L.load()
    _need_cuda(M)
    M = M.to(torch.float64).contiguous()
    m = M.shape[0]
    theta = torch.empty(m, dtype=torch.float64, device=M.device)
    V = torch.empty(m, m, dtype=torch.float64, device=M.device)
    nbytes = lib.bk_eigh_psd_workspace(m)
    ws = _ws(nbytes, M.device)
    sw = C.c_int32(0)
    L.check(lib.bk_eigh_psd(_ptr(M), m, m, _ptr(theta), _ptr(V), m, int(max_sweeps),
                            float(tol), C.byref(sw), _ptr(ws), nbytes, _stream(stream)),
            "bk_eigh_psd")
    return theta, V, int(sw.value)
