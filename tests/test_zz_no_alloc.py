"""The allocation-free dense solve (bk_svd_dense_noalloc) against the
workspace entry point (bk_svd_dense), both called through the C ABI.

Three calls in a row on one GPU, each smaller than the one before (the
static scratch keeps the previous call's contents), each compared with the
workspace entry point on the same input: the same kernels in the same fixed
reduction order, so Z and the Ritz values must be bit-identical; the Ritz
values also meet the oracle (Algorithm 2 in float64) at the parity bar of
their path."""
import ctypes as C

import numpy as np
import pytest

import workloads
from oracle import bki, philox
from tests.parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk
    from paper_1504_05477_amd import _lib as L

# (n, d, k, q, float64?, spectrum, seed): matrix-core FP32 path, FP64
# vector path, small FP32 vector path
CASES = [
    (4096, 2048, 32, 4, False, "inv", 141),
    (1200, 600, 10, 6, True, "inv_sqrt", 142),
    (600, 300, 8, 4, False, "inv_sqrt", 143),
]


def _opt():
    o = L.Options()
    o.struct_size = C.sizeof(L.Options)
    return o


def _solve(lib, A, k, q, seed, noalloc):
    n, d = A.shape
    code = L.F64 if A.dtype == torch.float64 else L.F32
    Z = torch.full((n, k), float("nan"), dtype=A.dtype, device=A.device)
    s = torch.full((k,), float("nan"), dtype=torch.float64, device=A.device)
    info = L.Info()
    o = _opt()
    stream = int(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        st = lib.bk_svd_dense_noalloc(A.data_ptr(), d, code, None, None, 0, n, d, k, q, seed,
                                      C.byref(o), Z.data_ptr(), k, s.data_ptr(),
                                      C.byref(info), stream)
    else:
        nbytes = lib.bk_svd_dense_workspace(n, d, k, q, code, C.byref(o))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        st = lib.bk_svd_dense(A.data_ptr(), d, code, None, None, 0, n, d, k, q, seed,
                              C.byref(o), Z.data_ptr(), k, s.data_ptr(), C.byref(info),
                              ws.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    assert st == L.OK, (noalloc, st)
    return Z.cpu().numpy(), s.cpu().numpy(), info.q_eff


def test_noalloc_matches_workspace_entry_point():
    lib = L.load()
    limit = 64 << 20
    for n, d, k, q, f64, spec, seed in CASES:
        print(f"noalloc case n={n} d={d} k={k} q={q} f64={f64}", flush=True)
        code = L.F64 if f64 else L.F32
        assert 0 < lib.bk_svd_dense_workspace(n, d, k, q, code, C.byref(_opt())) <= limit
        A64 = workloads.planted_dense(n, d, workloads.spectrum(spec, min(n, d)), seed)
        A = torch.as_tensor(A64).cuda()
        if not f64:
            A = A.float()
        Zn, sn, qn = _solve(lib, A, k, q, seed + 100, True)
        Zw, sw, qw = _solve(lib, A, k, q, seed + 100, False)
        assert qn == qw == q
        assert np.array_equal(sn, sw)
        assert np.array_equal(Zn, Zw)
        # and both meet the oracle on the same matrix and sketch
        Pi = philox.gaussian(seed + 100, d, k)
        Ah = A64 if f64 else A.double().cpu().numpy()
        if not f64:
            Pi = Pi.astype(np.float32).astype(np.float64)
        ref = bki.block_krylov(Ah, Pi, k, q, tau=1e-11 if f64 else 1e-5)
        compare(Zn, sn, ref, k, 1e-10 if f64 else 1e-5, 1e-8 if f64 else 1e-4)
