"""GPU parity of the block Lanczos Rayleigh-Ritz variant (Section 4.2):
the Krylov basis of Algorithm 2 with Q^T A A^T Q taken as the
block-tridiagonal matrix of the recurrence, against the oracle's block
Lanczos route (same sketch, same seed).  Bars as the plain solve: Ritz values
1e-10 (FP64) / 1e-5 (FP32) relative, leading-subspace angles 1e-8 / 1e-4."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import bki, philox
from tests.parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk


def _cuda(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _pi32(seed, d, k):
    return philox.gaussian(seed, d, k).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,d,k,q,spec", [
    (2000, 1000, 10, 8, "inv_sqrt"),   # the dense FP64 workload
    (600, 400, 8, 4, "inv"),
    (333, 257, 5, 3, "inv_sqrt"),      # ragged
    (500, 260, 1, 6, "inv"),           # k = 1: scalar Lanczos
    (129, 333, 5, 0, "inv"),           # q = 0: T is W_0^T W_0 alone
    (2000, 1000, 40, 3, "inv_sqrt"),   # k > 32: separate Cholesky launches
])
def test_lanczos_dense_f64(n, d, k, q, spec):
    sv = workloads.spectrum(spec, min(n, d))
    A = workloads.planted_dense(n, d, sv, 50 + n)
    ref, _ = bki.block_lanczos(A, philox.gaussian(60 + n, d, k), k, q)
    res = bk.svd_dense(_cuda(A), k, q, seed=60 + n, method="lanczos")
    assert res.info["q_eff"] == ref.q_eff
    compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, k, 1e-10, 1e-8)
    # the same Ritz values as the dense W^T W route, to rounding
    plain = bk.svd_dense(_cuda(A), k, q, seed=60 + n)
    np.testing.assert_allclose(res.sigma.cpu().numpy(), plain.sigma.cpu().numpy(), rtol=1e-11)


@pytest.mark.parametrize("n,d,k,q", [(1500, 700, 16, 5), (2048, 1024, 32, 10)])
def test_lanczos_dense_f32(n, d, k, q):
    A = workloads.planted_dense(n, d, workloads.spectrum("inv", min(n, d)), 3 + n)
    A = A.astype(np.float32)
    ref, _ = bki.block_lanczos(A.astype(np.float64), _pi32(70 + n, d, k), k, q, tau=1e-5)
    res = bk.svd_dense(_cuda(A), k, q, seed=70 + n, method="lanczos")
    assert res.info["q_eff"] == ref.q_eff
    compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, k, 1e-5, 1e-4)


def test_lanczos_breakdown_and_oversampling_f64():
    k = 4
    sig = np.linspace(4.0, 1.0, 2 * k)
    A = workloads.planted_dense(300, 200, sig, 12)
    res = bk.svd_dense(_cuda(A), k, 5, seed=22, method="lanczos")
    assert res.info["q_eff"] == 1
    assert np.allclose(res.sigma.cpu().numpy(), sig[:k], rtol=1e-12)
    # p = 12 columns per block for k = 8
    n, d, k, q, p = 1500, 800, 8, 4, 12
    B = workloads.planted_dense(n, d, workloads.spectrum("inv_sqrt", d), 61)
    ref, _ = bki.block_lanczos(B, philox.gaussian(91, d, p), k, q)
    r = bk.svd_dense(_cuda(B), k, q, seed=91, block_size=p, method="lanczos")
    compare(r.Z.cpu().numpy(), r.sigma.cpu().numpy(), ref, k, 1e-10, 1e-8)


def _termdoc(n, d, seed, median=30.0):
    rp, ci, va = workloads.term_document_csr(n, d, seed, median_len=median)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(n, d))
    return (rp, ci, va), M


@pytest.mark.parametrize("k,q", [(8, 4), (40, 2)])
def test_lanczos_csr_centred(k, q):
    (rp, ci, va), M = _termdoc(1200, 20000, 5)
    ref, _ = bki.block_lanczos(M, _pi32(77, 20000, k), k, q, center=True, tau=1e-5)
    res = bk.svd_csr(_cuda(rp), _cuda(ci), _cuda(va), 1200, 20000, k, q, seed=77,
                     center=True, method="lanczos")
    compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, k, 1e-5, 1e-4)


def test_lanczos_csr_term_document_full_size():
    """The 11000 x 130000 term-document workload (k = 20, q = 10, centred)."""
    w = workloads.WORKLOADS["csr2"]
    (rp, ci, va), M = _termdoc(w.n, w.d, w.seed_matrix, median=90.0)
    ref, _ = bki.block_lanczos(M, _pi32(w.seed_sketch, w.d, w.k), w.k, w.q, center=True,
                               tau=1e-5)
    res = bk.svd_csr(_cuda(rp), _cuda(ci), _cuda(va), w.n, w.d, w.k, w.q,
                     seed=w.seed_sketch, center=True, method="lanczos")
    assert res.info["q_eff"] == w.q
    compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, w.k, 1e-5, 1e-4)


def test_lanczos_rejects_backward():
    A = _cuda(workloads.planted_dense(200, 100, workloads.spectrum("inv", 100), 3))
    with pytest.raises(ValueError):
        bk.svd_dense(A, 4, 2, method="lanczos", save_for_backward=True)
