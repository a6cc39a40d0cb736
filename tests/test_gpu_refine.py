"""GPU parity of the wide-block FP32 path, the large eigen-solve, the
low-precision subspaces, the residual-norm certificate of the returned Ritz
pairs and the Jacobi convergence failure (through the C ABI)."""
import numpy as np
import pytest

import workloads
from oracle import bki, metrics, philox
from tests.parity import compare, gap_index, gap_tolerance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk
    from paper_1504_05477_amd import _lib as L


def _cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _pi32(seed, d, k):
    return philox.gaussian(seed, d, k).astype(np.float32).astype(np.float64)


# ---------------------------------------------------- wide FP32 blocks --
# The Grams of these blocks run on the FP32 matrix cores (2 n k^2 >= 1e9
# flops) and the Cholesky factors in the blocked one-workgroup kernel.
@pytest.mark.parametrize("n,d,k,q,spec", [(65536, 2048, 100, 2, "exp200"),
                                          (16384, 2048, 256, 2, "pow08"),
                                          (32768, 4096, 256, 3, "pow08")])
def test_svd_dense_f32_wide_blocks(n, d, k, q, spec):
    print(f"wide FP32 n={n} d={d} k={k} q={q} {spec}", flush=True)
    sv = workloads.spectrum(spec, min(n, d))
    A = workloads.planted_dense_torch(n, d, sv, 90 + k, device="cuda")
    Ah = A.cpu().numpy()
    ref = bki.block_krylov(bki.StreamedDense(Ah), _pi32(91 + k, d, k), k, q, tau=1e-5)
    res = bk.svd_dense(A, k, q, seed=91 + k)
    assert res.info["q_eff"] == ref.q_eff
    # exp(-i/200) + 1e-3 has no relative Ritz gap of 1e-2 (consecutive
    # values differ by ~theta_j / 100): the angle is taken on the widest
    # leading subspace with a gap >= 2e-3, to its Davis-Kahan tolerance
    rel_gap = 2e-3 if spec == "exp200" else 1e-2
    j = gap_index(ref.theta, k, rel_gap)
    tol = gap_tolerance(ref.theta, j, 1e-5, 1e-4)
    out = compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, k, 1e-5, tol,
                  rel_gap=rel_gap)
    print(out)


# ----------------------------------------------- eigen-solve at m = 2304 --
def test_tridiagonal_eigensolve_m2304():
    """The Rayleigh-Ritz matrix of the large dense workload's width (m =
    (q+1) k = 2304, the chip-wide Householder reduction) against the oracle
    in float64."""
    m, k = 2304, 256
    q = m // k - 1
    n, d = 3 * m + 17, 2 * m + 5
    A = workloads.planted_dense(n, d, workloads.spectrum("inv_sqrt", min(n, d)), 2304)
    ref = bki.block_krylov(A, philox.gaussian(6, d, k), k, q)
    res = bk.svd_dense(_cuda(A), k, q, seed=6)
    assert res.info["jacobi_sweeps"] == 0           # the tridiagonal path
    compare(res.Z.cpu().numpy(), res.sigma.cpu().numpy(), ref, k, 1e-10, 1e-8)


# ------------------------------------------------- low-precision subspace --
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_subspace_and_residuals(prec):
    """BF16 / FP8 copy plus the FP32 correction pass: Ritz values within
    1e-3 of the oracle's, the gap-separated leading subspace within the
    angle the Ritz error allows, and the residual certificate of every
    returned pair brackets a planted singular value (Bauer-Fike)."""
    n, d, k, q = 8192, 2048, 32, 6
    sv = workloads.spectrum("inv", d)
    A = workloads.planted_dense(n, d, sv, 25).astype(np.float32)
    ref = bki.block_krylov(A.astype(np.float64), _pi32(35, d, k), k, q, tau=1e-5)
    Ag = _cuda(A)
    if prec == "bf16":
        res = bk.svd_dense(bk.quantize(Ag, "bf16"), k, q, seed=35, A_master=Ag,
                           residuals=True)
    else:
        codes, sc = bk.quantize(Ag, "fp8")
        res = bk.svd_dense(codes, k, q, seed=35, a_scales=sc, A_master=Ag, residuals=True)
    Z, s = res.Z.cpu().numpy(), res.sigma.cpu().numpy()
    out = compare(Z, s, ref, k, 1e-3, 1e-2, orth_tol=1e-4)
    print(prec, out)
    r = res.residuals.cpu().numpy()
    # some singular value of the stored FP32 matrix within r_i / sigma_i of
    # sigma_i; the stored matrix's singular values are the planted ones to
    # within ||A32 - A||_2 <= 2^-24 ||A||_F
    # (plus the FP32 rounding floor of the certificate's own products)
    slack = 2.0 ** -24 * np.sqrt(np.sum(sv ** 2))
    for i in range(k):
        assert np.min(np.abs(sv - s[i])) <= (r[i] + 1e-5 * sv[0] ** 2) / s[i] + slack, (i, r[i])
    # and r agrees with the oracle's residuals of its own pairs up to what
    # the pairs differ by (r is 1-Lipschitz in (A A^T - theta I) z)
    ro = metrics.ritz_residuals(A.astype(np.float64), ref.Z, ref.sigma)
    dz = np.linalg.norm(Z - ref.Z, axis=0)
    bound = sv[0] ** 2 * dz + np.abs(s ** 2 - ref.sigma ** 2) + 1e-5 * sv[0] ** 2
    assert np.all(np.abs(r - ro) <= bound)


@pytest.mark.parametrize("f64", [True, False])
def test_residual_certificate_plain(f64):
    n, d, k, q = 3000, 1200, 12, 6
    sv = workloads.spectrum("inv_sqrt", d)
    A = workloads.planted_dense(n, d, sv, 26)
    if not f64:
        A = A.astype(np.float32)
    Pi = philox.gaussian(36, d, k) if f64 else _pi32(36, d, k)
    ref = bki.block_krylov(A.astype(np.float64), Pi, k, q, tau=1e-11 if f64 else 1e-5)
    res = bk.svd_dense(_cuda(A), k, q, seed=36, residuals=True)
    Z, s, r = res.Z.cpu().numpy(), res.sigma.cpu().numpy(), res.residuals.cpu().numpy()
    compare(Z, s, ref, k, 1e-10 if f64 else 1e-5, 1e-8 if f64 else 1e-4)
    ro = metrics.ritz_residuals(A.astype(np.float64), ref.Z, ref.sigma)
    dz = np.linalg.norm(Z - ref.Z, axis=0)
    floor = (1e-13 if f64 else 1e-5) * sv[0] ** 2
    assert np.all(np.abs(r - ro) <= sv[0] ** 2 * dz + np.abs(s ** 2 - ref.sigma ** 2) + floor)
    slack = 0.0 if f64 else 2.0 ** -24 * np.sqrt(np.sum(sv ** 2))
    for i in range(k):
        assert np.min(np.abs(sv - s[i])) <= (r[i] + floor) / s[i] + slack


def test_residual_certificate_csr_centred():
    n, d, k, q = 700, 3000, 6, 3
    rp, ci, va = workloads.term_document_csr(n, d, 27)
    import scipy.sparse as sp
    As = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(n, d))
    op = bki.LinearOperator(As, center=True)
    ref = bki.block_krylov(op, _pi32(37, d, k), k, q, tau=1e-5)
    res = bk.svd_csr(_cuda(rp), _cuda(ci), _cuda(va), n, d, k, q, seed=37, center=True,
                     residuals=True)
    Z, s, r = res.Z.cpu().numpy(), res.sigma.cpu().numpy(), res.residuals.cpu().numpy()
    compare(Z, s, ref, k, 1e-5, 1e-4)
    ro = metrics.ritz_residuals(op, ref.Z, ref.sigma)
    dz = np.linalg.norm(Z - ref.Z, axis=0)
    assert np.all(np.abs(r - ro) <= s[0] ** 2 * dz + np.abs(s ** 2 - ref.sigma ** 2)
                  + 1e-5 * s[0] ** 2)
    # an oversampled block cannot return the certificate (plans are p wide)
    with pytest.raises(ValueError):
        bk.svd_csr(_cuda(rp), _cuda(ci), _cuda(va), n, d, k, q, seed=37, block_size=k + 2,
                   residuals=True)


# ------------------------------------------------ Jacobi non-convergence --
def test_jacobi_sweep_limit_gives_enoconv():
    m, k = 90, 10
    n, d = 300, 200
    A = workloads.planted_dense(n, d, workloads.spectrum("inv_sqrt", d), 28)
    with pytest.raises(L.BKError) as ei:
        bk.svd_dense(_cuda(A), k, m // k - 1, seed=38, jacobi_block=16, max_sweeps=1)
    assert ei.value.status == L.ENOCONV
    # with the default limit the same solve converges
    res = bk.svd_dense(_cuda(A), k, m // k - 1, seed=38, jacobi_block=16)
    assert res.info["jacobi_sweeps"] > 1


# ------------------------------------------- close Ritz values, FP64 --
def test_close_pair_keeps_z_orthonormal():
    """Two singular values 5e-10 apart (relative): the inverse-iteration
    vectors of the pair are not in one cluster of the eigen-solve, and their
    overlap (~ eps ||T|| / gap ~ 4e-7) must be removed before Z = Q U_k.
    (q+1) k = d: the Krylov space is the whole row space, so the Ritz values
    are the singular values."""
    n, d, k, q = 300, 60, 6, 9
    sv = np.linspace(1.0, 0.2, d)
    sv[3] = sv[2] * (1.0 - 5e-10)
    A = workloads.planted_dense(n, d, sv, 29)
    ref = bki.block_krylov(A, philox.gaussian(39, d, k), k, q)
    res = bk.svd_dense(_cuda(A), k, q, seed=39)
    Z, s = res.Z.cpu().numpy(), res.sigma.cpu().numpy()
    assert np.abs(Z.T @ Z - np.eye(k)).max() <= 1e-12
    assert np.allclose(s, sv[:k], rtol=1e-12)
    # the pair's span, and the rest, against the oracle
    assert metrics.principal_angle(ref.Z[:, :2], Z[:, :2]) < 1e-8
    assert metrics.principal_angle(ref.Z[:, :4], Z[:, :4]) < 1e-8
