"""GPU checks of the reverse-mode adjoint (through the C ABI).

* central finite differences of the ORACLE's loss (CPU, float64) against the
  GPU gradient, for L1 = sum of the Ritz values and L2 = ||Z Z^T A||_F^2;
* the closed form of the exact-span case: when the Krylov space holds the
  whole column space, the Ritz values are the singular values and
  d(sum_{i<=k} sigma_i)/dA = U_k V_k^T;
* FP32 against FP64, and the torch.autograd.Function wrapper."""
import numpy as np
import pytest

import workloads
from oracle import bki, philox

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk


def _planted(n, d, seed, spec="inv"):
    sv = workloads.spectrum(spec, min(n, d))
    return workloads.planted_dense(n, d, sv, seed), sv


def _fd(loss, A, E, h):
    return (loss(A + h * E) - loss(A - h * E)) / (2 * h)


def test_sum_of_ritz_values_finite_differences():
    n, d, k, q, seed = 256, 128, 8, 3, 7
    A, _ = _planted(n, d, 11)
    Ag = torch.as_tensor(A).cuda()
    res = bk.svd_dense(Ag, k, q, seed=seed, save_for_backward=True)
    G = bk.svd_dense_backward(Ag, k, q, res, sigma_bar=torch.ones(k, dtype=torch.float64,
                                                                   device="cuda"))
    G = G.cpu().numpy()
    Pi = philox.gaussian(seed, d, k)
    loss = lambda X: float(np.sum(bki.block_krylov(X, Pi, k, q).sigma))  # noqa: E731
    rng = np.random.default_rng(3)
    for _ in range(4):
        E = rng.standard_normal((n, d))
        E /= np.linalg.norm(E)
        fd = _fd(loss, A, E, 1e-5)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


def test_projection_loss_finite_differences():
    # L2 = ||Z Z^T A||_F^2 = ||Z^T A||_F^2 through Z: Z_bar = 2 A A^T Z, plus
    # the explicit dependence on A, 2 Z Z^T A.
    n, d, k, q, seed = 200, 150, 6, 4, 5
    A, _ = _planted(n, d, 12, "inv_sqrt")
    Ag = torch.as_tensor(A).cuda()
    res = bk.svd_dense(Ag, k, q, seed=seed, save_for_backward=True)
    Z = res.Z
    Zbar = 2.0 * (Ag @ (Ag.T @ Z))
    G = bk.svd_dense_backward(Ag, k, q, res, Z_bar=Zbar) + 2.0 * (Z @ (Z.T @ Ag))
    G = G.cpu().numpy()
    Pi = philox.gaussian(seed, d, k)

    def loss(X):
        Zo = bki.block_krylov(X, Pi, k, q).Z
        return float(np.sum((Zo.T @ X) ** 2))
    rng = np.random.default_rng(4)
    for _ in range(3):
        E = rng.standard_normal((n, d))
        E /= np.linalg.norm(E)
        fd = _fd(loss, A, E, 1e-5)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


def test_exact_span_closed_form():
    # m = (q+1) k = d: the Krylov space is the whole column space, sigma_i(Z)
    # are the singular values and the gradient of their sum is U_k V_k^T.
    n, d, k, q = 256, 128, 8, 15
    A, _ = _planted(n, d, 13)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Ag = torch.as_tensor(A).cuda()
    res = bk.svd_dense(Ag, k, q, seed=21, save_for_backward=True)
    assert np.allclose(res.sigma.cpu().numpy(), s[:k], rtol=1e-10)
    G = bk.svd_dense_backward(Ag, k, q, res, sigma_bar=torch.ones(k, dtype=torch.float64,
                                                                   device="cuda")).cpu().numpy()
    want = U[:, :k] @ Vt[:k]
    assert np.linalg.norm(G - want) <= 1e-8 * np.sqrt(k)


def test_f32_matches_f64_and_closed_form():
    n, d, k, q = 2048, 1024, 16, 6
    A, sv = _planted(n, d, 14)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    ones = torch.ones(k, dtype=torch.float64, device="cuda")
    A64 = torch.as_tensor(A).cuda()
    A32 = A64.float()
    r64 = bk.svd_dense(A64, k, q, seed=3, save_for_backward=True)
    g64 = bk.svd_dense_backward(A64, k, q, r64, sigma_bar=ones).cpu().numpy()
    r32 = bk.svd_dense(A32, k, q, seed=3, save_for_backward=True)
    g32 = bk.svd_dense_backward(A32, k, q, r32, sigma_bar=ones).cpu().numpy()
    assert np.linalg.norm(g32 - g64) <= 1e-3 * np.linalg.norm(g64)
    # the Krylov subspace has converged well for this spectrum: close to U_k V_k^T
    err = np.linalg.norm(g64 - U[:, :k] @ Vt[:k]) / np.sqrt(k)
    assert err < 1e-2, err


def test_differentiation_workload_full_size():
    """8192 x 4096 FP32, sigma_i = 1/i, k = 32, q = 10: the gradient of the
    sum of the Ritz values against the planted U_k V_k^T (the gradient of
    the sum of the true top-k singular values); they differ only by the
    Krylov convergence error at q = 10."""
    w = workloads.WORKLOADS["dense4"]
    sv = workloads.spectrum(w.spectrum, min(w.n, w.d))
    A, (U, _, V) = workloads.planted_dense_torch(w.n, w.d, sv, w.seed_matrix,
                                                 return_factors=True)
    res = bk.svd_dense(A, w.k, w.q, seed=w.seed_sketch, save_for_backward=True)
    G = bk.svd_dense_backward(A, w.k, w.q, res,
                              sigma_bar=torch.ones(w.k, dtype=torch.float64, device="cuda"))
    want = (U[:, :w.k] @ V[:, :w.k].T).float()
    err = float(torch.linalg.norm(G - want) / np.sqrt(w.k))
    rel = np.abs(res.sigma.cpu().numpy() - sv[:w.k]) / sv[:w.k]
    print(f"dense4 gradient error ||G - U_k V_k^T||_F / sqrt(k) = {err:.3e}, "
          f"max Ritz rel err vs planted {rel.max():.2e}")
    assert err < 2e-3          # measured 2.8e-4
    assert rel.max() < 1e-6
    assert torch.isfinite(G).all()


def test_autograd_function():
    n, d, k, q = 300, 200, 5, 3
    A, _ = _planted(n, d, 15)
    At = torch.as_tensor(A).cuda().requires_grad_(True)
    Z, sig = bk.BKSVD.apply(At, k, q, 9)
    loss = sig.sum() + (Z.T @ At.detach()).pow(2).sum()
    loss.backward()
    Ag = At.detach()
    res = bk.svd_dense(Ag, k, q, seed=9, save_for_backward=True)
    ref = bk.svd_dense_backward(Ag, k, q, res, Z_bar=2.0 * (Ag @ (Ag.T @ res.Z)),
                                sigma_bar=torch.ones(k, dtype=torch.float64, device="cuda"))
    assert torch.allclose(At.grad, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("loss_kind", ["sum_sigma", "proj"])
def test_recomputed_backward_equals_stored_activation_backward(loss_kind):
    """The library's adjoint recomputes the Krylov blocks from the saved
    orthonormal blocks; reverse accumulation over every stored intermediate
    of Algorithm 2 (oracle/autodiff.py, torch autograd on the CPU) must give
    the same gradient in float64."""
    from oracle.autodiff import block_krylov_autograd
    n, d, k, q, seed = 256, 128, 6, 3, 9
    A, _ = _planted(n, d, 15)
    Ag = torch.as_tensor(A).cuda()
    res = bk.svd_dense(Ag, k, q, seed=seed, save_for_backward=True)
    At = torch.tensor(A, requires_grad=True)
    Zr, sr, _ = block_krylov_autograd(At, torch.tensor(philox.gaussian(seed, d, k)), k, q)
    if loss_kind == "sum_sigma":
        G = bk.svd_dense_backward(Ag, k, q, res, sigma_bar=torch.ones(k, dtype=torch.float64,
                                                                       device="cuda"))
        L = sr.sum()
    else:
        Z = res.Z
        G = bk.svd_dense_backward(Ag, k, q, res, Z_bar=2.0 * (Ag @ (Ag.T @ Z))) \
            + 2.0 * (Z @ (Z.T @ Ag))
        L = ((Zr.T @ At) ** 2).sum()
    (Gr,) = torch.autograd.grad(L, At)
    G, Gr = G.cpu().numpy(), Gr.numpy()
    err = np.abs(G - Gr).max() / np.abs(Gr).max()
    print(f"{loss_kind}: max |G_recompute - G_stored| / max |G| = {err:.2e}")
    assert err <= 1e-10
