"""Pins of the differentiable route of Algorithm 2 (oracle/autodiff.py), CPU:
its forward equals route A (bki.block_krylov); its gradients equal central
finite differences of route A's outputs; in the exact-span case the gradient
of the sum of the top-k Ritz values is the closed form U_k V_k^T."""
import numpy as np
import pytest

import workloads
from oracle import bki, metrics, philox
from oracle.autodiff import block_krylov_autograd

torch = pytest.importorskip("torch")


def _t(x, grad=False):
    return torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=grad)


def _fd(loss, A, E, h=1e-5):
    return (loss(A + h * E) - loss(A - h * E)) / (2 * h)


def test_forward_equals_route_a():
    A = workloads.planted_dense(120, 80, workloads.spectrum("inv", 80), 41)
    Pi = philox.gaussian(42, 80, 5)
    Z, s, _ = block_krylov_autograd(_t(A), _t(Pi), 5, 3)
    ref = bki.block_krylov(A, Pi, 5, 3)
    assert np.allclose(s.numpy(), ref.sigma, rtol=1e-12)
    assert metrics.principal_angle(Z.numpy(), ref.Z) < 1e-9


@pytest.mark.parametrize("loss_kind", ["sum_sigma", "proj"])
def test_gradient_matches_finite_differences_of_route_a(loss_kind):
    n, d, k, q = 60, 40, 3, 2
    A = workloads.planted_dense(n, d, workloads.spectrum("inv", d), 43)
    Pi = philox.gaussian(44, d, k)
    At = _t(A, grad=True)
    Z, s, _ = block_krylov_autograd(At, _t(Pi), k, q)
    L = s.sum() if loss_kind == "sum_sigma" else ((Z.T @ At) ** 2).sum()
    (G,) = torch.autograd.grad(L, At)
    G = G.numpy()

    def loss(X):
        r = bki.block_krylov(X, Pi, k, q)
        return float(np.sum(r.sigma)) if loss_kind == "sum_sigma" else float(
            np.sum((r.Z.T @ X) ** 2))
    rng = np.random.default_rng(45)
    for _ in range(3):
        E = rng.standard_normal((n, d))
        E /= np.linalg.norm(E)
        fd = _fd(loss, A, E)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


def test_exact_span_closed_form():
    # (q+1) k = d: the Krylov space is the column space of A^T-side, the Ritz
    # values are the singular values and d(sum_{i<=k} sigma_i)/dA = U_k V_k^T
    n, d, k, q = 70, 40, 4, 9
    A = workloads.planted_dense(n, d, workloads.spectrum("inv", d), 46)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    At = _t(A, grad=True)
    _, sig, _ = block_krylov_autograd(At, _t(philox.gaussian(47, d, k)), k, q)
    assert np.allclose(sig.detach().numpy(), s[:k], rtol=1e-12)
    (G,) = torch.autograd.grad(sig.sum(), At)
    assert np.abs(G.numpy() - U[:, :k] @ Vt[:k]).max() < 1e-10
