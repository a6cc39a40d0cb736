"""Algorithm 2 (route A) written with differentiable PyTorch CPU operations in
float64, for reference gradients of losses of its outputs.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` may
import it.  It shares no code with the GPU library.

The steps are those of ``bki.block_krylov`` (Section 2.1, Algorithm 2):
B_0 = A Pi, Q_0 = QR(B_0); for i = 1..q, B_i = A (A^T Q_{i-1}), projected
twice against the earlier blocks, Q_i = QR(B_i); then W = A^T Q, M = W^T W
and its top-k eigenpairs (Lemma 1), Z = Q U_k, sigma = sqrt(theta).  Every
intermediate is kept by autograd (stored activations), so ``torch.autograd``
gives the gradient of a loss of (Z, sigma) with respect to A by plain reverse
accumulation through the QR and symmetric eigen-decomposition rules.  No
breakdown handling: the inputs of the tests have well-conditioned blocks.
"""
from __future__ import annotations

import torch

__all__ = ["block_krylov_autograd"]


def _qr_pos(B: torch.Tensor) -> torch.Tensor:
    """Householder thin QR, columns signed so that diag(R) > 0."""
    Q, R = torch.linalg.qr(B)
    s = torch.sign(torch.diagonal(R))
    s = torch.where(s == 0, torch.ones_like(s), s)
    return Q * s


def block_krylov_autograd(A: torch.Tensor, Pi: torch.Tensor, k: int, q: int):
    """(Z, sigma, theta) of Algorithm 2 for a float64 CPU A (requires_grad as
    the caller wishes) and sketch Pi (d x p, p >= k)."""
    if A.dtype != torch.float64 or A.device.type != "cpu":
        raise ValueError("A must be a float64 CPU tensor")
    Pi = Pi.to(torch.float64)
    blocks = [_qr_pos(A @ Pi)]
    for _ in range(q):
        B = A @ (A.T @ blocks[-1])
        P = torch.cat(blocks, dim=1)
        for _ in range(2):
            B = B - P @ (P.T @ B)
        blocks.append(_qr_pos(B))
    Q = torch.cat(blocks, dim=1)
    W = A.T @ Q
    M = W.T @ W
    M = 0.5 * (M + M.T)
    theta, U = torch.linalg.eigh(M)             # ascending
    theta = torch.flip(theta, [0])
    U = torch.flip(U, [1])
    Z = Q @ U[:, :k]
    sigma = torch.sqrt(torch.clamp(theta[:k], min=0.0))
    return Z, sigma, theta
