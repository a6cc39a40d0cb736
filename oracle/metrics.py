"""Error measures of the paper, in float64 (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this.

* Frobenius-norm error, eq. (1):  ||A - Z Z^T A||_F / ||A - A_k||_F, computed
  through the matrix Pythagorean theorem of Section 3.2,
  ||A - Z Z^T A||_F^2 = ||A||_F^2 - ||Z^T A||_F^2.
* Spectral-norm error, eq. (2):   ||A - Z Z^T A||_2 / sigma_{k+1}.
* Per-vector error, eq. (3), reported as in Section 7 (largest deviation over
  the top k, relative to sigma_{k+1}^2):
  max_i |sigma_i^2 - z_i^T A A^T z_i| / sigma_{k+1}^2.
* The raw quantities behind them: ||A||_F^2, the captured energies
  z_i^T A A^T z_i, and the two norms of the residual A - Z Z^T A from their
  definitions (dense, small inputs).
* Largest principal angle between two k-dimensional subspaces.
* Residual norms of Ritz pairs, ||A A^T z_i - sigma_i^2 z_i||: for a unit z_i
  and the symmetric A A^T, some eigenvalue of A A^T lies within that norm of
  sigma_i^2 (Bauer-Fike), the certificate of the Rayleigh-Ritz values of
  Lemma 1.
"""
from __future__ import annotations

import numpy as np

__all__ = ["frobenius_ratio", "spectral_ratio", "per_vector_error",
           "principal_angle", "principal_angle_sin", "frobenius_sq", "captured",
           "residual_norms", "ritz_residuals"]


def _op(A):
    from .bki import LinearOperator
    return A if isinstance(A, LinearOperator) else LinearOperator(A)


def frobenius_sq(A) -> float:
    """||A||_F^2, or ||A - mu 1^T||_F^2 for a centred operator."""
    op = _op(A)
    if hasattr(op.A, "multiply"):
        fro2 = float(op.A.multiply(op.A).sum())
    else:
        fro2 = float(np.sum(np.asarray(op.A, dtype=np.float64) ** 2))
    if op.center:
        # ||A - mu 1^T||_F^2 = ||A||_F^2 - d ||mu||^2
        fro2 -= op.d * float(op.mu @ op.mu)
    return fro2


def captured(A, Z) -> np.ndarray:
    """z_i^T A A^T z_i = ||A^T z_i||^2 for each column of Z."""
    W = _op(A).tmul(np.asarray(Z, dtype=np.float64))
    return np.sum(W ** 2, axis=0)


def ritz_residuals(A, Z, sigma) -> np.ndarray:
    """||A A^T z_i - sigma_i^2 z_i||_2 for each column z_i of Z (centring of a
    centred operator included)."""
    op = _op(A)
    Z = np.asarray(Z, dtype=np.float64)
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    R = op.mul(op.tmul(Z)) - Z * s2[None, :]
    return np.sqrt(np.sum(R ** 2, axis=0))


def residual_norms(A, Z) -> tuple[float, float]:
    """(||R||_F, ||R||_2) of R = A - Z Z^T A from the definition; A dense, or
    a (small) operator that is materialised, centring included."""
    op = _op(A)
    D = op.A.toarray() if hasattr(op.A, "toarray") else np.asarray(op.A, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    if op.center:
        D = D - op.mu[:, None]
    Z = np.asarray(Z, dtype=np.float64)
    R = D - Z @ (Z.T @ D)
    return float(np.linalg.norm(R, "fro")), float(np.linalg.norm(R, 2))


def frobenius_ratio(A, Z, sigma_true, k: int) -> float:
    ZtA_sq = float(np.sum(captured(A, Z)))
    fro2 = frobenius_sq(A)
    tail = float(np.sum(np.asarray(sigma_true[k:], dtype=np.float64) ** 2))
    return float(np.sqrt(max(fro2 - ZtA_sq, 0.0) / tail))


def spectral_ratio(A, Z, sigma_true, k: int) -> float:
    """Dense: needs A as an ndarray (small inputs)."""
    A = np.asarray(A, dtype=np.float64)
    R = A - Z @ (Z.T @ A)
    return float(np.linalg.norm(R, 2) / sigma_true[k])


def per_vector_error(A, Z, sigma_true, k: int) -> float:
    cap = captured(A, Z)                 # z_i^T A A^T z_i
    s2 = np.asarray(sigma_true[:k], dtype=np.float64) ** 2
    return float(np.max(np.abs(s2 - cap)) / sigma_true[k] ** 2)


def principal_angle_sin(Z1, Z2) -> float:
    """sin of the largest principal angle between span(Z1) and span(Z2),
    both with orthonormal columns: ||Z2 - Z1 (Z1^T Z2)||_2 (accurate for small
    angles, unlike arccos of the smallest cosine)."""
    Z1 = np.asarray(Z1, dtype=np.float64)
    Z2 = np.asarray(Z2, dtype=np.float64)
    R = Z2 - Z1 @ (Z1.T @ Z2)
    return float(min(np.linalg.norm(R, 2), 1.0))


def principal_angle(Z1, Z2) -> float:
    return float(np.arcsin(principal_angle_sin(Z1, Z2)))
