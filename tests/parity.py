"""Shared checks of GPU results against the oracle (test helpers)."""
from __future__ import annotations

import numpy as np

from oracle import metrics


def gap_index(theta: np.ndarray, k: int, rel_gap: float = 1e-2) -> int:
    """Largest j <= k with (theta_j - theta_{j+1}) / theta_1 >= rel_gap
    (0 if none): span of the leading j Ritz vectors is well conditioned."""
    best = 0
    for j in range(1, k + 1):
        if j < len(theta) and (theta[j - 1] - theta[j]) / theta[0] >= rel_gap:
            best = j
    return best


def gap_tolerance(theta: np.ndarray, j: int, ritz_rtol: float, floor: float) -> float:
    """Davis-Kahan tolerance on the largest principal angle of the leading
    j-subspace: a Ritz-value tolerance of ritz_rtol admits a perturbation of
    M of ~2 ritz_rtol theta_1, which moves that subspace by at most its size
    over the relative gap (theta_j - theta_{j+1}) / theta_1 (factor 5 of
    slack); never below `floor`."""
    gap = (theta[j - 1] - theta[j]) / theta[0]
    return float(min(np.pi / 2, max(floor, 10.0 * ritz_rtol / gap)))


def angle_bound_at_k(theta: np.ndarray, k: int, ritz_rtol: float, angle_tol: float):
    """Tolerance on the largest principal angle of the whole k-dimensional
    Ritz subspace, or None when theta_k = theta_{k+1} (the subspace is not
    unique).  Davis-Kahan: a perturbation E of M moves span(U_k) by at most
    ||E|| / (theta_k - theta_{k+1}); a Ritz-value tolerance of ritz_rtol
    (relative on sigma) admits ||E|| up to ~2 ritz_rtol theta_1, taken with a
    factor 5 of slack."""
    if len(theta) <= k:
        return angle_tol               # the whole space: no gap to resolve
    gap = (theta[k - 1] - theta[k]) / theta[0]
    if not gap > 0:
        return None
    return float(min(np.pi / 2, max(angle_tol, 10.0 * ritz_rtol / gap)))


def compare(Zg, sg, ref, k: int, ritz_rtol: float, angle_tol: float, rel_gap=1e-2,
            orth_tol=None, angle_k=True):
    """Ritz values elementwise; the largest principal angle on the widest
    gap-separated leading subspace (which must exist) and, whenever theta_k >
    theta_{k+1}, on the whole k-subspace against its Davis-Kahan bound;
    orthonormality of Z."""
    Zg = np.asarray(Zg, dtype=np.float64)
    sg = np.asarray(sg, dtype=np.float64)
    rel = np.abs(sg - ref.sigma) / ref.sigma    # per Ritz value
    assert np.all(rel <= ritz_rtol), (rel.max(), ritz_rtol)
    assert np.all(np.diff(sg) <= 0)
    otol = orth_tol if orth_tol is not None else max(1e3 * ritz_rtol, 1e-12)
    assert np.abs(Zg.T @ Zg - np.eye(k)).max() <= otol
    j = gap_index(ref.theta, k, rel_gap)
    assert j >= 1, "no leading subspace with a relative Ritz gap >= rel_gap"
    ang = metrics.principal_angle(ref.Z[:, :j], Zg[:, :j])
    assert ang <= angle_tol, (j, ang)
    out = {"ritz_rel_max": float(rel.max()), "angle": ang, "j": j}
    if angle_k:
        tol_k = angle_bound_at_k(ref.theta, k, ritz_rtol, angle_tol)
        if tol_k is not None:
            ang_k = metrics.principal_angle(ref.Z, Zg)
            assert ang_k <= tol_k, (k, ang_k, tol_k)
            out.update({"angle_k": ang_k, "angle_k_tol": tol_k})
    return out
