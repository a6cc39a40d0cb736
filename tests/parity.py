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


def compare(Zg, sg, ref, k: int, ritz_rtol: float, angle_tol: float, rel_gap=1e-2,
            orth_tol=None):
    """Ritz values elementwise; the largest principal angle on the widest
    gap-separated leading subspace; orthonormality of Z."""
    Zg = np.asarray(Zg, dtype=np.float64)
    sg = np.asarray(sg, dtype=np.float64)
    rel = np.abs(sg - ref.sigma) / ref.sigma    # per Ritz value
    assert np.all(rel <= ritz_rtol), (rel.max(), ritz_rtol)
    assert np.all(np.diff(sg) <= 0)
    otol = orth_tol if orth_tol is not None else max(1e3 * ritz_rtol, 1e-12)
    assert np.abs(Zg.T @ Zg - np.eye(k)).max() <= otol
    j = gap_index(ref.theta, k, rel_gap)
    ang = metrics.principal_angle(ref.Z[:, :j], Zg[:, :j]) if j else 0.0
    assert ang <= angle_tol, (j, ang)
    return {"ritz_rel_max": float(rel.max()), "angle": ang, "j": j}
