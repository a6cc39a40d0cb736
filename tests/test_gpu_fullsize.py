"""Full-size parity of the 65536 x 16384 workload (planted sigma_i =
exp(-i/200) + 1e-3 plus 1e-4 Gaussian noise, k = 100, q = 12) in the launch
configuration the benchmark times: the FP32 path and the BF16 copy with the
FP32 correction pass, each against route A of the oracle on the stored FP32
matrix (float64).

Its spectrum has no leading gap of 1e-2 theta_1 (consecutive Ritz values
differ by about theta_j / 100), so the subspace is compared on the widest
leading subspace with a relative gap >= 2e-3, with the tolerance Davis-Kahan
gives for the Ritz-value tolerance over that gap (never below 1e-4 rad)."""
import numpy as np
import pytest

import workloads
from oracle import bki, metrics, philox
from tests.parity import gap_index, gap_tolerance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk


@pytest.fixture(scope="module")
def dense3():
    w = workloads.WORKLOADS["dense3"]
    sv = workloads.spectrum(w.spectrum, min(w.n, w.d))
    print(f"dense3 {w.n} x {w.d}, k={w.k}, q={w.q}", flush=True)
    A = workloads.planted_dense_torch(w.n, w.d, sv, w.seed_matrix, device="cuda",
                                      noise=w.noise, noise_seed=w.seed_noise)
    A64 = A.cpu().numpy().astype(np.float64)
    Pi = philox.gaussian(w.seed_sketch, w.d, w.k).astype(np.float32).astype(np.float64)
    ref = bki.block_krylov(A64, Pi, w.k, w.q, tau=1e-5)
    del A64
    return w, A, ref


def _check(w, res, ref, ritz_rtol):
    k = w.k
    Z = res.Z.cpu().numpy().astype(np.float64)
    s = res.sigma.cpu().numpy()
    rel = np.abs(s - ref.sigma) / ref.sigma
    j = gap_index(ref.theta, k, 2e-3)
    assert j >= 1
    tol = gap_tolerance(ref.theta, j, ritz_rtol, 1e-4)
    ang = metrics.principal_angle(ref.Z[:, :j], Z[:, :j])
    orth = np.abs(Z.T @ Z - np.eye(k)).max()
    print(f"Ritz rel max {rel.max():.2e} median {np.median(rel):.2e}; angle on the leading "
          f"{j} {ang:.2e} (tol {tol:.1e}); |Z^T Z - I| {orth:.1e}; q_eff {res.info['q_eff']}")
    assert res.info["q_eff"] == ref.q_eff
    assert rel.max() <= ritz_rtol, rel.max()
    assert ang <= tol
    assert orth <= 1e-4


def test_dense3_fp32_full_size(dense3):
    w, A, ref = dense3
    res = bk.svd_dense(A, w.k, w.q, seed=w.seed_sketch)
    _check(w, res, ref, 1e-5)


def test_dense3_bf16_refined_full_size(dense3):
    w, A, ref = dense3
    res = bk.svd_dense(bk.quantize(A, "bf16"), w.k, w.q, seed=w.seed_sketch, A_master=A)
    _check(w, res, ref, 1e-3)
