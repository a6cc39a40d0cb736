"""Host checks of the input generators (no method arithmetic here)."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("rows,cols,rowblk", [(3000, 700, 512), (2048, 1024, 256)])
def test_blocked_cholqr2_generator_matches_householder(rows, cols, rowblk):
    # The large planted factors (>= 2^31 entries) are drawn by row blocks and
    # orthonormalized by CholeskyQR2 instead of one library QR (whose 32-bit
    # indexing does not reach them).  On the CPU, with a small row block so
    # that several blocks and a ragged one are exercised, the result must be
    # the Householder Q of the same Gaussian made unique by diag(R) > 0.
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    x = workloads._gaussian_rows(rows, cols, g, "cpu", rowblk=rowblk)
    q_ref, r_ref = torch.linalg.qr(x)
    s = torch.sign(torch.diagonal(r_ref))
    q_ref = q_ref * s
    q = workloads._cholqr2_rows(x.clone(), rowblk=rowblk)
    assert torch.max(torch.abs(q - q_ref)).item() < 1e-12
    eye = torch.eye(cols, dtype=torch.float64)
    assert torch.max(torch.abs(q.t() @ q - eye)).item() < 1e-13


def test_orth_blocked_is_seed_deterministic():
    g1 = torch.Generator(device="cpu")
    g1.manual_seed(3)
    g2 = torch.Generator(device="cpu")
    g2.manual_seed(3)
    a = workloads._orth_blocked(1000, 200, g1, "cpu")
    b = workloads._orth_blocked(1000, 200, g2, "cpu")
    assert torch.equal(a, b)


def test_planted_dense_torch_cpu_factors():
    # A = U diag(sigma) V^T with the factors returned; the planted singular
    # values are A's (brute force: numpy SVD)
    sv = workloads.spectrum("pow08", 120)
    A, (U, sig, V) = workloads.planted_dense_torch(300, 120, sv, 5, device="cpu",
                                                   out_dtype=torch.float64,
                                                   return_factors=True)
    s = np.linalg.svd(A.numpy(), compute_uv=False)
    assert np.allclose(s, sv, rtol=1e-12)
    assert torch.max(torch.abs((U * sig) @ V.t() - A)).item() < 1e-14


def test_planted_dense_torch_storage_rounding():
    # the reported rounding norm is ||A_FP32 - A_FP64||_F of the same
    # product, and Weyl bounds the singular values of the stored matrix by it
    sv = workloads.spectrum("pow08", 120)
    st = {}
    A32 = workloads.planted_dense_torch(300, 120, sv, 5, device="cpu", stats=st)
    A64 = workloads.planted_dense_torch(300, 120, sv, 5, device="cpu",
                                        out_dtype=torch.float64)
    want = float(torch.linalg.norm(A32.double() - A64))
    assert st["storage_rounding_fro"] == pytest.approx(want, rel=1e-12)
    assert 0 < want < 2 ** -23 * float(torch.linalg.norm(A64))
    s = np.linalg.svd(A32.double().numpy(), compute_uv=False)
    assert np.max(np.abs(s - sv)) <= want
