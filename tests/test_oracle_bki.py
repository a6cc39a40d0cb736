"""Pins of the oracle's Block Krylov Iteration against what the paper and the
mathematics fix (not against the oracle itself):

* exact special cases that reduce to a dense SVD (numpy.linalg.svd);
* three independently coded span routes (Section 4.2: any orthonormalization
  of K gives the same result in exact arithmetic; Lemma 1 route);
* Ritz-value interlacing (proof of Theorem 10) and nestedness in q;
* Lemma 1's identity and Z^T Z = I;
* the matrix Pythagorean identity of Section 3.2;
* planted spectra with known sigma; breakdown / argument rules."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import workloads
from oracle import bki, metrics, philox


def _rand(n, d, seed):
    return np.random.default_rng(seed).standard_normal((n, d))


def _proj_dist(Z1, Z2):
    return np.linalg.norm(Z1 @ Z1.T - Z2 @ Z2.T, 2)


def test_exact_when_krylov_space_holds_column_space():
    # rank(A) = 12 <= m = (q+1)k: span Q = col(A), so Z = U_k and the Ritz
    # values are the true singular values (brute force: numpy SVD).
    A = workloads.planted_dense(40, 30, np.linspace(3.0, 0.5, 12), seed=1)
    k, q = 3, 3
    res = bki.block_krylov(A, philox.gaussian(11, 30, k), k, q)
    U, s, _ = np.linalg.svd(A)
    assert np.allclose(res.sigma, s[:k], rtol=1e-12, atol=0)
    assert _proj_dist(res.Z, U[:, :k]) < 1e-10


def test_exact_full_rank_square_space():
    # m = (q+1)k = min(n, d) = 30 with a generic full-rank A
    A = _rand(40, 30, 2)
    k, q = 3, 9
    res = bki.block_krylov(A, philox.gaussian(12, 30, k), k, q)
    U, s, _ = np.linalg.svd(A)
    assert res.q_eff == q
    assert np.allclose(res.sigma, s[:k], rtol=1e-10)
    assert _proj_dist(res.Z, U[:, :k]) < 1e-8


def test_rank_k_input_exact_at_q0():
    sig = np.array([5.0, 2.0, 1.0, 0.5])
    A = workloads.planted_dense(50, 35, sig, seed=3)
    res = bki.block_krylov(A, philox.gaussian(13, 35, 4), 4, 0)
    assert np.allclose(res.sigma, sig, rtol=1e-12)
    U, _, _ = np.linalg.svd(A)
    assert _proj_dist(res.Z, U[:, :4]) < 1e-12


def test_routes_agree():
    A = workloads.planted_dense(300, 200, workloads.spectrum("inv_sqrt", 200), seed=4)
    Pi = philox.gaussian(14, 200, 6)
    a = bki.block_krylov(A, Pi, 6, 4)
    b = bki.block_krylov_route_b(A, Pi, 6, 4)
    zc, sc = bki.rayleigh_ritz_svd(A, a.Q, 6)
    assert np.allclose(a.sigma, b.sigma, rtol=1e-10)
    assert np.allclose(a.sigma, sc, rtol=1e-12)
    assert metrics.principal_angle(a.Z, b.Z) < 1e-7
    assert metrics.principal_angle(a.Z, zc) < 1e-10
    # the bases themselves span the same space
    assert np.linalg.norm(a.Q - b.Q @ (b.Q.T @ a.Q), 2) < 1e-8


def test_interlacing_and_ritz_identity():
    A = _rand(120, 90, 5) * np.linspace(2.0, 0.1, 90)
    res = bki.block_krylov(A, philox.gaussian(15, 90, 5), 5, 3)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.all(res.sigma <= s[:5] * (1 + 1e-12))
    # sigma_i = ||A^T z_i|| (z_i^T A A^T z_i = theta_i, proof of Theorem 10)
    assert np.allclose(np.linalg.norm(A.T @ res.Z, axis=0), res.sigma, rtol=1e-12)
    # Z^T Z = I (Lemma 1) and Z^T A A^T Z is diagonal with theta
    assert np.allclose(res.Z.T @ res.Z, np.eye(5), atol=1e-13)
    G = (A.T @ res.Z).T @ (A.T @ res.Z)
    assert np.allclose(G, np.diag(res.sigma ** 2), atol=1e-12 * s[0] ** 2)


def test_lemma1_projection_identity():
    A = _rand(80, 60, 6)
    res = bki.block_krylov(A, philox.gaussian(16, 60, 4), 4, 2)
    Q = res.Q
    Ub, sb, Vb = np.linalg.svd(Q.T @ A, full_matrices=False)
    best = Q @ ((Ub[:, :4] * sb[:4]) @ Vb[:4])          # Q (Q^T A)_k
    assert np.allclose(res.Z @ (res.Z.T @ A), best, atol=1e-12)


def test_nested_in_q():
    A = workloads.planted_dense(200, 150, workloads.spectrum("inv", 150), seed=7)
    Pi = philox.gaussian(17, 150, 5)
    prev = None
    for q in range(0, 6):
        s = bki.block_krylov(A, Pi, 5, q).sigma
        if prev is not None:
            assert np.all(s >= prev * (1 - 1e-13))
        prev = s


def test_block_krylov_dominates_simultaneous_iteration():
    # span (A A^T)^q A Pi  is inside the Krylov space of the same Pi, so by
    # Courant-Fischer BKI's Ritz values are >= SI's at equal q (Section 2).
    A = workloads.planted_dense(300, 200, workloads.spectrum("inv_sqrt", 200), seed=8)
    Pi = philox.gaussian(18, 200, 8)
    for q in (0, 2, 4):
        b = bki.block_krylov(A, Pi, 8, q)
        s = bki.simultaneous_iteration(A, Pi, 8, q)
        assert np.all(b.sigma >= s.sigma * (1 - 1e-12))
        if q == 0:
            assert np.allclose(b.sigma, s.sigma, rtol=1e-12)
    sv = workloads.spectrum("inv_sqrt", 200)
    pv_b = metrics.per_vector_error(A, bki.block_krylov(A, Pi, 8, 4).Z, sv, 8)
    pv_s = metrics.per_vector_error(A, bki.simultaneous_iteration(A, Pi, 8, 4).Z, sv, 8)
    assert pv_b < pv_s


def test_oversampled_sketch_dominates_its_leading_columns():
    # Oversampling (Section 6): with Pi_k the first k columns of Pi_p, every
    # Krylov block of Pi_p contains the matching block of Pi_k, so the
    # space is nested and by Courant-Fischer the top-k Ritz values cannot
    # decrease; the oversampled per-vector error is no worse here.
    sv = workloads.spectrum("inv_sqrt", 200)
    A = workloads.planted_dense(300, 200, sv, seed=31)
    k, q = 6, 3
    Pp = philox.gaussian(41, 200, 10)
    rk = bki.block_krylov(A, Pp[:, :k], k, q)
    rp = bki.block_krylov(A, Pp, k, q)
    assert rp.Q.shape[1] == (q + 1) * 10 and rp.Z.shape[1] == k
    assert np.all(rp.sigma >= rk.sigma * (1 - 1e-13))
    assert np.all(rp.sigma <= sv[:k] * (1 + 1e-12))   # interlacing still holds
    assert (metrics.per_vector_error(A, rp.Z, sv, k)
            <= metrics.per_vector_error(A, rk.Z, sv, k) * (1 + 1e-9))
    # the same for Simultaneous Iteration
    sk = bki.simultaneous_iteration(A, Pp[:, :k], k, q)
    sp_ = bki.simultaneous_iteration(A, Pp, k, q)
    assert np.all(sp_.sigma >= sk.sigma * (1 - 1e-12))
    # BKI on the wider sketch still dominates SI on it
    assert np.all(rp.sigma >= sp_.sigma * (1 - 1e-12))


def test_oversampled_exact_span():
    # (q+1) p >= rank(A): the Krylov space holds the column space (exact)
    A = workloads.planted_dense(60, 40, np.linspace(4.0, 1.0, 15), seed=32)
    U, s, _ = np.linalg.svd(A)
    res = bki.block_krylov(A, philox.gaussian(42, 40, 5), 3, 2)   # k=3, p=5, m=15
    assert np.allclose(res.sigma, s[:3], rtol=1e-12)
    assert _proj_dist(res.Z, U[:, :3]) < 1e-10
    with pytest.raises(ValueError):
        bki.block_krylov(A, philox.gaussian(42, 40, 2), 3, 2)     # p < k
    with pytest.raises(ValueError):
        bki.block_krylov(A, philox.gaussian(42, 40, 14), 3, 2)    # (q+1) p > min(n, d)


def test_metrics_on_exact_singular_vectors():
    sv = workloads.spectrum("inv_sqrt", 60)
    A = workloads.planted_dense(90, 60, sv, seed=9)
    U, s, _ = np.linalg.svd(A)
    Uk = U[:, :6]
    assert np.allclose(s, sv, rtol=1e-12)
    assert metrics.per_vector_error(A, Uk, sv, 6) < 1e-12
    assert abs(metrics.spectral_ratio(A, Uk, sv, 6) - 1.0) < 1e-12
    assert abs(metrics.frobenius_ratio(A, Uk, sv, 6) - 1.0) < 1e-12


def test_residual_norms_and_captured_closed_forms():
    # Eckart-Young (Section 2): with Z the exact top-k left singular vectors
    # the residual is A - A_k, whose norms are sqrt(sum_{i>k} sigma_i^2) and
    # sigma_{k+1}; the captured energies are sigma_i^2; ||A||_F^2 is the sum
    # of all sigma_i^2.
    sv = workloads.spectrum("inv", 40)
    A = workloads.planted_dense(70, 40, sv, seed=16)
    U = np.linalg.svd(A)[0]
    fro, spec = metrics.residual_norms(A, U[:, :5])
    assert abs(fro - np.sqrt(np.sum(sv[5:] ** 2))) < 1e-12 * fro
    assert abs(spec - sv[5]) < 1e-12 * spec
    assert np.allclose(metrics.captured(A, U[:, :5]), sv[:5] ** 2, rtol=1e-12)
    assert abs(metrics.frobenius_sq(A) - np.sum(sv ** 2)) < 1e-12 * np.sum(sv ** 2)
    # a generic orthonormal Z: Pythagoras ties the three together, and the
    # spectral residual is at least sigma_{k+1} (optimality of A_k)
    Z = np.linalg.qr(np.random.default_rng(17).standard_normal((70, 5)))[0]
    fro, spec = metrics.residual_norms(A, Z)
    assert abs(fro ** 2 + np.sum(metrics.captured(A, Z)) - metrics.frobenius_sq(A)) < 1e-12
    assert spec >= sv[5] * (1 - 1e-12)
    # centring: the operator's materialised form is A with each row's mean
    # taken out (the row means computed here independently)
    rp, ci, va = workloads.term_document_csr(120, 500, seed=18, median_len=15)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(120, 500))
    Ac = M.toarray() - M.toarray().mean(axis=1, keepdims=True)
    op = bki.LinearOperator(M, center=True)
    Zc = np.linalg.qr(np.random.default_rng(19).standard_normal((120, 4)))[0]
    assert abs(metrics.frobenius_sq(op) - np.sum(Ac ** 2)) < 1e-10 * np.sum(Ac ** 2)
    Rc = Ac - Zc @ (Zc.T @ Ac)
    fro_c, spec_c = metrics.residual_norms(op, Zc)
    assert abs(fro_c - np.sqrt(np.sum(Rc ** 2))) < 1e-10 * fro_c
    assert abs(spec_c - np.linalg.svd(Rc, compute_uv=False)[0]) < 1e-10 * spec_c
    assert np.allclose(metrics.captured(op, Zc), np.sum((Ac.T @ Zc) ** 2, axis=0),
                       rtol=1e-10)


def test_frobenius_pythagoras_matches_direct():
    sv = workloads.spectrum("inv", 50)
    A = workloads.planted_dense(70, 50, sv, seed=10)
    Z = bki.block_krylov(A, philox.gaussian(20, 50, 4), 4, 1).Z
    direct = np.linalg.norm(A - Z @ (Z.T @ A), "fro") / np.sqrt(np.sum(sv[4:] ** 2))
    assert abs(metrics.frobenius_ratio(A, Z, sv, 4) - direct) < 1e-12


def test_principal_angle_against_scipy():
    rng = np.random.default_rng(11)
    Z1 = np.linalg.qr(rng.standard_normal((50, 5)))[0]
    Z2 = np.linalg.qr(Z1 + 1e-3 * rng.standard_normal((50, 5)))[0]
    want = np.max(scipy.linalg.subspace_angles(Z1, Z2))
    assert abs(metrics.principal_angle(Z1, Z2) - want) < 1e-12


def test_error_measures_shrink_with_q():
    # eq. (1) and eq. (3) errors are non-increasing in q (nested spaces)
    w = workloads.scaled(workloads.WORKLOADS["dense1"], 400, 200, k=10, q=0)
    sv = workloads.spectrum(w.spectrum, 200)
    A = workloads.planted_dense(w.n, w.d, sv, seed=w.seed_matrix)
    Pi = philox.gaussian(w.seed_sketch, w.d, w.k)
    fr, pv = [], []
    for q in range(0, 6):
        Z = bki.block_krylov(A, Pi, w.k, q).Z
        fr.append(metrics.frobenius_ratio(A, Z, sv, w.k))
        pv.append(metrics.per_vector_error(A, Z, sv, w.k))
    assert all(f >= 1 - 1e-12 for f in fr)
    assert all(b <= a * (1 + 1e-9) + 1e-14 for a, b in zip(fr, fr[1:]))
    assert all(b <= a * (1 + 1e-9) + 1e-14 for a, b in zip(pv, pv[1:]))
    assert pv[-1] < 0.1 * pv[0]


def test_breakdown_stops_at_invariant_space():
    # rank(A) = 2k exactly: block 1 completes the column space, block 2's
    # projected residual is rounding noise -> q_eff = 1, result exact.
    k = 4
    sig = np.linspace(4.0, 1.0, 2 * k)
    A = workloads.planted_dense(60, 45, sig, seed=12)
    res = bki.block_krylov(A, philox.gaussian(22, 45, k), k, 4)
    assert res.q_eff == 1
    assert res.Q.shape[1] == 2 * k
    assert np.allclose(res.sigma, sig[:k], rtol=1e-12)


def test_rank_error_and_validation():
    A = workloads.low_rank_dense(30, 20, 2, seed=13)
    with pytest.raises(bki.RankError):
        bki.block_krylov(A, philox.gaussian(1, 20, 3), 3, 0)
    with pytest.raises(bki.RankError):
        bki.block_krylov(np.zeros((30, 20)), philox.gaussian(1, 20, 2), 2, 1)
    B = _rand(30, 20, 14)
    for k, q in [(0, 1), (21, 0), (5, -1), (5, 4)]:
        with pytest.raises(ValueError):
            bki.block_krylov(B, philox.gaussian(1, 20, max(k, 1)), k, q)
    with pytest.raises(ValueError):
        bki.block_krylov(B, philox.gaussian(1, 19, 2), 2, 1)


def test_centered_operator_matches_explicit_centering():
    rp, ci, va = workloads.term_document_csr(300, 2000, seed=15, median_len=20)
    A = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(300, 2000))
    dense = A.toarray()
    Ac = dense - dense.mean(axis=1, keepdims=True)
    Pi = philox.gaussian(23, 2000, 5)
    r1 = bki.block_krylov(A, Pi, 5, 3, center=True)
    r2 = bki.block_krylov(Ac, Pi, 5, 3)
    assert np.allclose(r1.sigma, r2.sigma, rtol=1e-11)
    assert metrics.principal_angle(r1.Z, r2.Z) < 1e-8
    # the centred rows sum to zero, so 1 is orthogonal to every A_c^T direction
    assert abs(np.sum(Ac @ np.ones(2000))) < 1e-8
    sv = np.linalg.svd(Ac, compute_uv=False)
    assert np.all(r1.sigma <= sv[:5] * (1 + 1e-12))
    fr_direct = np.linalg.norm(Ac - r1.Z @ (r1.Z.T @ Ac)) / np.sqrt(np.sum(sv[5:] ** 2))
    op = bki.LinearOperator(A, center=True)
    assert abs(metrics.frobenius_ratio(op, r1.Z, sv, 5) - fr_direct) < 1e-10


def test_block_lanczos_tridiagonal_and_exact():
    # the recurrence's T is Q^T A A^T Q itself (block tridiagonal: the
    # entries outside the band vanish), and Q is orthonormal
    sv = workloads.spectrum("inv", 60)
    A = workloads.planted_dense(90, 60, sv, seed=24)
    Pi = philox.gaussian(25, 60, 4)
    r, T = bki.block_lanczos(A, Pi, 4, 5)
    M = r.Q.T @ (A @ (A.T @ r.Q))
    assert np.max(np.abs(M - T)) < 1e-13
    assert np.max(np.abs(r.Q.T @ r.Q - np.eye(24))) < 1e-13
    band = np.abs(np.subtract.outer(np.arange(24) // 4, np.arange(24) // 4)) > 1
    assert np.all(T[band] == 0.0) and np.max(np.abs(M[band])) < 1e-13
    # its span is the literal Krylov space of Algorithm 2 (route B's K)
    Kq = bki.block_krylov_route_b(A, Pi, 4, 2).Q
    r2, _ = bki.block_lanczos(A, Pi, 4, 2)
    assert metrics.principal_angle(Kq, r2.Q) < 1e-9
    # brute force: a rank-12 A with (q+1) k = 12 recovers the exact top k
    sig = np.linspace(3.0, 1.0, 12)
    B = workloads.planted_dense(50, 40, sig, seed=26)
    rb, _ = bki.block_lanczos(B, philox.gaussian(27, 40, 4), 4, 2)
    assert np.allclose(rb.sigma, sig[:4], rtol=1e-12)
    U = np.linalg.svd(B)[0][:, :4]
    assert metrics.principal_angle(rb.Z, U) < 1e-10


def test_block_lanczos_breakdown_and_centring():
    k = 4
    sig = np.linspace(4.0, 1.0, 2 * k)
    A = workloads.planted_dense(60, 45, sig, seed=28)
    r, T = bki.block_lanczos(A, philox.gaussian(29, 45, k), k, 4)
    assert r.q_eff == 1 and T.shape == (2 * k, 2 * k)
    assert np.allclose(r.sigma, sig[:k], rtol=1e-12)
    rp, ci, va = workloads.term_document_csr(200, 900, seed=30, median_len=15)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(200, 900))
    Ac = M.toarray() - M.toarray().mean(axis=1, keepdims=True)
    Pi = philox.gaussian(31, 900, 5)
    r1, _ = bki.block_lanczos(M, Pi, 5, 3, center=True)
    r2, _ = bki.block_lanczos(Ac, Pi, 5, 3)
    assert np.allclose(r1.sigma, r2.sigma, rtol=1e-11)
    assert metrics.principal_angle(r1.Z, r2.Z) < 1e-8


def test_sign_normalization():
    Z = np.array([[0.6, -0.8], [-0.8, 0.6]])
    out = bki.sign_normalize(Z)
    assert np.allclose(out, [[-0.6, 0.8], [0.8, -0.6]])
    tie = bki.sign_normalize(np.array([[-0.5], [0.5]]))
    assert tie[0, 0] > 0                      # tie -> the lower row decides


# ------------------------------------------- Algorithm 1 in closed form --
def _planted_factors(n, d, sig, seed):
    """U (n x r), V (d x r) with orthonormal columns and A = U diag(sig) V^T,
    built here (not by the oracle) from Householder QR of Gaussians."""
    rng = np.random.default_rng(seed)
    r = len(sig)
    U = np.linalg.qr(rng.standard_normal((n, r)))[0]
    V = np.linalg.qr(rng.standard_normal((d, r)))[0]
    return U, V, (U * sig) @ V.T


def _rr_closed_form(A, B):
    """Rayleigh-Ritz on span(B) by Lemma 1's route: Q from the SVD of B,
    then the singular values and left vectors of Q^T A (no eigen-solve)."""
    Q = np.linalg.svd(B, full_matrices=False)[0]
    Ub, s, _ = np.linalg.svd(Q.T @ A, full_matrices=False)
    return s, Q @ Ub


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_simultaneous_iteration_closed_form(q):
    # A = U S V^T:  (A A^T)^q A Pi = U S^(2q+1) (V^T Pi), so after q steps
    # Algorithm 1's block spans U diag(sigma^(2q+1)) V^T Pi exactly; the
    # Rayleigh-Ritz pairs of that span are fixed without iterating.
    sig = np.linspace(1.0, 0.3, 80)
    U, V, A = _planted_factors(120, 80, sig, 51)
    k = 4
    Pi = philox.gaussian(52, 80, 6)                    # p = 6 >= k
    res = bki.simultaneous_iteration(A, Pi, k, q)
    Vp = V.T @ Pi
    want_s, want_Z = _rr_closed_form(A, U @ (sig[:, None] ** (2 * q + 1) * Vp))
    assert np.allclose(res.sigma, want_s[:k], rtol=1e-10, atol=0)
    assert metrics.principal_angle(res.Z, want_Z[:, :k]) < 1e-8
    # the test tells q from q - 1 and q + 1: an off-by-one in the iteration
    # count moves the Ritz values far beyond the tolerance above
    for qq in (q - 1, q + 1):
        s_other = _rr_closed_form(A, U @ (sig[:, None] ** (2 * qq + 1) * Vp))[0][:k]
        assert np.max(np.abs(s_other - res.sigma) / res.sigma) > 1e-6


def test_simultaneous_iteration_exact_when_sketch_spans_column_space():
    # rank(A) = p: span(A Pi) = col(A) already, so every q returns the exact
    # top k (brute force: numpy SVD)
    sig = np.array([3.0, 2.5, 2.0, 1.2, 0.7, 0.4])
    U, V, A = _planted_factors(70, 50, sig, 53)
    for q in (0, 1, 3):
        res = bki.simultaneous_iteration(A, philox.gaussian(54, 50, 6), 3, q)
        assert np.allclose(res.sigma, sig[:3], rtol=1e-12)
        assert _proj_dist(res.Z, U[:, :3]) < 1e-10


def test_block_krylov_closed_form_span():
    # Algorithm 2's space is span{U S^(2i+1) V^T Pi, i = 0..q}; its
    # Rayleigh-Ritz pairs from the closed form, at q = 1..3
    sig = np.linspace(1.0, 0.3, 80)
    U, V, A = _planted_factors(120, 80, sig, 55)
    Pi = philox.gaussian(56, 80, 4)
    Vp = V.T @ Pi
    for q in (1, 2, 3):
        res = bki.block_krylov(A, Pi, 4, q)
        K = np.hstack([U @ (sig[:, None] ** (2 * i + 1) * Vp) for i in range(q + 1)])
        want_s, want_Z = _rr_closed_form(A, K)
        assert np.allclose(res.sigma, want_s[:4], rtol=1e-9)
        assert metrics.principal_angle(res.Z, want_Z[:, :4]) < 1e-7


# ------------------------------------- streamed FP32 operator, factor route --
def test_streamed_dense_matches_dense_operator():
    rng = np.random.default_rng(57)
    A32 = rng.standard_normal((1000, 300)).astype(np.float32)
    A64 = A32.astype(np.float64)
    op = bki.StreamedDense(A32, rows=128)             # 7 full blocks + a ragged one
    X = rng.standard_normal((300, 7))
    Y = rng.standard_normal((1000, 7))
    assert np.allclose(op.mul(X), A64 @ X, rtol=0, atol=1e-12)
    assert np.allclose(op.tmul(Y), A64.T @ Y, rtol=0, atol=1e-11)
    sv = workloads.spectrum("inv", 300)
    B32 = workloads.planted_dense(1000, 300, sv, 58).astype(np.float32)
    Pi = philox.gaussian(59, 300, 5)
    r1 = bki.block_krylov(bki.StreamedDense(B32, rows=100), Pi, 5, 4, tau=1e-5)
    r2 = bki.block_krylov(B32.astype(np.float64), Pi, 5, 4, tau=1e-5)
    assert np.allclose(r1.sigma, r2.sigma, rtol=1e-12)
    assert metrics.principal_angle(r1.Z, r2.Z) < 1e-9
    assert r1.q_eff == r2.q_eff


@pytest.mark.parametrize("n,d,r,q", [(150, 100, 100, 3), (90, 140, 90, 2), (200, 120, 40, 4)])
def test_planted_factor_route_matches_route_a(n, d, r, q):
    # Algorithm 2 is equivariant under A -> U A V^T with orthonormal factors:
    # the route that runs it on diag(sigma) with sketch V^T Pi and maps Z
    # back by U must equal route A on the assembled matrix
    sig = workloads.spectrum("pow08", r)
    U, V, A = _planted_factors(n, d, sig, 60 + n)
    k = 5
    Pi = philox.gaussian(61, d, k)
    a = bki.block_krylov(A, Pi, k, q)
    b = bki.block_krylov_planted(U, sig, V, Pi, k, q)
    assert a.q_eff == b.q_eff
    assert np.allclose(a.sigma, b.sigma, rtol=1e-11)
    assert metrics.principal_angle(a.Z, b.Z) < 1e-9
    assert np.allclose(b.Z.T @ b.Z, np.eye(k), atol=1e-13)
    # the columns agree one by one (sign rule applied after mapping back)
    assert np.max(np.abs(a.Z - b.Z)) < 1e-8


def test_planted_factor_route_exact_top_k():
    # (q+1) k >= rank: exact singular values and vectors, as route A
    sig = np.linspace(2.0, 0.5, 12)
    U, V, A = _planted_factors(60, 45, sig, 62)
    res = bki.block_krylov_planted(U, sig, V, philox.gaussian(63, 45, 3), 3, 3)
    assert np.allclose(res.sigma, sig[:3], rtol=1e-12)
    assert _proj_dist(res.Z, U[:, :3]) < 1e-10


class _RowBlocks:
    """An n x r factor read in row blocks through ``@`` (as a caller holding
    a factor too large to copy at once would supply it)."""

    def __init__(self, U, rows):
        self.U, self.rows, self.shape = U, rows, U.shape

    def __matmul__(self, X):
        return np.vstack([self.U[r0:r0 + self.rows] @ X
                          for r0 in range(0, self.shape[0], self.rows)])


def test_planted_factor_route_streamed_factor_without_basis():
    sig = workloads.spectrum("pow08", 100)
    U, V, A = _planted_factors(150, 100, sig, 64)
    Pi = philox.gaussian(65, 100, 5)
    a = bki.block_krylov_planted(U, sig, V, Pi, 5, 3)
    b = bki.block_krylov_planted(_RowBlocks(U, 37), sig, V, Pi, 5, 3, basis=False)
    assert b.Q is None
    assert np.array_equal(a.sigma, b.sigma)
    assert np.max(np.abs(a.Z - b.Z)) < 1e-13


# ------------------------------------------- residual norms of Ritz pairs --
def test_ritz_residuals_closed_forms():
    s = np.array([3.0, 2.0, 1.5, 0.5, 0.25])
    U, V, A = _planted_factors(40, 30, s, 70)
    # exact singular pairs: zero residual
    r0 = metrics.ritz_residuals(A, U[:, :3], s[:3])
    assert np.all(r0 < 1e-13)
    # z = (u1 + u2)/sqrt(2), sigma^2 = (s1^2 + s2^2)/2: A A^T z - sigma^2 z =
    # (s1^2 - s2^2)/2 (u1 - u2)/sqrt(2), of norm |s1^2 - s2^2|/2
    z = (U[:, :1] + U[:, 1:2]) / np.sqrt(2.0)
    sig = np.sqrt((s[0] ** 2 + s[1] ** 2) / 2.0)
    r = metrics.ritz_residuals(A, z, [sig])
    assert r[0] == pytest.approx((s[0] ** 2 - s[1] ** 2) / 2.0, rel=1e-13)
    # a wrong sigma on an exact vector: |s_j^2 - sigma^2|
    r = metrics.ritz_residuals(A, U[:, 2:3], [1.0])
    assert r[0] == pytest.approx(abs(s[2] ** 2 - 1.0), rel=1e-13)


def test_ritz_residuals_bauer_fike_and_centring():
    rng = np.random.default_rng(71)
    A = rng.standard_normal((60, 25))
    lam = np.linalg.eigvalsh(A @ A.T)           # includes the 35 zeros
    Z = np.linalg.qr(rng.standard_normal((60, 6)))[0]
    sig = rng.uniform(0.5, 8.0, 6)
    r = metrics.ritz_residuals(A, Z, sig)
    for i in range(6):
        assert np.min(np.abs(lam - sig[i] ** 2)) <= r[i] * (1 + 1e-12)
    # centred operator = the explicitly centred dense matrix
    Ac = A - A.mean(axis=1, keepdims=True)
    rc = metrics.ritz_residuals(bki.LinearOperator(A, center=True), Z, sig)
    assert np.allclose(rc, metrics.ritz_residuals(Ac, Z, sig), rtol=1e-12)
