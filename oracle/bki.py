"""Plain FP64 CPU oracle of randomized Block Krylov Iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything under
``oracle/``.  It shares no code with the GPU library and imports nothing from
it.

What it computes: the output of Algorithm 2 (Block Krylov Iteration, Section
2.1 of Musco & Musco, "Randomized Block Krylov Methods for Stronger and Faster
Approximate Singular Value Decomposition") for a given A, sketch Pi, rank k and
depth q, in float64 with NumPy/LAPACK:

  K  = [A Pi, (A A^T) A Pi, ..., (A A^T)^q A Pi]          (step 2)
  Q  = an orthonormal basis of span(K), n x (q+1)k         (step 3)
  M  = Q^T A A^T Q                                         (step 4)
  U_k = the top-k eigenvectors of the PSD matrix M         (step 5; SVD = eig)
  Z  = Q U_k,  Ritz values sigma_i = sqrt(theta_i)          (step 6, Lemma 1)

Readings of the paper taken here (each also listed in the design notes):
* q+1 blocks, so m = (q+1)k (step 2 lists q+1 blocks; steps 3-4 print "qk").
* The orthonormalization method is free: only span(K) matters (Section 4.2,
  the explicit-K-then-QR variant, and per-block reorthonormalization "gives an
  equivalent algorithm in exact arithmetic").  Route A orthonormalizes block
  by block (block classical Gram-Schmidt twice + Householder QR); route B forms
  the literally per-block-normalized K and QR's it at once; route C replaces
  the eigen-solve of M by the SVD of Q^T A (Lemma 1).
* Top-k: eigenvalues descending, ties to the lower index; each column of Z is
  signed so that its largest-magnitude entry (lowest row on ties) is positive.
* Ritz values are sigma_i = sqrt(max(theta_i, 0)) (Lemma 1: M = U S^2 U^T).
* Breakdown: block 0 numerically rank deficient (smallest singular value of
  A Pi <= tau ||A Pi||_F) -> RankError.  A later block whose projected
  residual is negligible as a whole (||B_proj||_F <= tau ||B||_F, B before the
  projection) stops the iteration there (q_eff = i - 1); this is exact when
  the Krylov space has become invariant.  A block that is only partly
  deficient is orthonormalized as it stands.
* Centering (footnote on PCA in Section 1): rows mean-centred implicitly,
  A_c = A - mu 1^T with mu the row means, applied as rank-1 corrections.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "RankError", "BKIResult", "LinearOperator", "validate",
    "block_krylov", "block_krylov_route_b", "rayleigh_ritz_svd",
    "rayleigh_ritz", "simultaneous_iteration", "sign_normalize", "block_lanczos",
    "block_tridiagonal", "StreamedDense", "block_krylov_planted",
]


class RankError(ValueError):
    """A Pi is numerically rank deficient (A = 0 or rank(A) < k)."""


@dataclasses.dataclass
class BKIResult:
    Z: np.ndarray          # n x k, orthonormal columns
    sigma: np.ndarray      # k Ritz values, descending
    theta: np.ndarray      # all m' eigenvalues of M, descending
    Q: np.ndarray          # n x m' orthonormal basis of the Krylov space
    Ubar: np.ndarray       # m' x m' eigenvectors of M (columns, descending)
    q_eff: int             # number of (A A^T) applications actually used


class LinearOperator:
    """A (dense ndarray or scipy.sparse matrix), optionally row-centred.

    mul(X)  = A X   - mu (1^T X)
    tmul(Y) = A^T Y - 1 (mu^T Y)      (mu = row means when centred, else 0)."""

    def __init__(self, A, center: bool = False):
        self.A = A
        self.n, self.d = A.shape
        self.center = center
        if center:
            rs = np.asarray(A.sum(axis=1), dtype=np.float64).reshape(-1)
            self.mu = rs / self.d
        else:
            self.mu = None

    def mul(self, X):
        out = np.asarray(self.A @ X, dtype=np.float64)
        if self.center:
            out = out - np.outer(self.mu, X.sum(axis=0))
        return out

    def tmul(self, Y):
        out = np.asarray(self.A.T @ Y, dtype=np.float64)
        if self.center:
            out = out - np.outer(np.ones(self.d), self.mu @ Y)
        return out


class StreamedDense(LinearOperator):
    """A dense FP32 matrix (the stored master copy of A) used in float64
    without an n x d float64 copy: every product upcasts ``rows`` rows at a
    time (exactly: every float32 is a float64) and multiplies them in
    float64; A^T Y adds the row blocks' float64 partial products in order.
    The same products as LinearOperator(A.astype(float64)) up to the order
    of the float64 sums; only the memory use differs.  No centring."""

    def __init__(self, A32, rows: int = 8192):
        A32 = np.asarray(A32)
        if A32.ndim != 2:
            raise ValueError("need a 2-D matrix")
        self.A = A32
        self.n, self.d = A32.shape
        self.center = False
        self.mu = None
        self.rows = int(rows)

    def _blocks(self):
        for r0 in range(0, self.n, self.rows):
            r1 = min(self.n, r0 + self.rows)
            yield r0, r1, np.asarray(self.A[r0:r1], dtype=np.float64)

    def mul(self, X):
        X = np.asarray(X, dtype=np.float64)
        out = np.empty((self.n, X.shape[1]))
        for r0, r1, blk in self._blocks():
            out[r0:r1] = blk @ X
        return out

    def tmul(self, Y):
        Y = np.asarray(Y, dtype=np.float64)
        out = np.zeros((self.d, Y.shape[1]))
        for r0, r1, blk in self._blocks():
            out += blk.T @ Y[r0:r1]
        return out


def validate(n: int, d: int, k: int, q: int, p: int | None = None) -> None:
    """Argument rules shared with the library's boundary (ValueError here).
    p is the block width (the sketch has p >= k columns, Section 6); the
    Krylov space has (q+1) p columns."""
    p = k if p is None else p
    if k < 1 or q < 0:
        raise ValueError("need k >= 1 and q >= 0")
    if p < k:
        raise ValueError("need block width p >= k")
    if k > min(n, d):
        raise ValueError("need k <= min(n, d)")
    if (q + 1) * p > min(n, d):
        raise ValueError("need (q+1) p <= min(n, d); use a dense SVD instead")


def sign_normalize(Z: np.ndarray) -> np.ndarray:
    """Flip each column so its largest-|.| entry (lowest index on ties) is > 0."""
    idx = np.argmax(np.abs(Z), axis=0)          # argmax returns the first maximum
    s = np.sign(Z[idx, np.arange(Z.shape[1])])
    s[s == 0] = 1.0
    return Z * s


def _qr_pos(B: np.ndarray):
    """Householder thin QR with diag(R) >= 0."""
    Qb, Rb = np.linalg.qr(B)
    s = np.sign(np.diag(Rb))
    s[s == 0] = 1.0
    return Qb * s, Rb * s[:, None]


def rayleigh_ritz(op: LinearOperator, Q: np.ndarray, k: int):
    """Steps 4-6 of Algorithm 2 on a given orthonormal basis Q.

    Forms W = A^T Q explicitly, M = W^T W (= Q^T A A^T Q), its eigenpairs in
    descending order, Z = Q U_k and sigma = sqrt(theta_1..k)."""
    W = op.tmul(Q)
    M = W.T @ W
    M = 0.5 * (M + M.T)
    theta, U = np.linalg.eigh(M)                # ascending
    order = np.argsort(-theta, kind="stable")   # descending, ties -> lower index
    theta = theta[order]
    U = U[:, order]
    Z = sign_normalize(Q @ U[:, :k])
    sigma = np.sqrt(np.maximum(theta[:k], 0.0))
    return Z, sigma, theta, U


def block_krylov(A, Pi, k: int, q: int, *, center: bool = False,
                 tau: float = 1e-12) -> BKIResult:
    """Route A: Algorithm 2 with the blocks orthonormalized as they are formed.

    B_0 = A Pi;  Q_0 = QR(B_0).
    For i = 1..q:  B_i = A (A^T Q_{i-1})  -- a vector of span{(A A^T)^i A Pi}
                   plus lower powers, so span{Q_0..Q_i} = span{K_0..K_i};
                   B_i <- (I - Q_<i Q_<i^T) B_i, done twice;
                   Q_i = QR(B_i).
    Then Rayleigh-Ritz on Q = [Q_0 .. Q_q].  A sketch of p > k columns
    (oversampling, Section 6) makes every block p wide; Rayleigh-Ritz still
    returns the top k."""
    op = A if isinstance(A, LinearOperator) else LinearOperator(A, center)
    n, d = op.n, op.d
    Pi = np.asarray(Pi, dtype=np.float64)
    if Pi.ndim != 2 or Pi.shape[0] != d:
        raise ValueError(f"Pi must be {d} x p")
    validate(n, d, k, q, Pi.shape[1])
    B = op.mul(Pi)
    sv = np.linalg.svd(B, compute_uv=False)
    if not np.all(np.isfinite(B)):
        raise ValueError("non-finite entries")
    if sv[-1] <= tau * max(np.linalg.norm(B), np.finfo(float).tiny):
        raise RankError("A Pi is numerically rank deficient")
    blocks = [_qr_pos(B)[0]]
    q_eff = q
    for i in range(1, q + 1):
        B = op.mul(op.tmul(blocks[-1]))
        before = np.linalg.norm(B)
        P = np.hstack(blocks)
        for _ in range(2):
            B = B - P @ (P.T @ B)
        if np.linalg.norm(B) <= tau * before:
            q_eff = i - 1
            break
        blocks.append(_qr_pos(B)[0])
    Q = np.hstack(blocks)
    Z, sigma, theta, U = rayleigh_ritz(op, Q, k)
    return BKIResult(Z, sigma, theta, Q, U, q_eff)


def block_krylov_route_b(A, Pi, k: int, q: int, *, center: bool = False) -> BKIResult:
    """Route B: the literal K = [K_0 .. K_q] with K_0 = orth(A Pi) and
    K_i = orth(A A^T K_{i-1}) (within-block normalization only, which keeps
    span K_i = span (A A^T)^i A Pi), then one Householder QR of all of K and
    the same Rayleigh-Ritz step.  For small q and well-conditioned inputs."""
    op = A if isinstance(A, LinearOperator) else LinearOperator(A, center)
    Pi = np.asarray(Pi, dtype=np.float64)
    validate(op.n, op.d, k, q, Pi.shape[1])
    Kb = [_qr_pos(op.mul(Pi))[0]]
    for _ in range(q):
        Kb.append(_qr_pos(op.mul(op.tmul(Kb[-1])))[0])
    Q = _qr_pos(np.hstack(Kb))[0]
    Z, sigma, theta, U = rayleigh_ritz(op, Q, k)
    return BKIResult(Z, sigma, theta, Q, U, q)


def rayleigh_ritz_svd(A, Q: np.ndarray, k: int, *, center: bool = False):
    """Route C (Lemma 1): Z = Q * (top-k left singular vectors of Q^T A),
    sigma = the top-k singular values of Q^T A.  No eigen-solve of M."""
    op = A if isinstance(A, LinearOperator) else LinearOperator(A, center)
    QtA = op.tmul(Q).T                       # (A^T Q)^T = Q^T A, m x d
    Ub, s, _ = np.linalg.svd(QtA, full_matrices=False)
    Z = sign_normalize(Q @ Ub[:, :k])
    return Z, s[:k]


def simultaneous_iteration(A, Pi, k: int, q: int, *, center: bool = False) -> BKIResult:
    """Algorithm 1: K = (A A^T)^q A Pi, re-orthonormalized after every
    application of A A^T (Section 4.1), then the same Rayleigh-Ritz on the
    p-dimensional span (p = columns of Pi >= k), top k returned."""
    op = A if isinstance(A, LinearOperator) else LinearOperator(A, center)
    Pi = np.asarray(Pi, dtype=np.float64)
    validate(op.n, op.d, k, 0, Pi.shape[1])
    X = _qr_pos(op.mul(Pi))[0]
    for _ in range(q):
        X = _qr_pos(op.mul(op.tmul(X)))[0]
    Z, sigma, theta, U = rayleigh_ritz(op, X, k)
    return BKIResult(Z, sigma, theta, X, U, q)


def block_tridiagonal(diag, sub) -> np.ndarray:
    """The symmetric block-tridiagonal matrix with diagonal blocks diag[i]
    and blocks sub[i] = T_{i+1,i} below the diagonal (sub[i]^T above)."""
    p = diag[0].shape[0]
    m = p * len(diag)
    T = np.zeros((m, m))
    for i, D in enumerate(diag):
        T[i * p:(i + 1) * p, i * p:(i + 1) * p] = 0.5 * (D + D.T)
    for i, B in enumerate(sub):
        T[(i + 1) * p:(i + 2) * p, i * p:(i + 1) * p] = B
        T[i * p:(i + 1) * p, (i + 1) * p:(i + 2) * p] = B.T
    return T


def block_lanczos(A, Pi, k: int, q: int, *, center: bool = False,
                  tau: float = 1e-12):
    """Route D (Section 4.2, the block Lanczos alternative): the same Krylov
    space built by the three-term recurrence of block Lanczos on A A^T,

        Q_0 B_0 = A Pi,
        Q_i B_i = A A^T Q_{i-1} - Q_{i-1} D_{i-1} - Q_{i-2} B_{i-1}^T,
        D_i = Q_i^T A A^T Q_i,

    so that T = Q^T A A^T Q is block tridiagonal (diagonal blocks D_i, B_i
    below the diagonal).  The recurrence alone loses orthogonality (the
    instability Section 4.2 warns of), so each new block is also projected
    against all earlier ones, twice, before its QR.  Rayleigh-Ritz then takes
    the eigenpairs of T instead of forming W^T W.  Breakdown and ordering
    rules as route A.  Returns (BKIResult, T)."""
    op = A if isinstance(A, LinearOperator) else LinearOperator(A, center)
    n, d = op.n, op.d
    Pi = np.asarray(Pi, dtype=np.float64)
    if Pi.ndim != 2 or Pi.shape[0] != d:
        raise ValueError(f"Pi must be {d} x p")
    validate(n, d, k, q, Pi.shape[1])
    B = op.mul(Pi)
    if not np.all(np.isfinite(B)):
        raise ValueError("non-finite entries")
    sv = np.linalg.svd(B, compute_uv=False)
    if sv[-1] <= tau * max(np.linalg.norm(B), np.finfo(float).tiny):
        raise RankError("A Pi is numerically rank deficient")
    blocks = [_qr_pos(B)[0]]
    diag, sub = [], []
    q_eff = q
    for i in range(1, q + 1):
        X = op.mul(op.tmul(blocks[-1]))          # A A^T Q_{i-1}
        before = np.linalg.norm(X)
        D = blocks[-1].T @ X
        diag.append(D)
        X = X - blocks[-1] @ D
        if len(sub):
            X = X - blocks[-2] @ sub[-1].T
        P = np.hstack(blocks)
        for _ in range(2):
            X = X - P @ (P.T @ X)
        if np.linalg.norm(X) <= tau * before:
            q_eff = i - 1
            break
        Qi, Bi = _qr_pos(X)
        blocks.append(Qi)
        sub.append(Bi)
    if len(diag) < len(blocks):               # the last block's D_q
        W = op.tmul(blocks[-1])
        diag.append(W.T @ W)
    T = block_tridiagonal(diag, sub)
    Q = np.hstack(blocks)
    theta, U = np.linalg.eigh(T)
    order = np.argsort(-theta, kind="stable")
    theta = theta[order]
    U = U[:, order]
    Z = sign_normalize(Q @ U[:, :k])
    sigma = np.sqrt(np.maximum(theta[:k], 0.0))
    return BKIResult(Z, sigma, theta, Q, U, q_eff), T


def block_krylov_planted(U, sigma, V, Pi, k: int, q: int, *,
                         tau: float = 1e-12, basis: bool = True) -> BKIResult:
    """Algorithm 2 on A = U diag(sigma) V^T (U n x r, V d x r, orthonormal
    columns), worked in the coordinates of the factors.

    A Pi = U (S V^T Pi) and A A^T = U S^2 U^T, so every Krylov block of A
    with sketch Pi is U times the matching block of the r x r diagonal
    matrix S = diag(sigma) with sketch V^T Pi.  Q = U Q_S is then an
    orthonormal basis of span(K), Q^T A A^T Q = Q_S^T S^2 Q_S, and
    Rayleigh-Ritz gives the same theta, Z = U Z_S (Lemma 1).  The breakdown
    tests see the same norms and singular values (U has orthonormal
    columns), so q_eff agrees as well.  route A (block_krylov) runs on S as
    it stands; only the n x r and d x r factor products are outside it.

    U may be any n x r object with ``shape`` and ``@`` (e.g. one that reads
    a large factor in row blocks).  basis=False leaves Q as None (mapping
    the n x m basis back costs an n x r x m product; Z needs n x r x k)."""
    import scipy.sparse as sp

    if isinstance(U, np.ndarray) or not hasattr(U, "__matmul__"):
        U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    if U.shape[1] != r or V.shape[1] != r:
        raise ValueError("U and V need one column per singular value")
    S = sp.diags(sigma, format="csr")
    Ps = V.T @ np.asarray(Pi, dtype=np.float64)
    validate(U.shape[0], V.shape[0], k, q, Ps.shape[1])
    res = block_krylov(S, Ps, k, q, tau=tau)
    Z = sign_normalize(np.asarray(U @ res.Z, dtype=np.float64))
    Q = np.asarray(U @ res.Q, dtype=np.float64) if basis else None
    return BKIResult(Z, res.sigma, res.theta, Q, res.Ubar, res.q_eff)
