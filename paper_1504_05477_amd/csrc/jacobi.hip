// Eigen-solve of the Rayleigh-Ritz matrix M = Q^T A A^T Q (Algorithm 2,
// step 5; M is symmetric PSD, so its SVD is its eigen-decomposition, Lemma 1).
//
// Method: one-sided (Hestenes) block Jacobi on the COLUMNS of M.  Plane
// rotations from the right, X <- X J, make the columns of X = M J mutually
// orthogonal; then X^T X = J^T M^2 J is diagonal, so J holds eigenvectors of
// M^2 -- which are those of M, because theta -> theta^2 is one-to-one on
// theta >= 0 -- and x_j = theta_j v_j.  The eigenvalues are the column norms
// and the top eigenvectors are the normalised columns, so no eigenvector
// matrix has to be accumulated (it can be, for callers that need every
// eigenvector).
//
// Columns are grouped in blocks of b; a sweep is a round-robin tournament of
// the nb blocks (nb - 1 rounds), one launch per round, one workgroup per
// block pair.  A workgroup forms the 2b x 2b Gram of its 2b columns,
// diagonalises it with a cyclic two-sided Jacobi in LDS (rotations of
// Golub & Van Loan's symmetric 2 x 2 Schur form), and rotates its columns
// (and those of V) by the result.  A pair whose columns are already
// orthogonal to tol (|x_i^T x_j| <= tol ||x_i|| ||x_j||) is left alone; the
// largest such ratio of the sweep is kept in the status word, and the sweep
// in which every pair passed the test is the last.
#include "kernels.hpp"

namespace bk {
namespace {

__device__ __forceinline__ int tournament(int pos, int round, int players) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (players - 1);
}

__global__ __launch_bounds__(256) void jacobi_init_kernel(
    const double* __restrict__ M, int64_t m, int64_t ldm, double* __restrict__ Xc,
    double* __restrict__ Vc, int64_t ldc, int64_t nbp) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= nbp * m) return;
  const int64_t c = i / m, r = i - c * m;
  Xc[c * ldc + r] = c < m ? 0.5 * (M[r * ldm + c] + M[c * ldm + r]) : 0.0;
  if (Vc) Vc[c * ldc + r] = (r == c) ? 1.0 : 0.0;
}

template <int B2>
__device__ double pair_offdiag(const double (*G)[B2 + 1], double* red) {
  const int t = threadIdx.x;
  double off = 0.0;
  for (int e = t; e < B2 * B2; e += 256) {
    const int gi = e / B2, gj = e % B2;
    if (gi < gj) {
      const double dd = G[gi][gi] * G[gj][gj];
      if (dd > 0.0) off = fmax(off, fabs(G[gi][gj]) / sqrt(dd));
    }
  }
  red[t] = off;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

template <int B2, bool WITHV>
__global__ __launch_bounds__(256) void jacobi_round_kernel(
    int64_t m, int nb, int round, double* __restrict__ Xc,
    double* __restrict__ Vc, int64_t ldc, double tol, int inner_max,
    Ctrl* ctrl) {
  constexpr int b = B2 / 2;
  constexpr int NP = B2 / 2;
  constexpr int CH = 64;
  __shared__ double G[B2][B2 + 1];
  __shared__ double U[B2][B2 + 1];
  __shared__ double P[CH][B2 + 1];
  __shared__ double red[256];
  __shared__ int64_t colidx[B2];
  __shared__ double rc[NP], rs[NP], rt[NP];
  __shared__ int rp[NP], rq[NP];

  const int t = threadIdx.x;
  const int w = blockIdx.x;
  const int I = tournament(w, round, nb);
  const int J = tournament(nb - 1 - w, round, nb);
  if (t < B2) colidx[t] = (t < b) ? static_cast<int64_t>(I) * b + t
                                  : static_cast<int64_t>(J) * b + (t - b);
  __syncthreads();

  // 1. Gram of the 2b columns, rows streamed through LDS in chunks.
  constexpr int EPT = (B2 * B2 + 255) / 256;
  double gacc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) gacc[i] = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += CH) {
    for (int idx = t; idx < CH * B2; idx += 256) {
      const int c = idx / CH, rr = idx % CH;
      P[rr][c] = (r0 + rr < m) ? Xc[colidx[c] * ldc + r0 + rr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = t + 256 * i;
      if (e < B2 * B2) {
        const int gi = e / B2, gj = e % B2;
        double s = 0.0;
        for (int rr = 0; rr < CH; ++rr) s += P[rr][gi] * P[rr][gj];
        gacc[i] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = t + 256 * i;
    if (e < B2 * B2) G[e / B2][e % B2] = gacc[i];
  }
  __syncthreads();

  // 2. Convergence measure of this pair.
  const double off = pair_offdiag<B2>(G, red);
  if (t == 0) atomic_max_nonneg(&ctrl->offmax, off);
  if (!(off > tol)) return;  // already orthogonal (uniform branch)

  // 3. Inner cyclic Jacobi on the 2b x 2b Gram, U accumulates the rotations.
  for (int e = t; e < B2 * B2; e += 256) U[e / B2][e % B2] = (e / B2 == e % B2) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < inner_max; ++sweep) {
    if (sweep > 0 && !(pair_offdiag<B2>(G, red) > tol)) break;
    for (int step = 0; step < B2 - 1; ++step) {
      if (t < NP) {
        const int p = tournament(t, step, B2);
        const int q = tournament(B2 - 1 - t, step, B2);
        const double a = G[p][p], d = G[q][q], bb = G[q][p];
        double c = 1.0, s = 0.0, tt = 0.0;
        // rotate only when the pair is not already orthogonal to tol
        // (relative to the two diagonal entries: keeps relative accuracy)
        if (fabs(bb) > tol * sqrt(fmax(a, 0.0) * fmax(d, 0.0)) && bb != 0.0) {
          const double tau = (d - a) / (2.0 * bb);
          tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        rp[t] = p;
        rq[t] = q;
        rc[t] = c;
        rs[t] = s;
        rt[t] = tt;
      }
      __syncthreads();
      // G <- J^T G J, one 2 x 2 block (pair w1 rows, pair w2 cols) per item.
      // The pair's own diagonal block gets the exact Jacobi update
      // (a - t b, d + t b, 0): recomputing it from products would cancel.
      for (int idx = t; idx < NP * NP; idx += 256) {
        const int w1 = idx / NP, w2 = idx % NP;
        const int p1 = rp[w1], q1 = rq[w1], p2 = rp[w2], q2 = rq[w2];
        if (w1 == w2) {
          const double tt = rt[w1];
          if (tt != 0.0) {
            const double bb = G[q1][p1];
            G[p1][p1] -= tt * bb;
            G[q1][q1] += tt * bb;
            G[p1][q1] = 0.0;
            G[q1][p1] = 0.0;
          }
          continue;
        }
        const double c1 = rc[w1], s1 = rs[w1], c2 = rc[w2], s2 = rs[w2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const double g11 = G[p1][p2], g12 = G[p1][q2], g21 = G[q1][p2], g22 = G[q1][q2];
        const double t11 = c1 * g11 - s1 * g21, t12 = c1 * g12 - s1 * g22;
        const double t21 = s1 * g11 + c1 * g21, t22 = s1 * g12 + c1 * g22;
        G[p1][p2] = t11 * c2 - t12 * s2;
        G[p1][q2] = t11 * s2 + t12 * c2;
        G[q1][p2] = t21 * c2 - t22 * s2;
        G[q1][q2] = t21 * s2 + t22 * c2;
      }
      // U <- U J
      for (int idx = t; idx < B2 * NP; idx += 256) {
        const int r = idx / NP, w2 = idx % NP;
        const int p = rp[w2], q = rq[w2];
        const double c = rc[w2], s = rs[w2];
        const double up = U[r][p], uq = U[r][q];
        U[r][p] = c * up - s * uq;
        U[r][q] = s * up + c * uq;
      }
      __syncthreads();
    }
  }

  // 4. Rotate the columns: X(:, cols) <- X(:, cols) U (and V alike).
  for (int pass = 0; pass < (WITHV ? 2 : 1); ++pass) {
    double* Base = pass == 0 ? Xc : Vc;
    for (int64_t r0 = 0; r0 < m; r0 += CH) {
      for (int idx = t; idx < CH * B2; idx += 256) {
        const int c = idx / CH, rr = idx % CH;
        P[rr][c] = (r0 + rr < m) ? Base[colidx[c] * ldc + r0 + rr] : 0.0;
      }
      __syncthreads();
      for (int idx = t; idx < CH * B2; idx += 256) {
        const int c = idx / CH, rr = idx % CH;
        if (r0 + rr < m) {
          double s = 0.0;
#pragma unroll 8
          for (int l = 0; l < B2; ++l) s += P[rr][l] * U[l][c];
          Base[colidx[c] * ldc + r0 + rr] = s;
        }
      }
      __syncthreads();
    }
  }
}

// norms[j] = ||x_j|| (signed by v_j^T x_j when V is kept), one wave per column.
__global__ __launch_bounds__(256) void col_norm_kernel(const double* __restrict__ Xc,
                                                       const double* __restrict__ Vc,
                                                       int64_t ldc, int64_t m,
                                                       double* __restrict__ norms) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= m) return;
  double ss = 0.0, dv = 0.0;
  for (int64_t r = lane; r < m; r += 64) {
    const double x = Xc[j * ldc + r];
    ss += x * x;
    if (Vc) dv += x * Vc[j * ldc + r];
  }
  for (int o = 32; o > 0; o >>= 1) {
    ss += __shfl_xor(ss, o);
    dv += __shfl_xor(dv, o);
  }
  if (lane == 0) {
    const double nrm = sqrt(ss);
    const double v = (Vc && dv < 0.0) ? -nrm : nrm;
    // NaN would break the strict order the rank sort relies on
    norms[j] = isnan(v) ? -INFINITY : v;
  }
}

// Descending order, ties to the lower index: rank by counting.
__global__ __launch_bounds__(1024) void rank_sort_kernel(const double* __restrict__ norms,
                                                         int64_t m,
                                                         double* __restrict__ theta,
                                                         int32_t* __restrict__ order) {
  for (int64_t j = threadIdx.x; j < m; j += 1024) {
    const double v = norms[j];
    int64_t rank = 0;
    for (int64_t i = 0; i < m; ++i) {
      const double o = norms[i];
      rank += (o > v) || (o == v && i < j);
    }
    theta[rank] = v;
    order[rank] = static_cast<int32_t>(j);
  }
}

__global__ __launch_bounds__(256) void gather_top_kernel(
    const double* __restrict__ Xc, const double* __restrict__ Vc, int64_t ldc,
    int64_t m, int k, const double* __restrict__ theta,
    const int32_t* __restrict__ order, double* __restrict__ Uk, int64_t ldu,
    double* __restrict__ ritz) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < m * k) {
    const int64_t r = i / k;
    const int c = static_cast<int>(i - r * k);
    int64_t j = order[c];
    j = j < 0 ? 0 : (j >= m ? m - 1 : j);
    double v;
    if (Vc) {
      v = Vc[j * ldc + r];
    } else {
      const double th = theta[c];
      v = th > 0.0 ? Xc[j * ldc + r] / th : 0.0;
    }
    Uk[r * ldu + c] = v;
  }
  if (ritz && i < k) ritz[i] = sqrt(fmax(theta[i], 0.0));
}

template <int B2>
void round_dispatch(bool withv, int64_t m, int nb, int round, double* Xc,
                    double* Vc, int64_t ldc, double tol, int inner_max, Ctrl* ctrl,
                    hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(nb / 2));
  if (withv)
    jacobi_round_kernel<B2, true><<<grid, 256, 0, s>>>(m, nb, round, Xc, Vc, ldc,
                                                       tol, inner_max, ctrl);
  else
    jacobi_round_kernel<B2, false><<<grid, 256, 0, s>>>(m, nb, round, Xc, Vc, ldc,
                                                        tol, inner_max, ctrl);
}

}  // namespace

int jacobi_default_block(int64_t m) { return m <= 64 ? 8 : 16; }

int64_t jacobi_padded_cols(int64_t m, int b) {
  int64_t nb = cdiv(m, b);
  if (nb % 2) ++nb;
  if (nb < 2) nb = 2;
  return nb * b;
}

void launch_jacobi_init(const double* M, int64_t m, int64_t ldm, double* Xc,
                        double* Vc, int64_t ldc, int64_t nbp, hipStream_t s) {
  jacobi_init_kernel<<<static_cast<unsigned>(cdiv(nbp * m, 256)), 256, 0, s>>>(
      M, m, ldm, Xc, Vc, ldc, nbp);
}

void launch_jacobi_round(int b, int64_t m, int nb, int round, double* Xc,
                         double* Vc, int64_t ldc, double tol, int inner_max,
                         Ctrl* ctrl, hipStream_t s) {
  if (b == 8)
    round_dispatch<16>(Vc != nullptr, m, nb, round, Xc, Vc, ldc, tol, inner_max,
                       ctrl, s);
  else
    round_dispatch<32>(Vc != nullptr, m, nb, round, Xc, Vc, ldc, tol, inner_max,
                       ctrl, s);
}

void launch_jacobi_finalize(const double* Xc, const double* Vc, int64_t ldc,
                            int64_t m, int k, double* theta_sorted,
                            int32_t* order, double* norms, double* Uk,
                            int64_t ldu, double* ritz, hipStream_t s) {
  col_norm_kernel<<<static_cast<unsigned>(cdiv(m, 4)), 256, 0, s>>>(Xc, Vc, ldc, m,
                                                                    norms);
  rank_sort_kernel<<<1, 1024, 0, s>>>(norms, m, theta_sorted, order);
  const int64_t tot = m * k > k ? m * k : k;
  gather_top_kernel<<<static_cast<unsigned>(cdiv(tot, 256)), 256, 0, s>>>(
      Xc, Vc, ldc, m, k, theta_sorted, order, Uk, ldu, ritz);
}

}  // namespace bk
