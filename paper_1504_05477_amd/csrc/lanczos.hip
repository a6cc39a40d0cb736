// The block-tridiagonal Rayleigh-Ritz matrix of block Lanczos (Section 4.2).
//
// The Krylov recurrence builds block i >= 1 as
//   B_i = A A^T Q_{i-1},   B_i - Q_<i C_i = Q_i R_i,
// with C_i = Q_<i^T B_i the projection coefficients (two passes, C_i = C1 +
// C2) and R_i = R3 R2 R1 from the three CholeskyQR passes.  Hence
//   T_{i-1,i-1} = Q_{i-1}^T A A^T Q_{i-1} = the rows of block i-1 in C_i,
//   T_{i,i-1}   = Q_i^T A A^T Q_{i-1}     = R_i,
// every other block of Q^T A A^T Q vanishes (Q_j^T A A^T Q_{i-1} with
// j < i-2 is (A A^T Q_j)^T Q_{i-1} and A A^T Q_j lies in span(Q_0..Q_{j+1})),
// and the last diagonal block is W_q^T W_q with W_q = A^T Q_q.  Blocks that
// broke down are zero (their R and C are zero), as in the dense product.
#include "kernels.hpp"

namespace bk {
namespace {

// P_i = R2_i R1_i for blocks i = 1 .. q (both upper triangular).
__global__ __launch_bounds__(256) void band_r21_kernel(int k, const double* __restrict__ Rband,
                                                       double* __restrict__ P) {
  const int i = 1 + static_cast<int>(blockIdx.y);
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= kk) return;
  const int r = static_cast<int>(e / k), c = static_cast<int>(e - static_cast<int64_t>(r) * k);
  const double* R1 = Rband + (3 * static_cast<int64_t>(i)) * kk;
  const double* R2 = R1 + kk;
  double s = 0.0;
  for (int b = r; b <= c; ++b) s += R2[static_cast<int64_t>(r) * k + b] * R1[static_cast<int64_t>(b) * k + c];
  P[static_cast<int64_t>(i) * kk + e] = s;  // zero below the diagonal (empty sum)
}

// M (m x m, ld ldm) = T, one thread per entry.
__global__ __launch_bounds__(256) void band_assemble_kernel(
    int64_t m, int k, int q, const double* __restrict__ Cband, int64_t cstride,
    const double* __restrict__ Rband, const double* __restrict__ P,
    const double* __restrict__ Tqq, double* __restrict__ M, int64_t ldm) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= m * m) return;
  const int64_t r = e / m, c = e - r * m;
  const int bi = static_cast<int>(r / k), bj = static_cast<int>(c / k);
  const int ri = static_cast<int>(r - static_cast<int64_t>(bi) * k);
  const int cj = static_cast<int>(c - static_cast<int64_t>(bj) * k);
  const int64_t kk = static_cast<int64_t>(k) * k;
  double v = 0.0;
  if (bi == bj) {
    const int64_t a = static_cast<int64_t>(ri) * k + cj, b = static_cast<int64_t>(cj) * k + ri;
    if (bi < q) {
      // block bi's rows of the two projection passes of block bi + 1
      const double* C1 = Cband + (2 * static_cast<int64_t>(bi + 1)) * cstride + bi * kk;
      const double* C2 = C1 + cstride;
      v = 0.5 * ((C1[a] + C2[a]) + (C1[b] + C2[b]));
    } else {
      v = 0.5 * (Tqq[a] + Tqq[b]);
    }
  } else if (bi == bj + 1 || bj == bi + 1) {
    // R_blk[rr][cc] = sum_{a = rr..cc} R3[rr][a] P[a][cc]; above the
    // diagonal its transpose
    const int blk = bi > bj ? bi : bj;
    const int rr = bi > bj ? ri : cj, cc = bi > bj ? cj : ri;
    const double* R3 = Rband + (3 * static_cast<int64_t>(blk) + 2) * kk;
    const double* Pb = P + static_cast<int64_t>(blk) * kk;
    for (int a = rr; a <= cc; ++a)
      v += R3[static_cast<int64_t>(rr) * k + a] * Pb[static_cast<int64_t>(a) * k + cc];
  }
  M[r * ldm + c] = v;
}

}  // namespace

int launch_block_tridiag(int64_t m, int k, int q, const double* Cband, int64_t cstride,
                         const double* Rband, double* P, const double* Tqq, double* M,
                         int64_t ldm, hipStream_t s) {
  int nl = 0;
  const int64_t kk = static_cast<int64_t>(k) * k;
  if (q > 0) {
    band_r21_kernel<<<dim3(static_cast<unsigned>(cdiv(kk, 256)), static_cast<unsigned>(q)), 256,
                      0, s>>>(k, Rband, P);
    ++nl;
  }
  band_assemble_kernel<<<static_cast<unsigned>(cdiv(m * m, 256)), 256, 0, s>>>(
      m, k, q, Cband, cstride, Rband, P, Tqq, M, ldm);
  return nl + 1;
}

}  // namespace bk
