// Top-k eigenpairs of the symmetric Rayleigh-Ritz matrix M (Algorithm 2,
// step 5) for moderate m, in three kernels:
//   1. Householder reduction M = H T H^T to tridiagonal T (one workgroup;
//      each step forms a reflector, the symmetric product p = beta M' v and
//      the rank-2 update M' -= v w^T + w v^T, Golub & Van Loan Sect. 8.3.1);
//   2. the k largest eigenvalues of T by multisection on Sturm counts, then
//      their eigenvectors by inverse iteration with a pivoted tridiagonal LU
//      (vectors of eigenvalues closer than a tiny tolerance are
//      re-orthogonalised inside their cluster);
//   3. back-transformation U_k = H_0 H_1 ... H_{m-3} X, one wavefront per
//      column.
// m serial reflector steps replace the O(m) rounds per sweep of Jacobi.
#include "kernels.hpp"

namespace bk {
namespace {

constexpr int TRI_THREADS = 1024;
constexpr int TRI_LDS_BLOCK = 120;  // trailing blocks up to this order live in LDS
constexpr int TRI_SMALL = 512;      // one-workgroup reduction up to this order

__device__ double block_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  // wave sums, then the 16 wave totals in order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TRI_THREADS / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// A (m x m, ld m, a symmetric copy of M, m <= TRI_THREADS) is reduced in
// place.  Outputs: reflector j (rows j+1..m-1) in column j of Vh
// (column-major, ld m), beta[j], diagonal dg[0..m), off-diagonal eo[0..m-1).
// The symmetric product and the rank-2 update run with threads owning
// columns of the trailing block (coalesced rows) and RG groups of rows whose
// partial sums are added in group order.
__global__ __launch_bounds__(TRI_THREADS) void tridiag_reduce_kernel(
    double* __restrict__ A, int64_t m, double* __restrict__ Vh,
    double* __restrict__ beta, double* __restrict__ dg, double* __restrict__ eo) {
  extern __shared__ double sm[];  // v, p, w: 3 m doubles; then the LDS block
  __shared__ double red[TRI_THREADS / 64];
  __shared__ double part[TRI_THREADS];
  __shared__ double s_beta;
  double* v = sm;
  double* p = sm + m;
  double* w = sm + 2 * m;
  double* blk = sm + 3 * m;  // TRI_LDS_BLOCK^2 doubles
  const int t = threadIdx.x;
  // Element (i, l) of the trailing matrix lives at base[(i - off) ld + l - off]:
  // in A (global, off 0) until it fits in LDS, then in blk.
  double* base = A;
  int64_t ld = m, off = 0;
  for (int64_t j = 0; j + 2 < m; ++j) {
    const int64_t j1 = j + 1;
    const int s = static_cast<int>(m - j1);
    if (base == A && m - j <= TRI_LDS_BLOCK) {
      const int64_t sb = m - j;
      for (int64_t idx = t; idx < sb * sb; idx += TRI_THREADS) {
        const int64_t r = idx / sb, c = idx - r * sb;
        blk[idx] = A[(j + r) * m + j + c];
      }
      __syncthreads();
      base = blk;
      ld = sb;
      off = j;
    }
    double* rowj = base + (j - off) * ld + (j1 - off);
    // x = column j below the diagonal = row j right of it (symmetric)
    double nrm2 = 0.0;
    for (int i = t; i < s; i += TRI_THREADS) {
      const double x = rowj[i];
      v[i] = x;
      nrm2 += x * x;
    }
    nrm2 = block_sum_1024(nrm2, red);
    if (t == 0) {
      const double x0 = v[0];
      const double nx = sqrt(nrm2);
      double b = 0.0, alpha = x0;
      if (nx > 0.0 && nrm2 - x0 * x0 > 0.0) {
        alpha = x0 >= 0.0 ? -nx : nx;
        const double v0 = x0 - alpha;
        const double vtv = nrm2 - x0 * x0 + v0 * v0;
        b = vtv > 0.0 ? 2.0 / vtv : 0.0;
        v[0] = v0;
      }
      s_beta = b;
      dg[j] = base[(j - off) * ld + (j - off)];
      eo[j] = alpha;
      beta[j] = b;
    }
    __syncthreads();
    const double b = s_beta;
    for (int i = t; i < s; i += TRI_THREADS) Vh[j * m + j1 + i] = v[i];
    if (b == 0.0) {  // column already reduced (uniform branch)
      __syncthreads();
      continue;
    }
    const int RG = (s <= TRI_THREADS / 4) ? 4 : ((s <= TRI_THREADS / 2) ? 2 : 1);
    const int CW = TRI_THREADS / RG;
    const int grp = t / CW, tc = t - grp * CW;
    const int rlen = (s + RG - 1) / RG;
    const int r0 = grp * rlen;
    const int r1 = (r0 + rlen < s) ? r0 + rlen : s;
    // p = b M' v, p_l = sum_i M'[i][l] v_i
    double acc = 0.0;
    if (tc < s) {
      const double* col = base + (j1 + r0 - off) * ld + (j1 - off) + tc;
      int i = r0;
      // eight independent loads in flight per thread
      for (; i + 8 <= r1; i += 8, col += 8 * ld) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = col[u * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += a[u] * v[i + u];
      }
      for (; i < r1; ++i, col += ld) acc += *col * v[i];
    }
    part[t] = acc;
    __syncthreads();
    if (t < s) {
      double sum = 0.0;
      for (int g = 0; g < RG; ++g) sum += part[g * CW + t];
      p[t] = b * sum;
    }
    __syncthreads();
    double vp = 0.0;
    for (int i = t; i < s; i += TRI_THREADS) vp += v[i] * p[i];
    vp = block_sum_1024(vp, red);
    const double K = 0.5 * b * vp;
    for (int i = t; i < s; i += TRI_THREADS) w[i] = p[i] - K * v[i];
    __syncthreads();
    // M' -= v w^T + w v^T
    if (tc < s) {
      const double vl = v[tc], wl = w[tc];
      double* col = base + (j1 + r0 - off) * ld + (j1 - off) + tc;
      int i = r0;
      for (; i + 8 <= r1; i += 8, col += 8 * ld) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = col[u * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) col[u * ld] = a[u] - (v[i + u] * wl + w[i + u] * vl);
      }
      for (; i < r1; ++i, col += ld) *col -= v[i] * wl + w[i] * vl;
    }
    __syncthreads();
  }
  if (t == 0) {
    auto el = [&](int64_t i, int64_t l) { return base[(i - off) * ld + (l - off)]; };
    if (m >= 2) {
      dg[m - 2] = el(m - 2, m - 2);
      dg[m - 1] = el(m - 1, m - 1);
      eo[m - 2] = el(m - 1, m - 2);
    } else {
      dg[0] = A[0];
    }
  }
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
__device__ int sturm_count(const double* dg, const double* e2, int64_t m, double x,
                           double pivmin) {
  int cnt = 0;
  double q = dg[0] - x;
  if (q < 0.0) ++cnt;
  for (int64_t i = 1; i < m; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = dg[i] - x - e2[i - 1] / q;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// LU with partial pivoting of (T - lam I) (LAPACK dgttrf layout): rD holds
// the reciprocals of the pivots, DU / DU2 the two superdiagonals, DL the
// multipliers, piv the row exchanges; the running pivot stays in a register.
__device__ void tri_factor(const double* __restrict__ dg, const double* __restrict__ eo,
                           int64_t m, double lam, double tiny, double* __restrict__ rD,
                           double* __restrict__ DU, double* __restrict__ DU2,
                           double* __restrict__ DL, int* __restrict__ piv) {
  double Dc = dg[0] - lam;           // current pivot candidate D[i]
  double DUc = (m > 1) ? eo[0] : 0.0;  // current DU[i]
#pragma unroll 4
  for (int64_t i = 0; i + 1 < m; ++i) {
    const double sub = eo[i];                       // T[i+1][i]
    const double Dn = dg[i + 1] - lam;              // D[i+1] before elimination
    const double DUn = (i + 2 < m) ? eo[i + 1] : 0.0;  // DU[i+1] before
    if (fabs(Dc) >= fabs(sub)) {
      if (Dc == 0.0) Dc = tiny;
      const double f = sub / Dc;
      rD[i] = 1.0 / Dc;
      DU[i] = DUc;
      DU2[i] = 0.0;
      DL[i] = f;
      piv[i] = 0;
      Dc = Dn - f * DUc;
      DUc = DUn;
    } else {
      const double f = Dc / sub;
      rD[i] = 1.0 / sub;
      DU[i] = Dn;
      DU2[i] = DUn;
      DL[i] = f;
      piv[i] = 1;
      Dc = DUc - f * Dn;
      DUc = -f * DUn;
    }
  }
  if (Dc == 0.0) Dc = tiny;
  rD[m - 1] = 1.0 / Dc;
}

// Solve with the factors of tri_factor, b -> x in place.
__device__ void tri_solve(int64_t m, const double* __restrict__ rD,
                          const double* __restrict__ DU, const double* __restrict__ DU2,
                          const double* __restrict__ DL, const int* __restrict__ piv,
                          double* __restrict__ b) {
  double cur = b[0];
#pragma unroll 8
  for (int64_t i = 0; i + 1 < m; ++i) {
    double nxt = b[i + 1];
    if (piv[i]) {
      const double tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    b[i] = cur;
    cur = nxt - DL[i] * cur;
  }
  b[m - 1] = cur;
  double x1 = b[m - 1] * rD[m - 1];  // x[i+1]
  b[m - 1] = x1;
  double x2 = 0.0;                    // x[i+2]
  if (m >= 2) {
    const double x0 = (b[m - 2] - DU[m - 2] * x1) * rD[m - 2];
    b[m - 2] = x0;
    x2 = x1;
    x1 = x0;
  }
#pragma unroll 8
  for (int64_t i = m - 3; i >= 0; --i) {
    const double x0 = (b[i] - DU[i] * x1 - DU2[i] * x2) * rD[i];
    b[i] = x0;
    x2 = x1;
    x1 = x0;
  }
}

// k largest eigenvalues (descending) and the eigenvectors of T (X, m x k,
// column-major: column c at X + c m).  scratch: k * 5 m doubles + k * m ints.
__global__ __launch_bounds__(TRI_THREADS) void tridiag_topk_kernel(
    const double* __restrict__ dgg, const double* __restrict__ eog, int64_t m, int k,
    double* __restrict__ theta, double* __restrict__ X, double* __restrict__ scratch,
    int* __restrict__ iscratch) {
  extern __shared__ double sm[];  // dg (m), eo (m), e2 (m), lo (k), hi (k)
  __shared__ int s_done;
  __shared__ double s_tnorm;
  double* dg = sm;
  double* eo = sm + m;
  double* e2 = sm + 2 * m;
  double* lo = sm + 3 * m;
  double* hi = lo + k;
  const int t = threadIdx.x;
  for (int64_t i = t; i < m; i += TRI_THREADS) {
    dg[i] = dgg[i];
    eo[i] = (i + 1 < m) ? eog[i] : 0.0;
    e2[i] = eo[i] * eo[i];
  }
  __syncthreads();
  if (t == 0) {
    double gl = INFINITY, gu = -INFINITY, tn = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(eo[i - 1]) : 0.0) + (i + 1 < m ? fabs(eo[i]) : 0.0);
      gl = fmin(gl, dg[i] - r);
      gu = fmax(gu, dg[i] + r);
      tn = fmax(tn, fabs(dg[i]) + r);
    }
    const double pad = 2.2e-16 * tn * 4.0 + 1e-300;
    s_tnorm = tn;
    for (int c = 0; c < k; ++c) {
      lo[c] = gl - pad;
      hi[c] = gu + pad;
    }
  }
  __syncthreads();
  const double tnorm = s_tnorm;
  const double pivmin = 1e-290 + 2.2e-16 * 2.2e-16 * tnorm * tnorm * 1e-10;
  // Multisection: P threads per eigenvalue evaluate the count at P interior
  // points; the bracket [lo, hi] of the c-th largest shrinks P+1 fold.
  const int P = k >= TRI_THREADS ? 1 : TRI_THREADS / k;
  for (int it = 0; it < 200; ++it) {
    if (t == 0) s_done = 1;
    __syncthreads();
    double* cnts = scratch;  // k * P ints stored as doubles
    for (int idx = t; idx < k * P; idx += TRI_THREADS) {
      const int c = idx / P, pp = idx % P;
      const double l = lo[c], h = hi[c];
      const double x = l + (h - l) * static_cast<double>(pp + 1) / static_cast<double>(P + 1);
      cnts[idx] = static_cast<double>(sturm_count(dg, e2, m, x, pivmin));
    }
    __syncthreads();
    for (int c = t; c < k; c += TRI_THREADS) {
      const double l = lo[c], h = hi[c];
      if (h - l <= 2.2e-16 * fmax(fabs(l), fabs(h)) * 2.0 + 1e-18 * tnorm + 1e-300) continue;
      const int target = static_cast<int>(m) - 1 - c;  // ascending index
      double nl = l, nh = h;
      for (int pp = 0; pp < P; ++pp) {
        const double x = l + (h - l) * static_cast<double>(pp + 1) / static_cast<double>(P + 1);
        if (cnts[c * P + pp] > target) {
          nh = x;
          break;
        }
        nl = x;
      }
      lo[c] = nl;
      hi[c] = nh;
      if (nh - nl > 2.2e-16 * fmax(fabs(nl), fabs(nh)) * 2.0 + 1e-18 * tnorm + 1e-300)
        s_done = 0;
    }
    __syncthreads();
    if (s_done) break;
  }
  for (int c = t; c < k; c += TRI_THREADS) theta[c] = 0.5 * (lo[c] + hi[c]);
  __syncthreads();
  // Inverse iteration; eigenvalues closer than ctol form a cluster handled
  // by one thread in order (modified Gram-Schmidt against earlier members).
  const double ctol = 1e-10 * tnorm + 1e-300;
  const double tiny = 2.2e-16 * tnorm + 1e-300;
  for (int c = t; c < k; c += TRI_THREADS) {
    const bool starts = (c == 0) || (theta[c - 1] - theta[c] > ctol);
    if (!starts) continue;
    int ce = c + 1;
    while (ce < k && theta[ce - 1] - theta[ce] <= ctol) ++ce;
    double* rD = scratch + static_cast<int64_t>(c) * 5 * m;
    double* DU = rD + m;
    double* DU2 = DU + m;
    double* DL = DU2 + m;
    int* piv = iscratch + static_cast<int64_t>(c) * m;
    for (int cc = c; cc < ce; ++cc) {
      double* x = X + static_cast<int64_t>(cc) * m;
      // start vector: deterministic, not orthogonal to any eigenvector in general
      for (int64_t i = 0; i < m; ++i) {
        const uint32_t h = static_cast<uint32_t>(i) * 2654435761u + static_cast<uint32_t>(cc) * 40503u;
        x[i] = 0.5 + static_cast<double>(h >> 8) * (1.0 / 16777216.0);
      }
      const double lam = theta[cc] + (cc - c) * 2.0 * tiny;  // split exact ties
      tri_factor(dg, eo, m, lam, tiny, rD, DU, DU2, DL, piv);
      for (int iter = 0; iter < 3; ++iter) {
        tri_solve(m, rD, DU, DU2, DL, piv, x);
        for (int pj = c; pj < cc; ++pj) {
          const double* y = X + static_cast<int64_t>(pj) * m;
          double dot = 0.0;
          for (int64_t i = 0; i < m; ++i) dot += y[i] * x[i];
          for (int64_t i = 0; i < m; ++i) x[i] -= dot * y[i];
        }
        double nn = 0.0;
        for (int64_t i = 0; i < m; ++i) nn += x[i] * x[i];
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int64_t i = 0; i < m; ++i) x[i] *= inv;
      }
    }
  }
}

// U_k (m x k, row-major ld ldu) = H_0 ... H_{m-3} X, X column-major (ld m);
// one wavefront per column, reflectors applied from the last to the first.
template <int VR>
__global__ __launch_bounds__(256) void tridiag_back_kernel(const double* __restrict__ Vh,
                                                           const double* __restrict__ beta,
                                                           int64_t m, int k,
                                                           double* __restrict__ X,
                                                           double* __restrict__ Uk,
                                                           int64_t ldu,
                                                           const double* __restrict__ theta,
                                                           double* __restrict__ ritz) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= k) return;
  const int lane = threadIdx.x & 63;
  if (ritz && lane == 0) ritz[c] = sqrt(fmax(theta[c], 0.0));
  const double* x = X + static_cast<int64_t>(c) * m;
  // column in registers (row lane + 64 u); next reflector prefetched
  double xr[VR], vc[VR], vn[VR];
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t i = lane + 64 * u;
    xr[u] = i < m ? x[i] : 0.0;
  }
  int64_t j = m - 3;
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t i = lane + 64 * u;
    vn[u] = (j >= 0 && i > j && i < m) ? Vh[j * m + i] : 0.0;
  }
  for (; j >= 0; --j) {
#pragma unroll
    for (int u = 0; u < VR; ++u) vc[u] = vn[u];
    const double b = beta[j];
    if (j > 0) {
#pragma unroll
      for (int u = 0; u < VR; ++u) {
        const int64_t i = lane + 64 * u;
        vn[u] = (i > j - 1 && i < m) ? Vh[(j - 1) * m + i] : 0.0;
      }
    }
    if (b == 0.0) continue;
    double dot = 0.0;
#pragma unroll
    for (int u = 0; u < VR; ++u) dot += vc[u] * xr[u];
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    const double f = b * dot;
#pragma unroll
    for (int u = 0; u < VR; ++u) xr[u] -= f * vc[u];
  }
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t i = lane + 64 * u;
    if (i < m) Uk[i * ldu + c] = xr[u];
  }
}

// ------------------------------------------------- large m (> TRI_SMALL) --
// The same reduction with the trailing block in global memory and the work
// of a step spread over the chip, in two launches per step:
//   tribig_step_kernel (one workgroup): finishes step j-1 (p = beta A' v
//     from the column partial sums, w = p - (beta v^T p / 2) v, which become
//     the pending update) and forms reflector j from column j with that
//     update applied (row j of the symmetric square, read contiguously);
//   tribig_update_kernel (grid): applies the pending update to the trailing
//     square (both triangles, a thread per column, 64-row groups) and
//     writes the partial sums of A' v_j per row group, added in group order
//     by the next step kernel.
constexpr int TBG_ROWS = 64;
constexpr int TBG_COLS = 256;

__global__ __launch_bounds__(1024) void tribig_step_kernel(
    double* __restrict__ A, int64_t m, int64_t j, double* __restrict__ v,
    double* __restrict__ vp, double* __restrict__ wp, const double* __restrict__ part, int G,
    double* __restrict__ Vh, double* __restrict__ beta, double* __restrict__ dg,
    double* __restrict__ eo) {
  extern __shared__ double p_s[];  // m
  __shared__ double red[TRI_THREADS / 64];
  __shared__ double s_diag;
  const int t = threadIdx.x;
  if (j >= 1) {
    // finish step j-1 over rows / columns j .. m-1
    const double bprev = beta[j - 1];
    double vtp = 0.0;
    for (int64_t l = j + t; l < m; l += TRI_THREADS) {
      double sum = 0.0;
      for (int g = 0; g < G; ++g) sum += part[g * m + l];
      const double pl = bprev * sum;
      p_s[l] = pl;
      vtp += v[l] * pl;
    }
    vtp = block_sum_1024(vtp, red);
    const double K = 0.5 * bprev * vtp;
    for (int64_t l = j + t; l < m; l += TRI_THREADS) {
      const double vl = v[l];
      vp[l] = vl;
      wp[l] = p_s[l] - K * vl;
    }
    __syncthreads();
  }
  const double vpj = vp[j], wpj = wp[j];
  if (j + 2 >= m) {  // last 2 x 2 block: its entries with the update applied
    if (t == 0) {
      const int64_t a = m - 2, c = m - 1;
      dg[a] = A[a * m + a] - 2.0 * vp[a] * wp[a];
      dg[c] = A[c * m + c] - 2.0 * vp[c] * wp[c];
      eo[a] = A[c * m + a] - vp[c] * wp[a] - wp[c] * vp[a];
    }
    return;
  }
  const int64_t j1 = j + 1;
  double nrm2 = 0.0;
  for (int64_t i = j + t; i < m; i += TRI_THREADS) {
    const double x = A[j * m + i] - vp[i] * wpj - wp[i] * vpj;
    if (i == j) {
      s_diag = x;
    } else {
      v[i] = x;
      nrm2 += x * x;
    }
  }
  nrm2 = block_sum_1024(nrm2, red);
  if (t == 0) {
    const double x0 = v[j1];
    const double nx = sqrt(nrm2);
    double b = 0.0, alpha = x0;
    if (nx > 0.0 && nrm2 - x0 * x0 > 0.0) {
      alpha = x0 >= 0.0 ? -nx : nx;
      const double v0 = x0 - alpha;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
      b = vtv > 0.0 ? 2.0 / vtv : 0.0;
      v[j1] = v0;
    }
    dg[j] = s_diag;
    eo[j] = alpha;
    beta[j] = b;
  }
  __syncthreads();
  for (int64_t i = j1 + t; i < m; i += TRI_THREADS) Vh[j * m + i] = v[i];
}

__global__ __launch_bounds__(TBG_COLS) void tribig_update_kernel(
    double* __restrict__ A, int64_t m, int64_t j, const double* __restrict__ v,
    const double* __restrict__ vp, const double* __restrict__ wp, double* __restrict__ part) {
  __shared__ double rv[TBG_ROWS], rvp[TBG_ROWS], rwp[TBG_ROWS];
  const int t = threadIdx.x;
  const int64_t j1 = j + 1;
  const int64_t r0 = j1 + static_cast<int64_t>(blockIdx.y) * TBG_ROWS;
  const int64_t r1 = (r0 + TBG_ROWS < m) ? r0 + TBG_ROWS : m;
  if (t < TBG_ROWS) {
    const int64_t i = r0 + t;
    rv[t] = i < m ? v[i] : 0.0;
    rvp[t] = i < m ? vp[i] : 0.0;
    rwp[t] = i < m ? wp[i] : 0.0;
  }
  __syncthreads();
  const int64_t l = j1 + static_cast<int64_t>(blockIdx.x) * TBG_COLS + t;
  if (l >= m) return;
  const double vpl = vp[l], wpl = wp[l];
  double* e = A + r0 * m + l;
  const int nr = static_cast<int>(r1 - r0);
  double acc = 0.0;
  int u = 0;
  for (; u + 8 <= nr; u += 8) {
    double ev[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ev[q] = e[(u + q) * m];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double nv = ev[q] - rvp[u + q] * wpl - rwp[u + q] * vpl;
      e[(u + q) * m] = nv;
      acc += nv * rv[u + q];
    }
  }
  for (; u < nr; ++u) {
    const double nv = e[u * m] - rvp[u] * wpl - rwp[u] * vpl;
    e[u * m] = nv;
    acc += nv * rv[u];
  }
  part[blockIdx.y * m + l] = acc;
}

__global__ __launch_bounds__(256) void sym_copy_kernel(const double* __restrict__ M, int64_t m,
                                                       int64_t ldm, double* __restrict__ A) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx / m, j = idx - i * m;
  A[idx] = 0.5 * (M[i * ldm + j] + M[j * ldm + i]);
}

}  // namespace

int64_t tridiag_scratch_doubles(int64_t m, int k) {
  // A copy + Vh + beta/dg/eo + X + solver scratch (5 m per eigenvalue) +
  // pivots (k m ints) + (large m) v, vp, wp and the row-group partials
  const int64_t groups = cdiv(m, TBG_ROWS);
  return 2 * m * m + 3 * m + static_cast<int64_t>(k) * m +
         std::max<int64_t>(static_cast<int64_t>(k) * 5 * m, static_cast<int64_t>(k) * 1024) +
         (static_cast<int64_t>(k) * m + 1) / 2 + 3 * m + groups * m + 64;
}

void launch_tridiag_topk(const double* M, int64_t m, int64_t ldm, int k, double* scratch,
                         double* theta, double* Uk, int64_t ldu, double* ritz, hipStream_t s) {
  double* A = scratch;
  double* Vh = A + m * m;
  double* beta = Vh + m * m;
  double* dg = beta + m;
  double* eo = dg + m;
  double* X = eo + m;
  double* sol = X + static_cast<int64_t>(k) * m;
  double* pivd = sol + std::max<int64_t>(static_cast<int64_t>(k) * 5 * m,
                                         static_cast<int64_t>(k) * 1024);
  int* piv = reinterpret_cast<int*>(pivd);
  double* v = pivd + (static_cast<int64_t>(k) * m + 1) / 2;
  double* vp = v + m;
  double* wp = vp + m;
  double* part = wp + m;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_reduce_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_topk_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    attr = true;
  }
  sym_copy_kernel<<<static_cast<unsigned>(cdiv(m * m, 256)), 256, 0, s>>>(M, m, ldm, A);
  launch_fill_f64(Vh, m * m, 0.0, s);
  if (m <= TRI_SMALL) {
    const int64_t sb = m < TRI_LDS_BLOCK ? m : TRI_LDS_BLOCK;
    tridiag_reduce_kernel<<<1, TRI_THREADS, (3 * m + sb * sb) * sizeof(double), s>>>(
        A, m, Vh, beta, dg, eo);
  } else {
    launch_fill_f64(v, 3 * m, 0.0, s);  // v, vp, wp
    int G = 0;
    for (int64_t j = 0; j + 2 < m; ++j) {
      tribig_step_kernel<<<1, TRI_THREADS, m * sizeof(double), s>>>(A, m, j, v, vp, wp, part, G,
                                                                    Vh, beta, dg, eo);
      const int64_t sj = m - j - 1;
      G = static_cast<int>(cdiv(sj, TBG_ROWS));
      tribig_update_kernel<<<dim3(static_cast<unsigned>(cdiv(sj, TBG_COLS)),
                                  static_cast<unsigned>(G)),
                             TBG_COLS, 0, s>>>(A, m, j, v, vp, wp, part);
    }
    tribig_step_kernel<<<1, TRI_THREADS, m * sizeof(double), s>>>(A, m, m - 2, v, vp, wp, part,
                                                                  G, Vh, beta, dg, eo);
  }
  tridiag_topk_kernel<<<1, TRI_THREADS, (3 * m + 2 * k) * sizeof(double), s>>>(dg, eo, m, k,
                                                                             theta, X, sol, piv);
  const unsigned gb = static_cast<unsigned>(cdiv(k, 4));
  if (m <= 1024)
    tridiag_back_kernel<16><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else if (m <= 2048)
    tridiag_back_kernel<32><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else  // m <= kTridiagMax = 64 * 40
    tridiag_back_kernel<40><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
}

}  // namespace bk
