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
constexpr int TRI_WAVES = TRI_THREADS / 64;
constexpr int64_t TRI_LDS_DOUBLES = 150 * 1024 / 8;  // dynamic LDS of the reduction
constexpr int TRI_VR = 16;                           // back-transformation: m <= 64 * TRI_VR

__device__ double block_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  // wave sums, then the 16 wave totals in order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TRI_WAVES; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ int64_t tri_off(int64_t r) { return r * (r + 1) / 2; }

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Householder tridiagonalisation of the symmetric A (m x m, ld m;
// m <= TRI_THREADS).  Outputs: reflector j (rows j+1..m-1) in column j of Vh
// (column-major, ld m), beta[j], diagonal dg[0..m), off-diagonal eo[0..m-1).
//
// Step j forms the reflector (v, beta) of column j, p = beta A' v and
// w = p - (beta v^T p / 2) v for the trailing block A', whose update
// A' -= v w^T + w v^T is left pending: step j+1 applies it to each element
// as it reads it for its own product and writes the element back once.
// Threads own columns of A' (RG groups of rows, added in group order), and
// the rows of a group sit in registers of the wavefront (lane u: row
// R0 + u) from where v_i, and the pending v_i, w_i, are broadcast.
// While A' is in global memory both triangles are kept and a column is
// read top to bottom.  Once its order is <= sb its lower triangle moves to
// LDS, packed by rows: a thread then reads row l left of the diagonal
// (pass A, read only) and, after a barrier, column l from the diagonal down
// (pass B, written back).
__global__ __launch_bounds__(TRI_THREADS) void tridiag_reduce_kernel(
    double* __restrict__ A, int64_t m, int64_t sb, double* __restrict__ Vh,
    double* __restrict__ beta, double* __restrict__ dg, double* __restrict__ eo) {
  extern __shared__ double sm[];
  __shared__ double red[TRI_WAVES];
  __shared__ double part[TRI_THREADS];
  __shared__ double s_beta, s_diag;
  double* v = sm;           // reflector of this step (absolute row index)
  double* vp = sm + m;      // pending update of the previous step: v, w
  double* wp = sm + 2 * m;
  double* pv = sm + 3 * m;  // p
  double* P = sm + 4 * m;   // packed lower triangle of the trailing block
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  for (int64_t i = t; i < m; i += TRI_THREADS) {
    v[i] = 0.0;
    vp[i] = 0.0;
    wp[i] = 0.0;
    pv[i] = 0.0;
  }
  bool inlds = false, pend = false;
  int64_t o = 0;
  __syncthreads();
  for (int64_t j = 0; j + 2 < m; ++j) {
    const int64_t j1 = j + 1;
    const int s = static_cast<int>(m - j1);
    if (!inlds && m - j <= sb) {
      for (int64_t r = wave; r < m - j; r += TRI_WAVES)
        for (int64_t c = lane; c <= r; c += 64) P[tri_off(r) + c] = A[(j + r) * m + j + c];
      inlds = true;
      o = j;
      __syncthreads();
    }
    // column j of the current matrix: stored value minus the pending update
    double nrm2 = 0.0;
    {
      const double vpj = vp[j], wpj = wp[j];
      for (int64_t i = j + t; i < m; i += TRI_THREADS) {
        const double e = inlds ? P[tri_off(i - o) + (j - o)] : A[i * m + j];
        const double x = e - vp[i] * wpj - wp[i] * vpj;
        if (i == j) {
          s_diag = x;
        } else {
          v[i] = x;
          nrm2 += x * x;
        }
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
      s_beta = b;
      dg[j] = s_diag;
      eo[j] = alpha;
      beta[j] = b;
    }
    __syncthreads();
    const double b = s_beta;
    for (int64_t i = j1 + t; i < m; i += TRI_THREADS) {
      Vh[j * m + i] = v[i];
      if (b == 0.0) v[i] = 0.0;  // identity reflector: no product
    }
    if (b == 0.0 && !pend) {  // nothing to apply, nothing to form (uniform)
      __syncthreads();
      continue;
    }
    __syncthreads();
    const int RG = (s <= TRI_THREADS / 4) ? 4 : ((s <= TRI_THREADS / 2) ? 2 : 1);
    const int CW = TRI_THREADS / RG;
    const int grp = t / CW, tc = t - grp * CW;
    const int rlen = (s + RG - 1) / RG;
    const int64_t R0 = j1 + static_cast<int64_t>(grp) * rlen;
    const int64_t R1 = (R0 + rlen < m) ? R0 + rlen : m;
    const int64_t l = j1 + tc;
    const bool colok = tc < s;
    const double vpl = colok ? vp[l] : 0.0, wpl = colok ? wp[l] : 0.0;
    const int64_t lw = j1 + (tc - lane);  // first column of this wavefront
    double acc = 0.0;
    for (int64_t c0 = R0; c0 < R1; c0 += 64) {  // chunks of 64 rows
      const int64_t ir = c0 + lane;
      const double qv = ir < R1 ? v[ir] : 0.0;
      const double qvp = ir < R1 ? vp[ir] : 0.0;
      const double qwp = ir < R1 ? wp[ir] : 0.0;
      const int cn = __builtin_amdgcn_readfirstlane(
          static_cast<int>((R1 - c0 < 64) ? R1 - c0 : 64));
      if (!inlds) {
        // whole column l (both triangles stored), written back; eight
        // loads in flight
        double* e = A + c0 * m + l;
        int u = 0;
        for (; u + 8 <= cn; u += 8, e += 8 * m) {
          double ev[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) ev[q] = colok ? e[q * m] : 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double nv = ev[q] - readlane_f64(qvp, u + q) * wpl - readlane_f64(qwp, u + q) * vpl;
            if (colok && pend) e[q * m] = nv;
            acc += nv * readlane_f64(qv, u + q);
          }
        }
        for (; u < cn; ++u, e += m) {
          const double ev = colok ? *e : 0.0;
          const double nv = ev - readlane_f64(qvp, u) * wpl - readlane_f64(qwp, u) * vpl;
          if (colok && pend) *e = nv;
          acc += nv * readlane_f64(qv, u);
        }
      } else {
        // pass A: row l left of the diagonal, i < l (read only)
        const int ua = __builtin_amdgcn_readfirstlane(static_cast<int>(
            (lw + 63 - c0 < cn) ? ((lw + 63 - c0 > 0) ? lw + 63 - c0 : 0) : cn));
        const double* ra = P + tri_off(l - o) + (c0 - o);
        int u = 0;
        for (; u + 8 <= ua; u += 8) {
          double ev[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) ev[q] = (colok && c0 + u + q < l) ? ra[u + q] : 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q)
            acc += (ev[q] - vpl * readlane_f64(qwp, u + q) - wpl * readlane_f64(qvp, u + q)) *
                   ((c0 + u + q < l) ? readlane_f64(qv, u + q) : 0.0);
        }
        for (; u < ua; ++u) {
          if (colok && c0 + u < l)
            acc += (ra[u] - vpl * readlane_f64(qwp, u) - wpl * readlane_f64(qvp, u)) *
                   readlane_f64(qv, u);
        }
      }
    }
    if (inlds) {
      __syncthreads();  // every pass-A read before any pass-B write
      for (int64_t c0 = R0; c0 < R1; c0 += 64) {
        const int64_t ir = c0 + lane;
        const double qv = ir < R1 ? v[ir] : 0.0;
        const double qvp = ir < R1 ? vp[ir] : 0.0;
        const double qwp = ir < R1 ? wp[ir] : 0.0;
        const int cn = __builtin_amdgcn_readfirstlane(
            static_cast<int>((R1 - c0 < 64) ? R1 - c0 : 64));
        // pass B: column l from the diagonal down, i >= l, written back
        const int ub = __builtin_amdgcn_readfirstlane(
            static_cast<int>((lw > c0) ? ((lw - c0 < cn) ? lw - c0 : cn) : 0));
        int64_t r = c0 + ub - o;
        double* e = P + tri_off(r) + (l - o);
        int u = ub;
        for (; u + 8 <= cn; u += 8) {
          double* ep[8];
          double ev[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            ep[q] = e;
            ++r;
            e += r;  // next packed row: offset grows by the row length
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) ev[q] = (colok && c0 + u + q >= l) ? *ep[q] : 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double nv = ev[q] - readlane_f64(qvp, u + q) * wpl - readlane_f64(qwp, u + q) * vpl;
            if (colok && c0 + u + q >= l) {
              if (pend) *ep[q] = nv;
              acc += nv * readlane_f64(qv, u + q);
            }
          }
        }
        for (; u < cn; ++u) {
          if (colok && c0 + u >= l) {
            const double nv = *e - readlane_f64(qvp, u) * wpl - readlane_f64(qwp, u) * vpl;
            if (pend) *e = nv;
            acc += nv * readlane_f64(qv, u);
          }
          ++r;
          e += r;
        }
      }
    }
    part[t] = acc;
    __syncthreads();
    if (t < s) {
      double sum = 0.0;
      for (int g = 0; g < RG; ++g) sum += part[g * CW + t];
      pv[j1 + t] = b * sum;
    }
    __syncthreads();
    double vtp = 0.0;
    for (int64_t i = j1 + t; i < m; i += TRI_THREADS) vtp += v[i] * pv[i];
    vtp = block_sum_1024(vtp, red);
    const double K = 0.5 * b * vtp;
    for (int64_t i = j1 + t; i < m; i += TRI_THREADS) {
      wp[i] = pv[i] - K * v[i];
      vp[i] = v[i];
    }
    pend = b != 0.0;
    __syncthreads();
  }
  if (t == 0) {
    auto el = [&](int64_t i, int64_t c) {  // i >= c
      return inlds ? P[tri_off(i - o) + (c - o)] : A[i * m + c];
    };
    if (m >= 2) {
      const int64_t a = m - 2, c = m - 1;
      dg[a] = el(a, a) - 2.0 * vp[a] * wp[a];
      dg[c] = el(c, c) - 2.0 * vp[c] * wp[c];
      eo[a] = el(c, a) - vp[c] * wp[a] - wp[c] * vp[a];
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
  double xr[TRI_VR], vc[TRI_VR], vn[TRI_VR];
#pragma unroll
  for (int u = 0; u < TRI_VR; ++u) {
    const int64_t i = lane + 64 * u;
    xr[u] = i < m ? x[i] : 0.0;
  }
  int64_t j = m - 3;
#pragma unroll
  for (int u = 0; u < TRI_VR; ++u) {
    const int64_t i = lane + 64 * u;
    vn[u] = (j >= 0 && i > j && i < m) ? Vh[j * m + i] : 0.0;
  }
  for (; j >= 0; --j) {
#pragma unroll
    for (int u = 0; u < TRI_VR; ++u) vc[u] = vn[u];
    const double b = beta[j];
    if (j > 0) {
#pragma unroll
      for (int u = 0; u < TRI_VR; ++u) {
        const int64_t i = lane + 64 * u;
        vn[u] = (i > j - 1 && i < m) ? Vh[(j - 1) * m + i] : 0.0;
      }
    }
    if (b == 0.0) continue;
    double dot = 0.0;
#pragma unroll
    for (int u = 0; u < TRI_VR; ++u) dot += vc[u] * xr[u];
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    const double f = b * dot;
#pragma unroll
    for (int u = 0; u < TRI_VR; ++u) xr[u] -= f * vc[u];
  }
#pragma unroll
  for (int u = 0; u < TRI_VR; ++u) {
    const int64_t i = lane + 64 * u;
    if (i < m) Uk[i * ldu + c] = xr[u];
  }
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
  // A copy + Vh + beta/dg/eo + X + solver scratch (5 m per eigenvalue) + ints
  return 2 * m * m + 3 * m + static_cast<int64_t>(k) * m +
         std::max<int64_t>(static_cast<int64_t>(k) * 5 * m, static_cast<int64_t>(k) * 1024) +
         static_cast<int64_t>(k) * m / 2 + 64;
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
  int* piv = reinterpret_cast<int*>(
      sol + std::max<int64_t>(static_cast<int64_t>(k) * 5 * m, static_cast<int64_t>(k) * 1024));
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
  // largest trailing order whose packed lower triangle fits beside 4 m doubles
  int64_t sb = 0;
  while (sb < m && 4 * m + (sb + 1) * (sb + 2) / 2 <= TRI_LDS_DOUBLES) ++sb;
  const size_t lds = static_cast<size_t>(4 * m + sb * (sb + 1) / 2) * sizeof(double);
  tridiag_reduce_kernel<<<1, TRI_THREADS, lds, s>>>(A, m, sb, Vh, beta, dg, eo);
  tridiag_topk_kernel<<<1, TRI_THREADS, (3 * m + 2 * k) * sizeof(double), s>>>(dg, eo, m, k,
                                                                             theta, X, sol, piv);
  tridiag_back_kernel<<<static_cast<unsigned>(cdiv(k, 4)), 256, 0, s>>>(Vh, beta, m, k, X, Uk,
                                                                       ldu, theta, ritz);
}

}  // namespace bk
