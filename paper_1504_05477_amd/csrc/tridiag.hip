// Top-k eigenpairs of the symmetric Rayleigh-Ritz matrix M (Algorithm 2,
// step 5) for moderate m, in three kernels:
//   1. Householder reduction M = H T H^T to tridiagonal T: each step forms
//      a reflector, the symmetric product p = beta M' v and the rank-2
//      update M' -= v w^T + w v^T (Golub & Van Loan Sect. 8.3.1); blocked
//      panels while the trailing block exceeds LDS, then one workgroup with
//      the block in LDS (for m <= 512; a grid per step beyond);
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
constexpr int TRI_SMALL = 512;      // one-workgroup reduction up to this order
constexpr int TRI_NB = 16;          // reflectors per panel of the blocked reduction
constexpr int TRI_SY = 32;          // tile order of the trailing rank-2 nb update
// dynamic LDS of the one-workgroup kernels (the static part[] and red[]
// arrays take the rest of the 160 KB)
constexpr int TRI_LDS_BYTES = 150 * 1024;

// Sum over the 64 lanes of a wavefront (all lanes active), the same value on
// every lane: DPP adds within quads (lane pairs, then pairs of pairs) and
// within 16-lane rows (rotations by 4 and 8), then the four row sums are read
// from lanes 0, 16, 32, 48 and added in that order.  Fixed order, no LDS.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return read_lane(v, 0) + read_lane(v, 16) + read_lane(v, 32) + read_lane(v, 48);
}

__device__ double block_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  // wave sums, then the 16 wave totals in order
  v = wave_sum(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TRI_THREADS / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Sum over the workgroup of one value per thread: wave sums by shuffles, then
// the 16 wave totals in wave order (the same on every thread, so every thread
// may take decisions on it).  One barrier; `red` must not be written again
// before a later barrier.
__device__ double wg_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  v = wave_sum(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < TRI_THREADS / 64; ++w) s += red[w];
  return s;
}

// Steps j_start .. m-3 with the trailing block of order sb0 = m - j_start in
// LDS (the earlier steps were taken by the panel kernels, which leave A's
// trailing block at j_start fully updated).  Outputs: reflector j (rows
// j+1..m-1) in column j of Vh (column-major, ld m), beta[j], diagonal
// dg[0..m), off-diagonal eo[0..m-1).
// The rank-2 update of step j-1 is applied lazily: to row j before it forms
// reflector j, and to the rest of the block in the same pass that forms
// p = beta M' v_j, so each element is read and written once per step.
// Threads own columns of the trailing block (RG groups of rows, partial sums
// added in group order); the reflector's scalars are formed by every thread
// from the same workgroup sum.
__global__ __launch_bounds__(TRI_THREADS) void tridiag_reduce_kernel(
    const double* __restrict__ A, int64_t m, int64_t j_start, double* __restrict__ Vh,
    double* __restrict__ beta, double* __restrict__ dg, double* __restrict__ eo) {
  extern __shared__ double sm[];  // v, pv, pw: 3 m doubles; then the block
  __shared__ double redA[TRI_THREADS / 64], redB[TRI_THREADS / 64];
  __shared__ double part[TRI_THREADS];
  const int t = threadIdx.x;
  const int sb0 = static_cast<int>(m - j_start);
  double* v = sm;
  double* pv = sm + m;      // pending update (v, w) of the previous step,
  double* pw = sm + 2 * m;  // index 0 = the current step's row j
  double* blk = sm + 3 * m;  // element (i, l) of the trailing square at
                             // blk[(i - j_start) sb0 + l - j_start]
  for (int idx = t; idx < sb0 * sb0; idx += TRI_THREADS) {
    const int r = idx / sb0, c = idx - r * sb0;
    blk[idx] = A[(j_start + r) * m + j_start + c];
  }
  for (int i = t; i < sb0; i += TRI_THREADS) {
    pv[i] = 0.0;
    pw[i] = 0.0;
  }
  __syncthreads();
  for (int64_t j = j_start; j + 2 < m; ++j) {
    const int64_t j1 = j + 1;
    const int s = static_cast<int>(m - j1);
    const int o = static_cast<int>(j - j_start);  // block row / column of j
    double* rowj = blk + o * sb0 + o;
    // row j with the pending update, columns j .. m-1
    const double pv0 = pv[0], pw0 = pw[0];
    double nrm2 = 0.0;
    for (int l = t; l <= s; l += TRI_THREADS) {
      const double x = rowj[l] - (pv0 * pw[l] + pw0 * pv[l]);
      if (l == 0) {
        dg[j] = x;
      } else {
        v[l - 1] = x;
        nrm2 += x * x;
      }
    }
    nrm2 = wg_sum_1024(nrm2, redA);
    // reflector scalars on every thread; v[0] stays x0 in LDS, v0 is used
    // for index 0 from registers
    const double x0 = v[0];
    const double nx = sqrt(nrm2);
    double b = 0.0, alpha = x0, v0 = x0;
    if (nx > 0.0 && nrm2 - x0 * x0 > 0.0) {
      alpha = x0 >= 0.0 ? -nx : nx;
      v0 = x0 - alpha;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
      b = vtv > 0.0 ? 2.0 / vtv : 0.0;
    }
    if (t == 0) {
      eo[j] = alpha;
      beta[j] = b;
    }
    for (int i = t; i < s; i += TRI_THREADS) Vh[j * m + j1 + i] = i == 0 ? v0 : v[i];
    // fused pass over rows / columns j1 .. m-1: apply the pending update
    // (pv, pw indexed from row j) and accumulate M' v
    const int CW = ((s + 63) / 64) * 64;
    const int RG = TRI_THREADS / CW;
    const int grp = t / CW, tc = t - grp * CW;
    const int rlen = (s + RG - 1) / RG;
    const int r0 = grp * rlen;
    const int r1 = (r0 + rlen < s) ? r0 + rlen : s;
    double acc = 0.0;
    if (grp < RG && tc < s) {
      const double pvl = pv[1 + tc], pwl = pw[1 + tc];
      double* col = rowj + sb0 + 1 + tc + r0 * sb0;  // (j1 + r0, j1 + tc)
#pragma unroll 4
      for (int i = r0; i < r1; ++i, col += sb0) {
        const double a = *col - (pv[1 + i] * pwl + pw[1 + i] * pvl);
        *col = a;
        acc += a * (i == 0 ? v0 : v[i]);
      }
    }
    part[t] = acc;
    __syncthreads();
    double pl = 0.0, vl = 0.0;
    if (t < s) {
      double sum = 0.0;
      for (int g = 0; g < RG; ++g) sum += part[g * CW + t];
      pl = b * sum;
      vl = t == 0 ? v0 : v[t];
    }
    const double vp = wg_sum_1024(vl * pl, redB);
    const double K = 0.5 * b * vp;
    // the pending update of the next step, indexed from row j1
    if (t < s) {
      pv[t] = vl;
      pw[t] = pl - K * vl;
    }
    __syncthreads();
  }
  if (t == 0) {
    // last 2 x 2 block with the pending update of step m-3 applied
    if (m >= 2) {
      const int o = sb0 - 2;
      const double* b2 = blk + o * sb0 + o;
      dg[m - 2] = b2[0] - 2.0 * pv[0] * pw[0];
      dg[m - 1] = b2[sb0 + 1] - 2.0 * pv[1] * pw[1];
      eo[m - 2] = b2[sb0] - (pv[1] * pw[0] + pw[1] * pv[0]);
    } else {
      dg[0] = A[0];
    }
  }
}

// ------------------------------------------ blocked steps (m <= TRI_SMALL) --
// While the trailing block is too large for LDS, reflectors are formed in
// panels of up to TRI_NB steps (the blocked reduction of Golub & Van Loan
// Sect. 8.3.1, as in LAPACK's sytrd): inside a panel the trailing block keeps
// its value A0 from the panel's start and the current matrix is
// A0 - V W^T - W V^T, V and W holding the panel's reflectors v_q and their
// vectors w_q = p_q - K_q v_q (zero above row j_q + 1).  A step reads A0 once
// for A0 v and corrects the product with V (W^T v) + W (V^T v); the
// rank-2 nb update of A0 runs once per panel over the whole chip.

// One workgroup, steps j0 .. j0 + nst - 1.  V and W live in LDS column by
// column (ld mr = m - j0, row x is row j0 + x); on exit their rows from
// j0 + nst on go to Vg, Wg (column q at q m, ld m, absolute rows).  The
// first R rows of the panel-start block (rows j0 .. j0 + R - 1, columns
// j0 .. m - 1) are staged in LDS once; each step's A0 v pass reads them
// there and the rest from memory, the rows dealt to the row groups in turn
// so that every group gets its share of both.
__global__ __launch_bounds__(TRI_THREADS) void tri_panel_kernel(
    const double* __restrict__ A, int64_t m, int64_t j0, int nst, int R,
    double* __restrict__ Vg, double* __restrict__ Wg, double* __restrict__ Vh,
    double* __restrict__ beta, double* __restrict__ dg, double* __restrict__ eo) {
  extern __shared__ double sm[];  // v[m], p[m], c[2 TRI_NB], V, W [TRI_NB x mr], A0s [R x mr]
  __shared__ double red[TRI_THREADS / 64];
  __shared__ double part[TRI_THREADS];
  __shared__ double s_beta;
  const int64_t mr = m - j0;
  double* v = sm;
  double* p = v + m;
  double* c = p + m;
  double* V = c + 2 * TRI_NB;
  double* W = V + TRI_NB * mr;
  double* A0s = W + TRI_NB * mr;
  const int t = threadIdx.x;
  for (int64_t idx = t; idx < 2 * TRI_NB * mr; idx += TRI_THREADS) V[idx] = 0.0;
  for (int64_t idx = t; idx < static_cast<int64_t>(R) * mr; idx += TRI_THREADS) {
    const int64_t r = idx / mr, cc = idx - r * mr;
    A0s[idx] = A[(j0 + r) * m + j0 + cc];
  }
  __syncthreads();
  for (int jj = 0; jj < nst; ++jj) {
    const int64_t j = j0 + jj, j1 = j + 1;
    const int s = static_cast<int>(m - j1);
    // row j of the current matrix, columns j .. m-1 (x = panel row)
    double nrm2 = 0.0;
    for (int l = t; l <= s; l += TRI_THREADS) {
      const int64_t xl = jj + l;
      double x = A[j * m + j + l];
      for (int q = 0; q < jj; ++q)
        x -= V[q * mr + jj] * W[q * mr + xl] + W[q * mr + jj] * V[q * mr + xl];
      if (l == 0) {
        dg[j] = x;
      } else {
        v[l - 1] = x;
        nrm2 += x * x;
      }
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
      eo[j] = alpha;
      beta[j] = b;
    }
    __syncthreads();
    const double b = s_beta;
    for (int i = t; i < s; i += TRI_THREADS) Vh[j * m + j1 + i] = v[i];
    if (b == 0.0) {  // column already reduced: V, W columns jj stay zero
      __syncthreads();
      continue;
    }
    const int RG = (s <= TRI_THREADS / 4) ? 4 : ((s <= TRI_THREADS / 2) ? 2 : 1);
    const int CW = TRI_THREADS / RG;
    const int grp = t / CW, tc = t - grp * CW;
    // A0' v over rows / columns j1 .. m-1; group grp takes rows grp,
    // grp + RG, ...: those of the staged rows (i < iL) from LDS first
    double acc = 0.0;
    if (tc < s) {
      const int64_t iL64 = j0 + R - j1;
      const int iL = static_cast<int>(iL64 < s ? iL64 : s);
      const int64_t off = j1 - j0;
      const double* lcol = A0s + off * mr + off + tc;
      int i = grp;
      for (; i < iL; i += RG) acc += lcol[static_cast<int64_t>(i) * mr] * v[i];
      const double* col = A + (j1 + i) * m + j1 + tc;
      const int64_t step = static_cast<int64_t>(RG) * m;
      for (; i + 7 * RG < s; i += 8 * RG, col += 8 * step) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = col[u * step];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += a[u] * v[i + u * RG];
      }
      for (; i < s; i += RG, col += step) acc += *col * v[i];
    }
    part[t] = acc;
    // c[q] = W'^T v, c[jj + q] = V'^T v over the panel rows of j1 .. m-1
    {
      const int wv = t >> 6, ln = t & 63;
      for (int qq = wv; qq < 2 * jj; qq += TRI_THREADS / 64) {
        const double* colq = (qq < jj ? W + qq * mr : V + (qq - jj) * mr) + jj + 1;
        double sum = 0.0;
        for (int i = ln; i < s; i += 64) sum += colq[i] * v[i];
        sum = wave_sum(sum);
        if (ln == 0) c[qq] = sum;
      }
    }
    __syncthreads();
    if (t < s) {
      double sum = 0.0;
      for (int g = 0; g < RG; ++g) sum += part[g * CW + t];
      const int64_t xl = jj + 1 + t;
      for (int q = 0; q < jj; ++q) sum -= V[q * mr + xl] * c[q] + W[q * mr + xl] * c[jj + q];
      p[t] = b * sum;
    }
    __syncthreads();
    double vp = 0.0;
    for (int i = t; i < s; i += TRI_THREADS) vp += v[i] * p[i];
    vp = block_sum_1024(vp, red);
    const double K = 0.5 * b * vp;
    for (int i = t; i < s; i += TRI_THREADS) {
      const int64_t xi = jj + 1 + i;
      V[jj * mr + xi] = v[i];
      W[jj * mr + xi] = p[i] - K * v[i];
    }
    __syncthreads();
  }
  const int64_t jn = j0 + nst;
  for (int64_t idx = t; idx < TRI_NB * (m - jn); idx += TRI_THREADS) {
    const int64_t q = idx / (m - jn), i = jn + idx - q * (m - jn);
    Vg[q * m + i] = V[q * mr + (i - j0)];
    Wg[q * m + i] = W[q * mr + (i - j0)];
  }
}

// A0[i][l] -= sum_q V[i][q] W[l][q] + W[i][q] V[l][q] over the trailing
// square i, l >= jn; TRI_SY x TRI_SY tiles, a thread per column and every
// eighth row of its tile.
__global__ __launch_bounds__(256) void tri_syr2k_kernel(double* __restrict__ A, int64_t m,
                                                        int64_t jn, const double* __restrict__ Vg,
                                                        const double* __restrict__ Wg, int nst) {
  __shared__ double vr[TRI_NB][TRI_SY], wr[TRI_NB][TRI_SY];
  const int t = threadIdx.x;
  const int64_t i0 = jn + static_cast<int64_t>(blockIdx.y) * TRI_SY;
  const int64_t l0 = jn + static_cast<int64_t>(blockIdx.x) * TRI_SY;
  for (int idx = t; idx < TRI_NB * TRI_SY; idx += 256) {
    const int q = idx / TRI_SY, r = idx - q * TRI_SY;
    const int64_t i = i0 + r;
    const bool ok = q < nst && i < m;
    vr[q][r] = ok ? Vg[q * m + i] : 0.0;
    wr[q][r] = ok ? Wg[q * m + i] : 0.0;
  }
  __syncthreads();
  const int tx = t & (TRI_SY - 1), ty = t / TRI_SY;
  const int64_t l = l0 + tx;
  if (l >= m) return;
  double vl[TRI_NB], wl[TRI_NB];
#pragma unroll
  for (int q = 0; q < TRI_NB; ++q) {
    vl[q] = q < nst ? Vg[q * m + l] : 0.0;
    wl[q] = q < nst ? Wg[q * m + l] : 0.0;
  }
  for (int r = ty; r < TRI_SY; r += 256 / TRI_SY) {
    const int64_t i = i0 + r;
    if (i >= m) break;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < TRI_NB; ++q) sum += vr[q][r] * wl[q] + wr[q][r] * vl[q];
    A[i * m + l] -= sum;
  }
}

// 1 / q from the hardware reciprocal and two Newton steps (each roughly
// squares the relative error; the last one leaves about one ulp), four
// dependent operations instead of the division sequence.
__device__ __forceinline__ double recip_f64(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// Number of eigenvalues of T below x, from the signs of the leading
// principal minors a_i of T - x I: a_i = (d_i - x) a_{i-1} - e_{i-1}^2 a_{i-2}
// (a_{-1} = 1), whose ratios a_i / a_{i-1} are the LDL^T pivots, so a pivot
// is negative exactly where consecutive minors change sign.  A pivot of
// magnitude below pivmin is replaced by -pivmin (a_i = -pivmin a_{i-1}) and
// so counted.  No division: one fma, a compare and a select per step on the
// dependency chain (e^2 a_{i-2} is formed a step ahead).  The minors are
// rescaled by a power of two every eight steps (exact); T must be scaled so
// that its entries are at most about 1, so that eight steps cannot overflow.
// The diagonal and e^2 are read eight at a time ahead of the chain.
__device__ int sturm_count(const double* dg, const double* e2, int64_t m, double x,
                           double pivmin) {
  double ap = 1.0;
  double a = dg[0] - x;
  if (fabs(a) < pivmin) a = -pivmin;
  bool sg = a < 0.0;
  int cnt = sg ? 1 : 0;
  int64_t i = 1;
  for (; i + 8 <= m; i += 8) {
    double dd[8], ee[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dd[u] = dg[i + u] - x;
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double an = fma(dd[u], a, -ee[u] * ap);
      if (fabs(an) < pivmin * fabs(a)) an = -pivmin * a;
      ap = a;
      a = an;
      const bool sn = a < 0.0;
      cnt += (sn != sg) ? 1 : 0;
      sg = sn;
    }
    int ex;
    (void)frexp(a, &ex);
    a = ldexp(a, -ex);
    ap = ldexp(ap, -ex);
  }
  for (; i < m; ++i) {
    double an = fma(dg[i] - x, a, -e2[i - 1] * ap);
    if (fabs(an) < pivmin * fabs(a)) an = -pivmin * a;
    ap = a;
    a = an;
    const bool sn = a < 0.0;
    cnt += (sn != sg) ? 1 : 0;
    sg = sn;
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
      const double r = recip_f64(Dc);
      const double f = sub * r;
      rD[i] = r;
      DU[i] = DUc;
      DU2[i] = 0.0;
      DL[i] = f;
      piv[i] = 0;
      Dc = Dn - f * DUc;
      DUc = DUn;
    } else {
      const double r = recip_f64(sub);
      const double f = Dc * r;
      rD[i] = r;
      DU[i] = Dn;
      DU2[i] = DUn;
      DL[i] = f;
      piv[i] = 1;
      Dc = DUc - f * Dn;
      DUc = -f * DUn;
    }
  }
  if (Dc == 0.0) Dc = tiny;
  rD[m - 1] = recip_f64(Dc);
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

// Gershgorin bounds of T (diagonal dgg, off-diagonal eog, m) and its
// infinity norm, by one workgroup of `nt` threads (order-free min / max).
__device__ void tri_gershgorin(const double* __restrict__ dgg, const double* __restrict__ eog,
                               int64_t m, int nt, double* red, double* gl, double* gu,
                               double* tn) {
  const int t = threadIdx.x;
  double l = INFINITY, u = -INFINITY, n = 0.0;
  for (int64_t i = t; i < m; i += nt) {
    const double r = (i > 0 ? fabs(eog[i - 1]) : 0.0) + (i + 1 < m ? fabs(eog[i]) : 0.0);
    l = fmin(l, dgg[i] - r);
    u = fmax(u, dgg[i] + r);
    n = fmax(n, fabs(dgg[i]) + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_xor(l, o));
    u = fmax(u, __shfl_xor(u, o));
    n = fmax(n, __shfl_xor(n, o));
  }
  const int nw = nt >> 6, w = t >> 6;
  if ((t & 63) == 0) {
    red[w] = l;
    red[nw + w] = u;
    red[2 * nw + w] = n;
  }
  __syncthreads();
  l = red[0];
  u = red[nw];
  n = red[2 * nw];
  for (int q = 1; q < nw; ++q) {
    l = fmin(l, red[q]);
    u = fmax(u, red[nw + q]);
    n = fmax(n, red[2 * nw + q]);
  }
  *gl = l;
  *gu = u;
  *tn = n;
}

// The c-th largest eigenvalue of T (c = blockIdx.x) by multisection: the
// BS_THREADS threads evaluate the Sturm count at P = BS_THREADS interior
// points x_0 < ... < x_{P-1} of the bracket [lo, hi] (count(lo) <= target <
// count(hi), target = m - 1 - c its ascending index); the new bracket is
// [x_b, x_{b+1}] for b the last point with count <= target (lo for b = -1,
// hi for b = P-1), P + 1 fold smaller.  One workgroup per eigenvalue: no
// synchronization between them.
constexpr int BS_THREADS = 256;

__global__ __launch_bounds__(BS_THREADS) void tridiag_bisect_kernel(
    const double* __restrict__ dgg, const double* __restrict__ eog, int64_t m, int k,
    double* __restrict__ theta) {
  extern __shared__ double sm[];  // dg (m), e2 (m)
  __shared__ double red[3 * BS_THREADS / 64];
  __shared__ double s_lo, s_hi;
  __shared__ int s_best;
  double* dg = sm;
  double* e2 = sm + m;
  const int t = threadIdx.x, c = blockIdx.x;
  double gl, gu, tnorm;
  tri_gershgorin(dgg, eog, m, BS_THREADS, red, &gl, &gu, &tnorm);
  // the Sturm counts run on T sc, sc a power of two with |T sc| <= 1 (exact
  // scaling: the counts are those of T at the unscaled points)
  int tex = 0;
  (void)frexp(tnorm > 0.0 ? tnorm : 1.0, &tex);
  const double sc = ldexp(1.0, -tex);
  for (int64_t i = t; i < m; i += BS_THREADS) {
    dg[i] = dgg[i] * sc;
    const double e = (i + 1 < m) ? eog[i] * sc : 0.0;
    e2[i] = e * e;
  }
  __syncthreads();
  const double pad = 2.2e-16 * tnorm * 4.0 + 1e-300;
  const double pivmin = (1e-290 + 2.2e-16 * 2.2e-16 * tnorm * tnorm * 1e-10) * sc;
  const int P = BS_THREADS;
  auto settled = [&](double l, double h) {
    return h - l <= 2.2e-16 * fmax(fabs(l), fabs(h)) * 2.0 + 1e-18 * tnorm + 1e-300;
  };
  auto point = [&](double l, double h, int pp) {
    return l + (h - l) * static_cast<double>(pp + 1) / static_cast<double>(P + 1);
  };
  if (t == 0) {
    s_lo = gl - pad;
    s_hi = gu + pad;
    s_best = -1;
  }
  __syncthreads();
  const int target = static_cast<int>(m) - 1 - c;
  for (int it = 0; it < 200; ++it) {
    const double l = s_lo, h = s_hi;
    if (settled(l, h)) break;  // (uniform)
    if (sturm_count(dg, e2, m, point(l, h, t) * sc, pivmin) <= target) atomicMax(&s_best, t);
    __syncthreads();
    if (t == 0) {
      const int b = s_best;
      s_lo = b >= 0 ? point(l, h, b) : l;
      s_hi = b + 1 < P ? point(l, h, b + 1) : h;
      s_best = -1;
    }
    __syncthreads();
  }
  if (t == 0) theta[c] = 0.5 * (s_lo + s_hi);
}

// Inverse iteration for the eigenvalues theta (descending) of T, into X
// (m x k, column-major: column c at X + c m).  Eigenvalues closer than ctol
// form a cluster handled by one workgroup (the one of its first member) in
// order, modified Gram-Schmidt against the earlier members.  A workgroup is
// one wavefront: lane 0 runs the factorization and the two triangular
// sweeps, the wavefront the start vector, dot products and scalings.
// use_lds: the factors and the working vector in LDS, else in scratch
// (5 m doubles per eigenvalue) and iscratch (m ints).
__global__ __launch_bounds__(64) void tridiag_invit_kernel(
    const double* __restrict__ dgg, const double* __restrict__ eog, int64_t m, int k,
    const double* __restrict__ theta, double* __restrict__ X, double* __restrict__ scratch,
    int* __restrict__ iscratch, int use_lds) {
  extern __shared__ double sm[];  // dg (m), eo (m) [, rD DU DU2 DL x (5 m), piv (m ints)]
  __shared__ double red[3];
  const int t = threadIdx.x, c = blockIdx.x;
  double* dg = sm;
  double* eo = sm + m;
  for (int64_t i = t; i < m; i += 64) {
    dg[i] = dgg[i];
    eo[i] = (i + 1 < m) ? eog[i] : 0.0;
  }
  double gl, gu, tnorm;
  tri_gershgorin(dgg, eog, m, 64, red, &gl, &gu, &tnorm);
  const double ctol = 1e-10 * tnorm + 1e-300;
  const double tiny = 2.2e-16 * tnorm + 1e-300;
  if (c > 0 && theta[c - 1] - theta[c] <= ctol) return;  // (uniform) not a first member
  int ce = c + 1;
  while (ce < k && theta[ce - 1] - theta[ce] <= ctol) ++ce;
  double* rD;
  double* xw = nullptr;
  int* piv;
  if (use_lds) {
    rD = sm + 2 * m;
    xw = rD + 4 * m;
    piv = reinterpret_cast<int*>(rD + 5 * m);
  } else {
    rD = scratch + static_cast<int64_t>(c) * 5 * m;
    piv = iscratch + static_cast<int64_t>(c) * m;
  }
  double* DU = rD + m;
  double* DU2 = DU + m;
  double* DL = DU2 + m;
  for (int cc = c; cc < ce; ++cc) {
    double* xg = X + static_cast<int64_t>(cc) * m;
    double* x = use_lds ? xw : xg;
    // start vector: deterministic, not orthogonal to any eigenvector in general
    for (int64_t i = t; i < m; i += 64) {
      const uint32_t h = static_cast<uint32_t>(i) * 2654435761u + static_cast<uint32_t>(cc) * 40503u;
      x[i] = 0.5 + static_cast<double>(h >> 8) * (1.0 / 16777216.0);
    }
    const double lam = theta[cc] + (cc - c) * 2.0 * tiny;  // split exact ties
    if (t == 0) tri_factor(dg, eo, m, lam, tiny, rD, DU, DU2, DL, piv);
    __syncthreads();
    // two solves: with lam accurate to a few ulps the first already damps
    // every other eigenvector by ~ eps |lam| / gap, the second is margin
    for (int iter = 0; iter < 2; ++iter) {
      if (t == 0) tri_solve(m, rD, DU, DU2, DL, piv, x);
      __syncthreads();
      for (int pj = c; pj < cc; ++pj) {
        const double* y = X + static_cast<int64_t>(pj) * m;  // (written by this workgroup)
        double dot = 0.0;
        for (int64_t i = t; i < m; i += 64) dot += y[i] * x[i];
        dot = wave_sum(dot);
        for (int64_t i = t; i < m; i += 64) x[i] -= dot * y[i];
        __syncthreads();
      }
      double nn = 0.0;
      for (int64_t i = t; i < m; i += 64) nn += x[i] * x[i];
      nn = wave_sum(nn);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int64_t i = t; i < m; i += 64) x[i] *= inv;
      __syncthreads();
    }
    if (use_lds)
      for (int64_t i = t; i < m; i += 64) xg[i] = x[i];
    __syncthreads();
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
  // column in registers (row lane + 64 u); the next AH reflectors in flight
  // (a ring of register sets, rotated by the unrolled loop)
  constexpr int AH = VR <= 8 ? 4 : (VR <= 16 ? 2 : 1);
  double xr[VR], vq[AH][VR], bq[AH];
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t i = lane + 64 * u;
    xr[u] = i < m ? x[i] : 0.0;
  }
  auto fetch = [&](int64_t jj, double (&vv)[VR], double& bb) {
    bb = jj >= 0 ? beta[jj] : 0.0;
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t i = lane + 64 * u;
      vv[u] = (jj >= 0 && i > jj && i < m) ? Vh[jj * m + i] : 0.0;
    }
  };
  auto apply = [&](const double (&vv)[VR], double bb) {
    if (bb == 0.0) return;
    double dot = 0.0;
#pragma unroll
    for (int u = 0; u < VR; ++u) dot += vv[u] * xr[u];
    dot = wave_sum(dot);
    const double f = bb * dot;
#pragma unroll
    for (int u = 0; u < VR; ++u) xr[u] -= f * vv[u];
  };
  // reflectors j = m - 3 down to 0; slot q holds j = m - 3 - (step mod AH)
#pragma unroll
  for (int q = 0; q < AH; ++q) fetch(m - 3 - q, vq[q], bq[q]);
  for (int64_t j0 = m - 3; j0 >= 0; j0 -= AH) {
#pragma unroll
    for (int q = 0; q < AH; ++q) {
      const int64_t j = j0 - q;
      if (j >= 0) apply(vq[q], bq[q]);
      fetch(j - AH, vq[q], bq[q]);
    }
  }
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t i = lane + 64 * u;
    if (i < m) Uk[i * ldu + c] = xr[u];
  }
}

// The same back-transformation for large m with the rows of a column spread
// over a workgroup of 256 threads (row t + 256 u in lane t, u < VR) and CPW
// columns per workgroup sharing each reflector's loads: short per-lane rows
// leave registers for AH reflectors in flight (one reflector's loads cost a
// memory latency, the per-reflector work a few hundred cycles).  The dot
// products: wave sums, then the four wavefronts' partials through LDS (two
// alternating slots, one barrier per reflector).
template <int VR, int CPW>
__global__ __launch_bounds__(256) void tridiag_back_wg_kernel(
    const double* __restrict__ Vh, const double* __restrict__ beta, int64_t m, int k,
    const double* __restrict__ X, double* __restrict__ Uk, int64_t ldu,
    const double* __restrict__ theta, double* __restrict__ ritz) {
  constexpr int AH = 4;
  __shared__ double part[2][4][CPW];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int c0 = blockIdx.x * CPW;
  if (ritz && t < CPW && c0 + t < k) ritz[c0 + t] = sqrt(fmax(theta[c0 + t], 0.0));
  double xr[CPW][VR];
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t i = t + 256 * u;
      xr[cc][u] = (c0 + cc < k && i < m) ? X[static_cast<int64_t>(c0 + cc) * m + i] : 0.0;
    }
  double vq[AH][VR], bq[AH];
  auto fetch = [&](int64_t jj, double (&vv)[VR], double& bb) {
    bb = jj >= 0 ? beta[jj] : 0.0;
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t i = t + 256 * u;
      vv[u] = (jj >= 0 && i > jj && i < m) ? Vh[jj * m + i] : 0.0;
    }
  };
  int slot = 0;
  auto apply = [&](const double (&vv)[VR], double bb) {
    double dot[CPW];
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      double d = 0.0;
#pragma unroll
      for (int u = 0; u < VR; ++u) d += vv[u] * xr[cc][u];
      d = wave_sum(d);
      dot[cc] = d;
    }
    if (lane == 0) {
#pragma unroll
      for (int cc = 0; cc < CPW; ++cc) part[slot][wv][cc] = dot[cc];
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      const double f =
          bb * (((part[slot][0][cc] + part[slot][1][cc]) + part[slot][2][cc]) + part[slot][3][cc]);
#pragma unroll
      for (int u = 0; u < VR; ++u) xr[cc][u] -= f * vv[u];
    }
    slot ^= 1;  // the next reflector writes the other slot (no second barrier)
  };
  // reflectors j = m - 3 down to 0; slot q holds j = m - 3 - (step mod AH)
#pragma unroll
  for (int q = 0; q < AH; ++q) fetch(m - 3 - q, vq[q], bq[q]);
  for (int64_t j0 = m - 3; j0 >= 0; j0 -= AH) {
#pragma unroll
    for (int q = 0; q < AH; ++q) {
      const int64_t j = j0 - q;
      if (j >= 0) apply(vq[q], bq[q]);  // (uniform)
      fetch(j - AH, vq[q], bq[q]);
    }
  }
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t i = t + 256 * u;
      if (c0 + cc < k && i < m) Uk[i * ldu + c0 + cc] = xr[cc][u];
    }
}

// ------------------------------------------------- large m (> TRI_SMALL) --
// The same reduction with the trailing block in global memory and the work
// of a step spread over the chip, in three launches per step:
//   tribig_reduce_kernel (grid): p = beta A' v of step j-1 from the row-group
//     partial sums, and partials of v^T p;
//   tribig_step_kernel (one workgroup): finishes step j-1 (w = p - (beta
//     v^T p / 2) v, which with v becomes the pending update) and forms
//     reflector j from column j with that update applied (row j of the
//     symmetric square, read contiguously);
//   tribig_update_kernel (grid): applies the pending update to the trailing
//     square (both triangles, a thread per column, 64-row groups) and
//     writes the partial sums of A' v_j per row group, added in group order
//     by the next step kernel.
constexpr int TBG_ROWS = 64;
constexpr int TBG_COLS = 256;

// Finish of step j-1 over the chip: p_l = beta_{j-1} (sum over the row
// groups, in group order, of the partials of A' v_{j-1}) for l >= j, and
// the workgroup's partial of v_{j-1}^T p (its 256 entries in order).
__global__ __launch_bounds__(256) void tribig_reduce_kernel(int64_t m, int64_t j,
                                                            const double* __restrict__ v,
                                                            const double* __restrict__ part,
                                                            int G, const double* __restrict__ beta,
                                                            double* __restrict__ pbuf,
                                                            double* __restrict__ dotpart) {
  __shared__ double red[4];
  const int t = threadIdx.x;
  const int64_t l = j + static_cast<int64_t>(blockIdx.x) * 256 + t;
  double vp = 0.0;
  if (l < m) {
    double sum = 0.0;
    int g = 0;
    for (; g + 8 <= G; g += 8) {
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = part[static_cast<int64_t>(g + u) * m + l];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += q[u];
    }
    for (; g < G; ++g) sum += part[static_cast<int64_t>(g) * m + l];
    const double pl = beta[j - 1] * sum;
    pbuf[l] = pl;
    vp = v[l] * pl;
  }
  // fixed order: lanes by butterfly, then the four wavefronts in order
  for (int o = 32; o > 0; o >>= 1) vp += __shfl_xor(vp, o);
  if ((t & 63) == 0) red[t >> 6] = vp;
  __syncthreads();
  if (t == 0) dotpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(1024) void tribig_step_kernel(
    double* __restrict__ A, int64_t m, int64_t j, double* __restrict__ v,
    double* __restrict__ vp, double* __restrict__ wp, const double* __restrict__ pbuf,
    const double* __restrict__ dotpart, int ND, double* __restrict__ Vh,
    double* __restrict__ beta, double* __restrict__ dg, double* __restrict__ eo) {
  __shared__ double red[TRI_THREADS / 64];
  __shared__ double s_diag;
  const int t = threadIdx.x;
  if (j >= 1) {
    // finish step j-1 over rows / columns j .. m-1: p and the partials of
    // v^T p came from the reduction kernel (added here in order)
    const double bprev = beta[j - 1];
    double vtp = 0.0;
    for (int b = 0; b < ND; ++b) vtp += dotpart[b];
    const double K = 0.5 * bprev * vtp;
    for (int64_t l = j + t; l < m; l += TRI_THREADS) {
      const double vl = v[l];
      vp[l] = vl;
      wp[l] = pbuf[l] - K * vl;
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

// ------------------------------ one cooperative grid for the large-m steps --
// The same reduction with every step inside one launch of G co-resident
// workgroups (a cooperative launch, which fails rather than start fewer):
// row i of the matrix lives in the registers of workgroup i mod G, thread t
// holding columns t + 1024 e.  Step j:
//   (1) every workgroup forms reflector j from row j (published by its
//       owner) with the pending update of step j-1 applied: the same
//       operations in the same order everywhere, so every copy agrees;
//   (2) each workgroup applies the pending update to its rows i > j and
//       forms p_i = beta (M' v_j)_i; the owner of row j+1 publishes that row;
//   (3) grid barrier;
//   (4) every workgroup reads p and forms K = beta v^T p / 2 and w = p - K v,
//       the pending update of step j+1.
// One grid barrier per step.  p and the published row alternate between two
// buffers by step parity: no workgroup gets more than a phase ahead of
// another.  Everything one workgroup hands to another (p, the row, the
// barrier flags) goes through device-scope relaxed atomic loads and stores,
// which are coherent across the XCDs' L2 caches by themselves, so the
// barrier needs no cache write-back or invalidation: each thread waits for
// its own stores to complete before its workgroup posts its flag.  Each
// workgroup has a flag of its own (no contended atomic); a wait gives up
// after TCO_SPIN polls (a co-resident grid never needs that many), sets
// `stall` and stops waiting at every later barrier, so the launch always
// ends.
constexpr int TCO_THREADS = 1024;
constexpr int TCO_E = 3;     // columns per thread: m <= 3072
constexpr int TCO_RL = 10;   // rows per workgroup: m <= 10 G
constexpr unsigned TCO_SPIN = 1u << 22;

struct TcoSync {
  int stall;
  unsigned go;         // the last step workgroup 0 released
  unsigned flag[256];  // per workgroup: the last step it finished (G <= 256)
};

__device__ __forceinline__ void tco_put(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double tco_get(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier of step `step` (>= 1): every thread's stores complete (vmcnt
// counts stores on this target); then workgroup 0 polls the flags of the
// others (a thread per flag) and posts `go`, while each other workgroup
// posts its own flag and polls `go` with one thread.  Flags only grow, so
// nothing is reset, and no two workgroups write one address.  (Every
// workgroup polling every flag took 26.2 ms for the m = 2304 reduction,
// this gather-and-release form 23.5 ms: a poll round of G flags per
// workgroup is G^2 loads at the device coherence point.)
__device__ __forceinline__ void tco_grid_sync(TcoSync* sy, unsigned step) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  unsigned* go = &sy->go;
  if (blockIdx.x == 0) {
    if (threadIdx.x > 0 && threadIdx.x < gridDim.x) {
      unsigned polls = 0;
      while (__hip_atomic_load(&sy->flag[threadIdx.x], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) < step) {
        if (__hip_atomic_load(&sy->stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++polls > TCO_SPIN) {
          __hip_atomic_store(&sy->stall, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(go, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    __hip_atomic_store(&sy->flag[blockIdx.x], step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned polls = 0;
    while (__hip_atomic_load(go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < step) {
      if (__hip_atomic_load(&sy->stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++polls > TCO_SPIN) {
        __hip_atomic_store(&sy->stall, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__global__ void tco_init_kernel(TcoSync* sy) {
  if (threadIdx.x == 0) {
    sy->stall = 0;
    sy->go = 0u;
  }
  sy->flag[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(TCO_THREADS) void tri_coop_kernel(
    const double* __restrict__ A, int64_t m, double* __restrict__ Vh, double* __restrict__ beta,
    double* __restrict__ dg, double* __restrict__ eo, double* pbuf, double* rbuf,
    TcoSync* sy) {
  __shared__ double spv[TCO_E * TCO_THREADS], spw[TCO_E * TCO_THREADS];
  __shared__ double redA[TCO_THREADS / 64], redB[TCO_THREADS / 64];
  __shared__ double prow[TCO_RL * TCO_THREADS];  // the rows' per-thread partials of M' v
  __shared__ double bc[2];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int G = static_cast<int>(gridDim.x), g = static_cast<int>(blockIdx.x);
  // own rows g + r G, r < TCO_RL; columns t + 1024 e
  double a[TCO_RL][TCO_E];
#pragma unroll
  for (int r = 0; r < TCO_RL; ++r) {
    const int64_t i = g + static_cast<int64_t>(r) * G;
#pragma unroll
    for (int e = 0; e < TCO_E; ++e) {
      const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
      a[r][e] = (i < m && l < m) ? A[i * m + l] : 0.0;
    }
  }
  // pending update (v, w) of the previous step: own columns in registers,
  // the whole vectors in LDS (rows read them by index); the published row
  double pv[TCO_E], pw[TCO_E], xr[TCO_E];
#pragma unroll
  for (int e = 0; e < TCO_E; ++e) {
    const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
    pv[e] = 0.0;
    pw[e] = 0.0;
    spv[l] = 0.0;
    spw[l] = 0.0;
    xr[e] = l < m ? A[l] : 0.0;  // row 0
  }
  __syncthreads();
  for (int64_t j = 0; j + 2 < m; ++j) {
    const int par = static_cast<int>(j & 1);
    const int64_t j1 = j + 1;
    // (1) reflector j from x = row j with the pending update, columns >= j
    const double pvj = spv[j], pwj = spw[j];
    double x[TCO_E];
    double nrm2 = 0.0;
#pragma unroll
    for (int e = 0; e < TCO_E; ++e) {
      const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
      x[e] = 0.0;
      if (l >= j && l < m) {
        x[e] = xr[e] - (pvj * pw[e] + pwj * pv[e]);
        if (l == j) bc[0] = x[e];
        if (l == j1) bc[1] = x[e];
        if (l > j) nrm2 += x[e] * x[e];
      }
    }
    nrm2 = wg_sum_1024(nrm2, redA);  // (its barrier also publishes bc)
    const double djj = bc[0], x0 = bc[1];
    const double nx = sqrt(nrm2);
    double b = 0.0, alpha = x0, v0 = x0;
    if (nx > 0.0 && nrm2 - x0 * x0 > 0.0) {
      alpha = x0 >= 0.0 ? -nx : nx;
      v0 = x0 - alpha;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
      b = vtv > 0.0 ? 2.0 / vtv : 0.0;
    }
    double vv[TCO_E];
#pragma unroll
    for (int e = 0; e < TCO_E; ++e) {
      const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
      vv[e] = (l == j1) ? v0 : ((l > j1 && l < m) ? x[e] : 0.0);
      if (g == 0 && l > j && l < m) Vh[j * m + l] = vv[e];
    }
    if (g == 0 && t == 0) {
      dg[j] = djj;
      eo[j] = alpha;
      beta[j] = b;
    }
    // (2) own rows i > j: the pending update, then their partials of M' v
#pragma unroll
    for (int r = 0; r < TCO_RL; ++r) {
      const int64_t i = g + static_cast<int64_t>(r) * G;
      double ps = 0.0;
      if (i > j && i < m) {  // (uniform)
        const double pvi = spv[i], pwi = spw[i];
#pragma unroll
        for (int e = 0; e < TCO_E; ++e) {
          const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
          if (l > j && l < m) {
            a[r][e] -= pvi * pw[e] + pwi * pv[e];
            ps += a[r][e] * vv[e];
          }
        }
        prow[r * TCO_THREADS + t] = ps;
        if (i == j1) {  // the owner publishes row j+1
#pragma unroll
          for (int e = 0; e < TCO_E; ++e) {
            const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
            if (l < m) tco_put(rbuf + par * m + l, a[r][e]);
          }
        }
      }
    }
    __syncthreads();
    // wavefront r sums row r's 1024 partials: lane l adds entries l, l + 64,
    // ... in order, then the wave sum (one reduction per row instead of a
    // wave sum per row in every wavefront, which took most of this phase)
    if (wv < TCO_RL) {
      const int64_t i = g + static_cast<int64_t>(wv) * G;
      if (i > j && i < m) {  // (uniform per wavefront)
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < TCO_THREADS / 64; ++q) sum += prow[wv * TCO_THREADS + lane + 64 * q];
        sum = wave_sum(sum);
        if (lane == 0) tco_put(pbuf + par * m + i, b * sum);
      }
    }
    // (3)
    tco_grid_sync(sy, static_cast<unsigned>(j + 1));
    // (4) p on own columns, K, the next pending update, the next row
    double pl[TCO_E];
    double vp = 0.0;
#pragma unroll
    for (int e = 0; e < TCO_E; ++e) {
      const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
      pl[e] = (l > j && l < m) ? tco_get(pbuf + par * m + l) : 0.0;
      vp += vv[e] * pl[e];
      xr[e] = (l > j && l < m) ? tco_get(rbuf + par * m + l) : 0.0;
    }
    vp = wg_sum_1024(vp, redB);
    const double K = 0.5 * b * vp;
#pragma unroll
    for (int e = 0; e < TCO_E; ++e) {
      const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
      pv[e] = vv[e];
      pw[e] = pl[e] - K * vv[e];
      spv[l] = pv[e];
      spw[l] = pw[e];
    }
    __syncthreads();
  }
  // last 2 x 2 block: rows m-2 and m-1 (updated through step m-4) with the
  // pending update of step m-3
#pragma unroll
  for (int r = 0; r < TCO_RL; ++r) {
    const int64_t i = g + static_cast<int64_t>(r) * G;
    if (i >= m - 2 && i < m) {
#pragma unroll
      for (int e = 0; e < TCO_E; ++e) {
        const int64_t l = t + static_cast<int64_t>(e) * TCO_THREADS;
        if (l == i) dg[i] = a[r][e] - 2.0 * spv[i] * spw[i];
        if (i == m - 2 && l == m - 1)
          eo[i] = a[r][e] - (spv[i] * spw[l] + spw[i] * spv[l]);
      }
    }
  }
}

// Reorthogonalization of the inverse-iteration vectors (columns of X,
// column-major, ld m).  Inverse iteration only orthogonalizes within groups
// of eigenvalues closer than 1e-10 ||T||; a pair separated by a gap g keeps
// an overlap of ~ eps ||T|| / g.  One CholeskyQR pass over all k columns in
// eigenvalue order (X <- X R^-1, R^T R = X^T X), i.e. Gram-Schmidt with the
// larger eigenvalue's vector kept, removes those overlaps; for well
// separated pairs the corrections are rounding-sized.
// G = X^T X: a 16 x 16 tile per workgroup, rows in 64-row chunks through
// LDS; G_ij and G_ji get the same products in the same order (symmetric).
__global__ __launch_bounds__(256) void xgram_kernel(const double* __restrict__ X, int64_t m,
                                                    int k, double* __restrict__ G) {
  __shared__ double xi[64][17], xj[64][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  double acc = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int c = e >> 6, r = e & 63;
      const int64_t row = r0 + r;
      xi[r][c] = (i0 + c < k && row < m) ? X[static_cast<int64_t>(i0 + c) * m + row] : 0.0;
      xj[r][c] = (j0 + c < k && row < m) ? X[static_cast<int64_t>(j0 + c) * m + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 16
    for (int r = 0; r < 64; ++r) acc += xi[r][ty] * xj[r][tx];
    __syncthreads();
  }
  const int i = i0 + ty, j = j0 + tx;
  if (i < k && j < k) G[static_cast<int64_t>(i) * k + j] = acc;
}

// Xn[:, c] = sum_{l <= c} X[:, l] Rinv[l][c] (a thread per entry, rows
// consecutive across threads).
__global__ __launch_bounds__(256) void xapply_kernel(const double* __restrict__ X, int64_t m,
                                                     int k, const double* __restrict__ Rinv,
                                                     double* __restrict__ Xn) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= m * k) return;
  const int c = static_cast<int>(idx / m);
  const int64_t i = idx - static_cast<int64_t>(c) * m;
  double sum = 0.0;
  for (int l = 0; l <= c; ++l) sum += X[static_cast<int64_t>(l) * m + i] * Rinv[static_cast<int64_t>(l) * k + c];
  Xn[idx] = sum;
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
  // pivots (k m ints) + (large m) v, vp, wp and the row-group partials +
  // (small m) the panel's V and W
  // + the reorthogonalization: the new X, G, R, R^-1, the Cholesky's work
  // and a status word it may write
  const int64_t groups = cdiv(m, TBG_ROWS);
  const int64_t kk = static_cast<int64_t>(k) * k;
  return 2 * m * m + 3 * m + static_cast<int64_t>(k) * m +
         std::max<int64_t>(static_cast<int64_t>(k) * 5 * m, static_cast<int64_t>(k) * 1024) +
         (static_cast<int64_t>(k) * m + 1) / 2 + 3 * m + groups * m + 2 * TRI_NB * m + 64 +
         static_cast<int64_t>(k) * m + 3 * kk + chol_work_doubles(k) + 8 +
         m + cdiv(m, 256) + 64 +  // p and the v^T p partials of the large-m steps
         4 * m + 136;             // the cooperative grid's p, row and barrier flags
}

namespace {
// Workgroups of the cooperative reduction on the current device (one per
// CU), 0 if the device cannot take it.
int tco_grid(hipStream_t s) {
  static int cached[64] = {0};  // 0: not asked yet, -1: none, else G
  int dev = 0;
  if (hipStreamGetDevice(s, &dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int coop = 0, cus = 0, nb = 0;
    const bool ok =
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(tri_coop_kernel), TCO_THREADS, 0) == hipSuccess;
    cached[dev] = (ok && coop && cus > 0 && nb >= 1) ? cus : -1;
  }
  return cached[dev] > 0 ? cached[dev] : 0;
}

__global__ void tco_report_kernel(const TcoSync* sy, Ctrl* ctrl) {
  if (sy->stall) atomicOr(&ctrl->flags, CTRL_STALL);
}
}  // namespace

void launch_tridiag_topk(const double* M, int64_t m, int64_t ldm, int k, double* scratch,
                         double* theta, double* Uk, int64_t ldu, double* ritz, Ctrl* ctrl,
                         hipStream_t s) {
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
  double* Vg = part + cdiv(m, TBG_ROWS) * m;
  double* Wg = Vg + TRI_NB * m;
  const int64_t kk = static_cast<int64_t>(k) * k;
  double* pbuf = Wg + TRI_NB * m + 64;
  double* dotpart = pbuf + m;
  double* Xn = dotpart + cdiv(m, 256) + 64;
  double* Gx = Xn + static_cast<int64_t>(k) * m;
  double* Rx = Gx + kk;
  double* Rix = Rx + kk;
  double* cwork = Rix + kk;
  Ctrl* cdummy = reinterpret_cast<Ctrl*>(cwork + chol_work_doubles(k));
  double* cpb = cwork + chol_work_doubles(k) + 8;  // cooperative grid: p (2 m),
  double* crb = cpb + 2 * m;                       // the published row (2 m),
  TcoSync* csy = reinterpret_cast<TcoSync*>(crb + 2 * m);  // the barrier
  static bool attr = false;
  if (!attr) {
    for (const void* f : {reinterpret_cast<const void*>(tridiag_reduce_kernel),
                          reinterpret_cast<const void*>(tridiag_bisect_kernel),
                          reinterpret_cast<const void*>(tridiag_invit_kernel),
                          reinterpret_cast<const void*>(tri_panel_kernel)})
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, TRI_LDS_BYTES);
    attr = true;
  }
  sym_copy_kernel<<<static_cast<unsigned>(cdiv(m * m, 256)), 256, 0, s>>>(M, m, ldm, A);
  launch_fill_f64(Vh, m * m, 0.0, s);
  if (m <= TRI_SMALL) {
    // order of the largest trailing block that fits in LDS beside v, p, w
    const int64_t room = TRI_LDS_BYTES / static_cast<int64_t>(sizeof(double)) - 3 * m;
    int64_t sb = static_cast<int64_t>(std::sqrt(static_cast<double>(room)));
    while (sb * sb > room) --sb;
    if (sb > m) sb = m;
    // blocked panels until the trailing block fits (sb >= 3 keeps every
    // panel step a full reflector step, j + 2 < m)
    int64_t j = 0;
    while (m - j > sb) {
      const int nst = static_cast<int>(std::min<int64_t>(TRI_NB, m - sb - j));
      const int64_t mr = m - j;
      const int64_t base = 2 * m + 2 * TRI_NB + 2 * TRI_NB * mr;  // doubles
      // rows of the panel-start block staged in the LDS left over
      const int64_t free_d = TRI_LDS_BYTES / static_cast<int64_t>(sizeof(double)) - base;
      const int R = static_cast<int>(std::max<int64_t>(0, std::min<int64_t>(mr, free_d / mr)));
      const size_t lds = static_cast<size_t>(base + static_cast<int64_t>(R) * mr) * sizeof(double);
      tri_panel_kernel<<<1, TRI_THREADS, lds, s>>>(A, m, j, nst, R, Vg, Wg, Vh, beta, dg, eo);
      const int64_t jn = j + nst;
      const unsigned g = static_cast<unsigned>(cdiv(m - jn, TRI_SY));
      tri_syr2k_kernel<<<dim3(g, g), 256, 0, s>>>(A, m, jn, Vg, Wg, nst);
      j = jn;
    }
    tridiag_reduce_kernel<<<1, TRI_THREADS, (3 * m + (m - j) * (m - j)) * sizeof(double), s>>>(
        A, m, j, Vh, beta, dg, eo);
  } else if (const int Gc = std::min(tco_grid(s), 256);
             Gc > 0 && m <= static_cast<int64_t>(TCO_E) * TCO_THREADS &&
             m <= static_cast<int64_t>(TCO_RL) * Gc &&
             [&] {
               tco_init_kernel<<<1, 256, 0, s>>>(csy);
               const double* a0 = A;
               void* args[] = {&a0, &m, &Vh, &beta, &dg, &eo, &cpb, &crb, &csy};
               if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(tri_coop_kernel),
                                              dim3(Gc), dim3(TCO_THREADS), args, 0,
                                              s) != hipSuccess) {
                 (void)hipGetLastError();  // not taken: the launch-per-step path below
                 return false;
               }
               if (ctrl) tco_report_kernel<<<1, 1, 0, s>>>(csy, ctrl);
               return true;
             }()) {
    // reduced by the cooperative grid
  } else {
    launch_fill_f64(v, 3 * m, 0.0, s);  // v, vp, wp
    int G = 0, ND = 0;
    // reduce (grid) -> step (one workgroup) -> update (grid) per step
    auto finish = [&](int64_t j) {
      if (j >= 1) {
        ND = static_cast<int>(cdiv(m - j, 256));
        tribig_reduce_kernel<<<static_cast<unsigned>(ND), 256, 0, s>>>(m, j, v, part, G, beta,
                                                                       pbuf, dotpart);
      }
      tribig_step_kernel<<<1, TRI_THREADS, 0, s>>>(A, m, j, v, vp, wp, pbuf, dotpart, ND, Vh,
                                                   beta, dg, eo);
    };
    for (int64_t j = 0; j + 2 < m; ++j) {
      finish(j);
      const int64_t sj = m - j - 1;
      G = static_cast<int>(cdiv(sj, TBG_ROWS));
      tribig_update_kernel<<<dim3(static_cast<unsigned>(cdiv(sj, TBG_COLS)),
                                  static_cast<unsigned>(G)),
                             TBG_COLS, 0, s>>>(A, m, j, v, vp, wp, part);
    }
    finish(m - 2);
  }
  // eigenvalues: a workgroup each; eigenvectors: a workgroup per cluster,
  // its factors in LDS when they fit beside the tridiagonal
  tridiag_bisect_kernel<<<static_cast<unsigned>(k), BS_THREADS, 2 * m * sizeof(double), s>>>(
      dg, eo, m, k, theta);
  const size_t inv_lds = (7 * m + (m + 1) / 2) * sizeof(double);
  const int use_lds = inv_lds <= static_cast<size_t>(TRI_LDS_BYTES) ? 1 : 0;
  tridiag_invit_kernel<<<static_cast<unsigned>(k), 64, use_lds ? inv_lds : 2 * m * sizeof(double),
                         s>>>(dg, eo, m, k, theta, X, sol, piv, use_lds);
  // Gram-Schmidt over all k vectors in eigenvalue order (CholeskyQR; the
  // Cholesky's failure reports go to a status word nobody reads: a Gram of
  // unit vectors this close to I has no failing pivot)
  const unsigned gt = static_cast<unsigned>(cdiv(k, 16));
  xgram_kernel<<<dim3(gt, gt), 256, 0, s>>>(X, m, k, Gx);
  launch_ctrl_init(cdummy, 0, s);
  launch_chol(k, Gx, nullptr, CHOL_REPEAT, 1 << 30, 0.0, 0.0, Rx, Rix, cwork, cdummy, s);
  xapply_kernel<<<static_cast<unsigned>(cdiv(m * k, 256)), 256, 0, s>>>(X, m, k, Rix, Xn);
  X = Xn;
  const unsigned gb = static_cast<unsigned>(cdiv(k, 4));
  if (m <= 256)
    tridiag_back_kernel<4><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else if (m <= 512)
    tridiag_back_kernel<8><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else if (m <= 1024)  // a workgroup per 4 columns, rows spread over it
    tridiag_back_wg_kernel<4, 4><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else if (m <= 2048)
    tridiag_back_wg_kernel<8, 4><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
  else  // m <= kTridiagMax = 256 * 10
    tridiag_back_wg_kernel<10, 4><<<gb, 256, 0, s>>>(Vh, beta, m, k, X, Uk, ldu, theta, ritz);
}

}  // namespace bk
