// Small FP64 kernels of the orthonormalization (Algorithm 2, step 3) and
// the output step: fills and copies, the one-workgroup Cholesky +
// triangular inverse behind CholeskyQR, and column sign normalisation.
#include "kernels.hpp"

namespace bk {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T* p, int64_t n, T v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void copy2d_kernel(const TS* src, int64_t lds,
                                                     TD* dst, int64_t ldd,
                                                     int64_t rows, int64_t cols) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols, c = i - r * cols;
  dst[r * ldd + c] = static_cast<TD>(src[r * lds + c]);
}

__global__ __launch_bounds__(256) void axpy_kernel(const double* x, double* y,
                                                   int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) y[i] += x[i];
}

__global__ void ctrl_init_kernel(Ctrl* c, int32_t q) {
  if (threadIdx.x == 0) {
    c->flags = 0;
    c->q_eff = q;
    c->csr_bad = 0;
    c->pad0 = 0;
    c->offmax = 0ull;
    c->pad1 = 0ull;
  }
}

__global__ void ctrl_reset_off_kernel(Ctrl* c) {
  if (threadIdx.x == 0) c->offmax = 0ull;
}

// Fixed-order block reduction (sum) over blockDim.x (a power of two) threads.
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = static_cast<int>(blockDim.x) / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Upper Cholesky factor S of (G + shift I) (G = S^T S), right-looking, in S
// (LDS or global, k x k).  Returns false when a pivot is not positive and
// finite; *minpiv receives the smallest diagonal of S.
__device__ bool chol_factor(int k, const double* G, double shift, double* S,
                            double* minpiv, int* fail) {
  const int t = threadIdx.x;
  const int NT = static_cast<int>(blockDim.x);
  // 2-D thread layout: 16 columns x NT / 16 rows (no integer division in loops)
  const int tx = t & 15, ty = t >> 4, NY = NT >> 4;
  for (int r = ty; r < k; r += NY)
    for (int c = tx; c < k; c += 16)
      S[r * k + c] = (c >= r) ? G[r * k + c] + (r == c ? shift : 0.0) : 0.0;
  if (t == 0) {
    *fail = 0;
    *minpiv = INFINITY;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double piv = S[j * k + j];
      if (!(piv > 0.0) || !isfinite(piv)) {
        *fail = 1;
      } else {
        const double dj = sqrt(piv);
        S[j * k + j] = dj;
        if (dj < *minpiv) *minpiv = dj;
      }
    }
    __syncthreads();
    if (*fail) return false;
    const double inv = 1.0 / S[j * k + j];
    for (int c = j + 1 + t; c < k; c += NT) S[j * k + c] *= inv;
    __syncthreads();
    for (int rr = j + 1 + ty; rr < k; rr += NY) {
      const double srj = S[j * k + rr];
      for (int cc = rr + tx; cc < k; cc += 16) S[rr * k + cc] -= srj * S[j * k + cc];
    }
    __syncthreads();
  }
  return true;
}

// Relative size below which a pivot of the unshifted factor of A Pi counts
// as zero: tau, but at least sqrt(shift_coef), the level of the shift that
// the first CholeskyQR pass adds anyway.  The Gram of an exactly rank
// deficient block has pivots of rounding size (~ n u tr) of either sign, so
// a smaller threshold would decide by the summation order.
__device__ __forceinline__ double rank_floor(double tau, double shift_coef) {
  return fmax(tau, sqrt(shift_coef));
}

// Modes:
//  CHOL_FIRST_BLOCK0  first pass on A Pi: a Cholesky pivot of the unshifted
//                     factor <= rank_floor ||A Pi||_F flags CTRL_RANK; then
//                     the shifted factor (shift = shift_coef * trace(G)).
//  CHOL_FIRST         first pass on a projected block i >= 1: when
//                     ||B||_F <= tau * ||B_pre||_F (traces of G and Gpre)
//                     the Krylov space is invariant: q_eff = min(q_eff,
//                     i - 1) and the block becomes zero; else shifted factor.
//  CHOL_REPEAT        plain factor of an almost orthonormal block.
// On any failure R and Rinv are zero, so the applied block is zero.
__global__ __launch_bounds__(256) void chol_kernel(int k, const double* G,
                                                   const double* Gpre, int mode,
                                                   int block, double tau,
                                                   double shift_coef, double* R,
                                                   double* Rinv, double* work,
                                                   Ctrl* ctrl, int use_lds) {
  extern __shared__ double dyn[];
  __shared__ double red[256];
  __shared__ double minpiv;
  __shared__ int fail;
  __shared__ int decision;  // 0 go on, 1 zero block
  const int t = threadIdx.x;
  const int NT = static_cast<int>(blockDim.x);
  double* S = use_lds ? dyn : work;
  double* Ri = use_lds ? dyn + k * k : Rinv;

  double trp = 0.0, prp = 0.0;
  int bad = 0;
  for (int i = t; i < k * k; i += NT)
    if (!isfinite(G[i])) bad = 1;
  for (int i = t; i < k; i += NT) {
    trp += G[i * k + i];
    if (mode == CHOL_FIRST) prp += Gpre[i * k + i];
  }
  const int anybad = __syncthreads_or(bad);
  const double tr = block_sum(trp, red);
  const double pre = (mode == CHOL_FIRST) ? block_sum(prp, red) : 0.0;
  if (t == 0) {
    decision = 0;
    if (anybad) {
      atomicOr(&ctrl->flags, CTRL_NONFINITE);
      decision = 1;
    } else if (mode == CHOL_FIRST) {
      if (!(sqrt(tr) > tau * sqrt(pre))) {
        atomicMin(&ctrl->q_eff, block - 1);
        decision = 1;
      }
    } else if (!(tr > 0.0)) {
      if (mode == CHOL_FIRST_BLOCK0) atomicOr(&ctrl->flags, CTRL_RANK);
      decision = 1;
    }
  }
  __syncthreads();
  if (!decision && mode == CHOL_FIRST_BLOCK0) {
    const bool ok = chol_factor(k, G, 0.0, S, &minpiv, &fail);
    if (t == 0 && (!ok || !(minpiv > rank_floor(tau, shift_coef) * sqrt(tr)))) {
      atomicOr(&ctrl->flags, CTRL_RANK);
      decision = 1;
    }
    __syncthreads();
  }
  if (!decision) {
    const double shift = (mode == CHOL_REPEAT) ? 0.0 : shift_coef * tr;
    const bool ok = chol_factor(k, G, shift, S, &minpiv, &fail);
    if (t == 0 && !ok) {
      if (block == 0) atomicOr(&ctrl->flags, CTRL_RANK);
      else atomicMin(&ctrl->q_eff, block - 1);
      decision = 1;
    }
    __syncthreads();
  }
  if (decision) {
    for (int i = t; i < k * k; i += NT) {
      R[i] = 0.0;
      Rinv[i] = 0.0;
    }
    return;
  }
  // Rinv = S^-1 (upper), one column per thread by back substitution
  // (no barriers): Rinv[i][j] = -(sum_{l=i+1..j} S[i][l] Rinv[l][j]) / S[i][i].
  for (int j = t; j < k; j += NT) {
    for (int i = j + 1; i < k; ++i) Ri[i * k + j] = 0.0;
    Ri[j * k + j] = 1.0 / S[j * k + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += S[i * k + l] * Ri[l * k + j];
      Ri[i * k + j] = -s / S[i * k + i];
    }
  }
  __syncthreads();
  for (int i = t; i < k * k; i += NT) {
    R[i] = S[i];
    if (use_lds) Rinv[i] = Ri[i];
  }
}

__device__ __forceinline__ double lane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// LDS written by lanes of one wavefront becomes visible to its other lanes
// (LDS operations of a wavefront complete in order; this keeps the compiler
// from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Upper Cholesky factor of (G + shift I) in registers of one wavefront:
// lane c holds column c (a[r] = S[r][c], rows r <= c meaningful), the k x k
// problem padded to K with the identity.  Right-looking: every lane posts
// its entry of row j to rb (2 x 64 doubles of LDS), reads the pivot and the
// row back, forms 1 / sqrt(pivot) itself and applies the rank-1 update with
// one FMA per entry.  rinv[j] = 1 / S[j][j].  Returns false on a
// non-positive or non-finite pivot.
template <int K>
__device__ bool chol_regs(int k, const double (&g)[K], double shift, double (&a)[K],
                          double (&rinv)[K], double& minpiv, double* rb) {
  const int c = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < K; ++r)
    a[r] = (c < k) ? ((r <= c) ? g[r] + (r == c ? shift : 0.0) : 0.0) : (r == c ? 1.0 : 0.0);
  minpiv = INFINITY;
  bool ok = true;
  // two row buffers, alternating: row j + 1 is posted as soon as its own
  // entry of step j's update is done, and the rest of the update overlaps
  // the post
  rb[c] = a[0];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < K; ++j) {  // no early exit: the loop stays unrolled
    const double* b = rb + (j & 1) * 64;
    // the whole row j (entries j .. K-1) requested at once, before the
    // pivot's dependent chain: one LDS round trip per step
    double bv[K];
#pragma unroll
    for (int r = j; r < K; ++r) bv[r] = b[r];
    double d = bv[j];
    if (!(d > 0x1p-1000) || !isfinite(d)) {  // (a pivot below 2^-1000 is a breakdown)
      ok = false;
      d = 1.0;
    }
    // 1/sqrt(d): hardware estimate and two Newton steps (quadratic), then
    // sqrt(d) = d / sqrt(d) with one Newton correction; short dependency
    // chains for the serial loop
    double inv = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    inv = fma(inv, fma(-hd * inv, inv, 0.5), inv);
    inv = fma(inv, fma(-hd * inv, inv, 0.5), inv);
    const double s0 = d * inv;
    const double rd = fma(fma(-s0, s0, d), 0.5 * inv, s0);
    if (j < k) minpiv = fmin(minpiv, rd);
    rinv[j] = inv;
    a[j] = (c == j) ? rd : a[j] * inv;  // row j of the factor (lanes c >= j)
    // S[j][r] S[j][c] = b[r] (a[j] / sqrt(d)): one FMA per entry
    const double tj = a[j] * inv;
    if (j + 1 < K) {
      a[j + 1] -= bv[j + 1] * tj;
      rb[((j + 1) & 1) * 64 + c] = a[j + 1];  // (every lane: no branch)
      wave_lds_sync();
    }
#pragma unroll
    for (int r = j + 2; r < K; ++r) a[r] -= bv[r] * tj;
  }
  return ok;
}

// The mode logic of the CholeskyQR factor for k <= 64 in one wavefront
// (lane c holds g = column c of G; tr = trace G, pre = trace Gpre): the
// breakdown and rank tests, then the factor in a / rinv.  Returns true when
// the block is dropped (zero factor); ctrl is updated when `report`.
template <int K>
__device__ bool chol_wave_factor(int k, const double (&g)[K], int bad, double tr, double pre,
                                 int mode, int block, double tau, double shift_coef,
                                 bool report, Ctrl* ctrl, double (&a)[K], double (&rinv)[K],
                                 double* rb) {
  const int c = threadIdx.x & 63;
  report = report && c == 0;
  bool zero = false;
  if (__any(bad)) {
    if (report) atomicOr(&ctrl->flags, CTRL_NONFINITE);
    zero = true;
  } else if (mode == CHOL_FIRST) {
    if (!(sqrt(tr) > tau * sqrt(pre))) {
      if (report) atomicMin(&ctrl->q_eff, block - 1);
      zero = true;
    }
  } else if (!(tr > 0.0)) {
    if (mode == CHOL_FIRST_BLOCK0 && report) atomicOr(&ctrl->flags, CTRL_RANK);
    zero = true;
  }
  double minpiv = 0.0;
  if (!zero && mode == CHOL_FIRST_BLOCK0) {
    const bool ok = chol_regs<K>(k, g, 0.0, a, rinv, minpiv, rb);
    if (!ok || !(minpiv > rank_floor(tau, shift_coef) * sqrt(tr))) {
      if (report) atomicOr(&ctrl->flags, CTRL_RANK);
      zero = true;
    }
  }
  if (!zero) {
    const double shift = (mode == CHOL_REPEAT) ? 0.0 : shift_coef * tr;
    if (!chol_regs<K>(k, g, shift, a, rinv, minpiv, rb)) {
      if (report) {
        if (block == 0) atomicOr(&ctrl->flags, CTRL_RANK);
        else atomicMin(&ctrl->q_eff, block - 1);
      }
      zero = true;
    }
  }
  return zero;
}

// CholeskyQR factor for k <= 64 in one wavefront (same modes and outputs as
// chol_kernel): R = chol(G [+ shift]) and Rinv = R^-1 by back substitution,
// lane c forming column c of Rinv.
template <int K>
__global__ __launch_bounds__(64) void chol_wave_kernel(int k, const double* __restrict__ G,
                                                       const double* __restrict__ Gpre, int mode,
                                                       int block, double tau,
                                                       double shift_coef, double* __restrict__ R,
                                                       double* __restrict__ Rinv, Ctrl* ctrl) {
  const int c = threadIdx.x;
  double g[K];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const double x = (r < k && c < k) ? G[r * k + c] : 0.0;
    if (!isfinite(x)) bad = 1;
    g[r] = x;
  }
  const double tr = wave_sum_f64(c < k ? G[c * k + c] : 0.0);
  const double pre = (mode == CHOL_FIRST) ? wave_sum_f64(c < k ? Gpre[c * k + c] : 0.0) : 0.0;
  double a[K], rinv[K];
  __shared__ double rb[128];
  const bool zero = chol_wave_factor<K>(k, g, bad, tr, pre, mode, block, tau, shift_coef, true,
                                        ctrl, a, rinv, rb);
  if (zero) {
    for (int i = c; i < k * k; i += 64) {
      R[i] = 0.0;
      Rinv[i] = 0.0;
    }
    return;
  }
  // x = column c of R^-1: x_i = (delta_ic - sum_{l > i} R[i][l] x_l) / R[i][i]
  double x[K];
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    double sum = 0.0;
#pragma unroll
    for (int l = i + 1; l < K; ++l) sum += lane_f64(a[i], l) * x[l];
    x[i] = ((i == c ? 1.0 : 0.0) - sum) * rinv[i];
  }
  if (c < k) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
      if (r < k) {
        R[r * k + c] = (r <= c) ? a[r] : 0.0;
        Rinv[r * k + c] = (r <= c) ? x[r] : 0.0;
      }
    }
  }
}

// --------------------------------------------- chip-wide blocked Cholesky --
// For 64 < k <= kCholBlockedMax: the factor of CholeskyQR as a short chain
// of kernels instead of one workgroup walking a k x k matrix in memory:
//   scan     the working copy S = upper(G) over the chip, with a check of
//            every entry for finiteness and the traces;
//   decide   the mode logic (non-finite, breakdown and rank tests) and the
//            shift on the diagonal (block 0 first unshifted, for its rank
//            test);
//   panel p  one wavefront factors the 32 x 32 diagonal block R_pp in
//            registers and inverts it; the panel row R_p,j = R_pp^-T S_p,j
//            (a thread per column j);
//   update p S_ij -= sum_r R_ri R_rj on the trailing upper triangle, one
//            workgroup per 32 x 32 tile;
//   inverse  R^-1 by doubling: neighbouring diagonal blocks joined level by
//            level, X12 = -X11 R12 X22, a workgroup per 32 x 32 tile;
//   end      failure reports to ctrl, R = upper(S), zeros below the
//            diagonals (everything zero after a failure).
// Every kernel after decide returns at once when the state says the block is
// dropped or a pivot failed.  All sums run in a fixed order.
constexpr int CM = 32;

constexpr int CM_SCAN_WG = 64;  // workgroups of the copy / finiteness scan

struct CholMState {
  int decision;  // 1: dropped before or at the rank test
  int fail;      // 1: a pivot was not positive and finite
  int pad0, pad1;
  double minpiv;
  double tr;                 // trace of G
  double pre;                // trace of Gpre (CHOL_FIRST)
  int bad[CM_SCAN_WG];       // per scan workgroup: a non-finite entry of G
};

// S = upper triangle of G (zeros below), every entry checked for
// finiteness (a flag per workgroup); workgroup 0 also sums the traces.
__global__ __launch_bounds__(256) void cholm_scan_kernel(int k, const double* __restrict__ G,
                                                         const double* __restrict__ Gpre,
                                                         int mode, CholMState* st,
                                                         double* __restrict__ S) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int64_t kk = static_cast<int64_t>(k) * k;
  int bad = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + t; i < kk; i += CM_SCAN_WG * 256) {
    const double g = G[i];
    if (!isfinite(g)) bad = 1;
    const int r = static_cast<int>(i / k), c = static_cast<int>(i - static_cast<int64_t>(r) * k);
    S[i] = (c >= r) ? g : 0.0;
  }
  const int anybad = __syncthreads_or(bad);
  if (t == 0) st->bad[blockIdx.x] = anybad;
  if (blockIdx.x == 0) {
    double trp = 0.0, prp = 0.0;
    for (int i = t; i < k; i += 256) {
      trp += G[static_cast<int64_t>(i) * k + i];
      if (mode == CHOL_FIRST) prp += Gpre[static_cast<int64_t>(i) * k + i];
    }
    const double tr = block_sum(trp, red);
    const double pre = (mode == CHOL_FIRST) ? block_sum(prp, red) : 0.0;
    if (t == 0) {
      st->tr = tr;
      st->pre = pre;
    }
  }
}

// The mode logic (non-finite, breakdown, rank tests) and the shift of the
// first pass on the diagonal of S (block 0 is factored unshifted first,
// for its rank test).
__global__ __launch_bounds__(256) void cholm_decide_kernel(int k, int mode, int block, double tau,
                                                           double shift_coef, Ctrl* ctrl,
                                                           CholMState* st,
                                                           double* __restrict__ S) {
  __shared__ int s_dec;
  __shared__ double s_tr;
  const int t = threadIdx.x;
  const int b = t < CM_SCAN_WG ? st->bad[t] : 0;
  const int anybad = __syncthreads_or(b);
  if (t == 0) {
    const double tr = st->tr, pre = st->pre;
    int dec = 0;
    if (anybad) {
      atomicOr(&ctrl->flags, CTRL_NONFINITE);
      dec = 1;
    } else if (mode == CHOL_FIRST) {
      if (!(sqrt(tr) > tau * sqrt(pre))) {
        atomicMin(&ctrl->q_eff, block - 1);
        dec = 1;
      }
    } else if (!(tr > 0.0)) {
      if (mode == CHOL_FIRST_BLOCK0) atomicOr(&ctrl->flags, CTRL_RANK);
      dec = 1;
    }
    st->decision = dec;
    st->fail = 0;
    st->minpiv = INFINITY;
    s_dec = dec;
    s_tr = tr;
  }
  __syncthreads();
  if (s_dec || mode != CHOL_FIRST) return;
  const double shift = shift_coef * s_tr;
  for (int i = t; i < k; i += 256) S[static_cast<int64_t>(i) * k + i] += shift;
}

// Block 0: the unshifted factor decides the rank; then S = G + shift I.
__global__ __launch_bounds__(256) void cholm_rank_kernel(int k, const double* __restrict__ G,
                                                         double tau, double shift_coef, Ctrl* ctrl,
                                                         CholMState* st, double* __restrict__ S) {
  __shared__ int s_dec;
  __shared__ double s_tr;
  const int t = threadIdx.x;
  if (t == 0) {
    int dec = st->decision;
    if (!dec && (st->fail || !(st->minpiv > rank_floor(tau, shift_coef) * sqrt(st->tr)))) {
      atomicOr(&ctrl->flags, CTRL_RANK);
      dec = 1;
      st->decision = 1;
    }
    st->fail = 0;
    st->minpiv = INFINITY;
    s_dec = dec;
    s_tr = st->tr;
  }
  __syncthreads();
  if (s_dec) return;
  const double shift = shift_coef * s_tr;
  for (int64_t i = t; i < static_cast<int64_t>(k) * k; i += 256) {
    const int r = static_cast<int>(i / k), c = static_cast<int>(i - static_cast<int64_t>(r) * k);
    S[i] = (c >= r) ? G[i] + (r == c ? shift : 0.0) : 0.0;
  }
}

// Diagonal block p: one wavefront factors S_pp (32 x 32, trailing updates
// applied) and inverts it: R_pp into R, R_pp^-1 into Rinv.  Lane c holds
// column c; both loops are rolled (a kernel this short and serial is bound
// by instruction fetch when unrolled: ~50 KB of straight-line code took
// ~26 us) and keep their register indices static by shifting: at step j
// the lane's array holds rows j, j+1, ... of its column (zeros past the
// block), so the pivot row is always entry 0.  Step j posts its row of the
// current matrix to LDS, reads it back whole (one round trip), forms
// 1 / sqrt(pivot) from the hardware estimate and two Newton steps, keeps
// row j of R in LDS and applies the rank-1 update while shifting.  The
// inverse X = R_pp^-1 is formed in the same loop from X R = I, a row of X
// per lane: lane i keeps acc_c = sum_{l < j} X_il R_lc for the columns
// c >= j (shifted like the column), takes X_ij = (delta_ij - acc_j) / R_jj
// once row j of R is known and adds X_ij R_jc to the rest (a back
// substitution after the loop, with its own register shifts, took as long
// as the factorization).
__global__ __launch_bounds__(64) void cholm_diag_kernel(int k, int o, const double* __restrict__ S,
                                                        double* __restrict__ R,
                                                        double* __restrict__ Rinv,
                                                        CholMState* st) {
  __shared__ __align__(16) double rb[64];            // row j of the current matrix
  __shared__ __align__(16) double Rs[CM][2 * CM];   // rows of R_pp, zero past column CM
  __shared__ double Xs[CM][CM + 1];                  // rows of R_pp^-1
  if (st->decision || st->fail) return;
  const int c = threadIdx.x;  // lanes 0..31: columns; 32..63 hold zeros
  const int bs = (k - o < CM) ? k - o : CM;
  double a[CM];
#pragma unroll
  for (int r = 0; r < CM; ++r) {
    // upper triangle of the block, padded with the identity to CM
    double g = 0.0;
    if (c < bs && r < bs) g = (r <= c) ? S[static_cast<int64_t>(o + r) * k + o + c] : 0.0;
    else if (c < CM && r == c) g = 1.0;
    a[r] = g;
  }
  double acc[CM];  // acc[r] = sum_{l < j} X_cl R_l,j+r for this lane's row c of X
#pragma unroll
  for (int r = 0; r < CM; ++r) acc[r] = 0.0;
  bool ok = true;
  double mp = INFINITY;
#pragma unroll 1
  for (int j = 0; j < CM; ++j) {
    rb[c] = a[0];
    wave_lds_sync();
    double bv[CM];
#pragma unroll
    for (int r = 0; r < CM; ++r) bv[r] = rb[j + r];
    double d = bv[0];
    if (!(d > 0x1p-1000) || !isfinite(d)) {  // (a pivot below 2^-1000 is a breakdown)
      ok = false;
      d = 1.0;
    }
    double inv = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    inv = fma(inv, fma(-hd * inv, inv, 0.5), inv);
    inv = fma(inv, fma(-hd * inv, inv, 0.5), inv);
    const double s0 = d * inv;
    const double rd = fma(fma(-s0, s0, d), 0.5 * inv, s0);
    if (j < bs) mp = fmin(mp, rd);
    const double rjc = (c == j) ? rd : a[0] * inv;  // R[j][c] (zero for c < j)
    Rs[j][c] = (c >= j && c < CM) ? rjc : 0.0;
    // row c of X: X_cj = (delta_cj - acc_j) / R_jj, then acc_l += X_cj R_jl
    // for l > j, with R_jl = bv[l - j] / R_jj
    const double xcj = ((c == j ? 1.0 : 0.0) - acc[0]) * inv;
    if (c < CM) Xs[c][j] = xcj;
    const double wj = xcj * inv;
    const double tj = a[0] * inv * inv;  // S[j][c] / pivot
#pragma unroll
    for (int r = 0; r + 1 < CM; ++r) {
      a[r] = a[r + 1] - bv[r + 1] * tj;
      acc[r] = fma(wj, bv[r + 1], acc[r + 1]);
    }
    a[CM - 1] = 0.0;
    acc[CM - 1] = 0.0;
    wave_lds_sync();  // (row j's reads come before the next post)
  }
  wave_lds_sync();
  if (ok && c < bs) {
#pragma unroll
    for (int r = 0; r < CM; ++r) {
      if (r <= c) {
        R[static_cast<int64_t>(o + r) * k + o + c] = Rs[r][c];
        Rinv[static_cast<int64_t>(o + r) * k + o + c] = Xs[r][c];
      }
    }
  }
  if (c == 0) {
    if (!ok) st->fail = 1;
    else if (mp < st->minpiv) st->minpiv = mp;
  }
}

// Trailing update after diagonal block p, a workgroup per 32 x 32 tile
// (ti, tj), ti <= tj, of the trailing upper triangle: the two panel-row
// blocks R_p,ti = R_pp^-T S_p,ti and R_p,tj (32 x 32 x 32 each, from the
// raw rows of S, which stay untouched), then S_ti,tj -= R_p,ti^T R_p,tj.
// The diagonal tiles store their panel-row block into R.
__global__ __launch_bounds__(256) void cholm_update_kernel(int k, int o, int bs,
                                                           double* __restrict__ S,
                                                           double* __restrict__ R,
                                                           const double* __restrict__ Rinv,
                                                           const CholMState* st) {
  __shared__ double Ri[CM][CM + 1], Pi[CM][CM + 1], Pj[CM][CM + 1];
  if (st->decision || st->fail) return;
  const int t = threadIdx.x;
  const int base = o + bs, rest = k - base;
  const int nt = (rest + CM - 1) / CM;
  // blockIdx.x -> tile (ti, tj), ti <= tj, row-major over the upper triangle
  int e = static_cast<int>(blockIdx.x), ti = 0;
  while (e >= nt - ti) {
    e -= nt - ti;
    ++ti;
  }
  const int tj = ti + e;
  // all 12 loads in flight: addresses clamped into the k x k arrays, the
  // values outside the blocks replaced by zero after the load
#pragma unroll
  for (int q = 0; q < CM * CM / 256; ++q) {
    const int idx = t + 256 * q;
    const int r = idx / CM, c = idx % CM;
    const int gi = base + CM * ti + c, gj = base + CM * tj + c;
    const int64_t row = static_cast<int64_t>(min(o + r, k - 1)) * k;
    const double vr = Rinv[row + min(o + c, k - 1)];
    const double vi = S[row + min(gi, k - 1)];
    const double vj = S[row + min(gj, k - 1)];
    Ri[r][c] = (r < bs && c < bs && r <= c) ? vr : 0.0;  // R_pp^-1 (upper)
    Pi[r][c] = (r < bs && gi < k) ? vi : 0.0;
    Pj[r][c] = (r < bs && gj < k) ? vj : 0.0;
  }
  __syncthreads();
  // panel rows: X[r][c] = sum_{l <= r} Rinv_pp[l][r] P[l][c], four per
  // thread (each sum in increasing l; P's entries read once per l)
  const int tx = t & 31, ty = t >> 5;
  double xi[4] = {0.0, 0.0, 0.0, 0.0}, xj[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int l = 0; l < CM; ++l) {
    const double pi = Pi[l][tx], pj = Pj[l][tx];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double w = Ri[l][ty + 8 * u];
      xi[u] += w * pi;
      xj[u] += w * pj;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    Pi[ty + 8 * u][tx] = xi[u];
    Pj[ty + 8 * u][tx] = xj[u];
  }
  __syncthreads();
  if (ti == tj) {
    const int gc = base + CM * ti + tx;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = ty + 8 * u;
      if (r < bs && gc < k) R[static_cast<int64_t>(o + r) * k + gc] = Pi[r][tx];
    }
  }
  // S_ti,tj -= X_i^T X_j (each sum in increasing r), the four rows' entries
  // of S loaded before the sums
  const int j = base + CM * tj + tx;
  double sv[4], sum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + CM * ti + ty + 8 * u;
    sv[u] = S[static_cast<int64_t>(min(i, k - 1)) * k + min(j, k - 1)];
  }
#pragma unroll 8
  for (int r = 0; r < CM; ++r) {
    const double pj = Pj[r][tx];
#pragma unroll
    for (int u = 0; u < 4; ++u) sum[u] += Pi[r][ty + 8 * u] * pj;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + CM * ti + ty + 8 * u;
    if (i < k && j < k && i <= j) S[static_cast<int64_t>(i) * k + j] = sv[u] - sum[u];
  }
}

// R^-1 by doubling (after the diagonal blocks' inverses): at level L the
// pairs of neighbouring diagonal blocks of 2^(L-1) 32-blocks become one,
// with X12 = -X11 (R12 X22): phase 0 forms T = R12 X22 into the scratch S
// (no longer needed once R is complete), phase 1 writes -X11 T into R^-1.
// A workgroup per 32 x 32 output tile; the lower triangles of the diagonal
// blocks of R^-1 (not written by the diagonal kernel) read as zero.
template <int PHASE>
__global__ __launch_bounds__(256) void cholm_invlevel_kernel(int k, int nbb,
                                                             const double* __restrict__ R,
                                                             double* __restrict__ Rinv,
                                                             double* __restrict__ T,
                                                             const CholMState* st) {
  __shared__ double Ab[CM][CM + 1], Bb[CM][CM + 1];
  if (st->decision || st->fail) return;
  const int nb = (k + CM - 1) / CM;
  const int per = nbb * nbb;
  const int pair = blockIdx.x / per, rem = blockIdx.x - pair * per;
  const int ti = rem / nbb, tj = rem - (rem / nbb) * nbb;
  const int b1 = pair * 2 * nbb, b2 = b1 + nbb;  // first block of each half
  const int I = b1 + ti, J = b2 + tj;
  if (J >= nb) return;  // (uniform) past the last block
  const int t = threadIdx.x, tx = t & 31, ty = t >> 5;
  // PHASE 0: sum over L in [b2, J] of R[I][L] Rinv[L][J]
  // PHASE 1: sum over L in [I, b2) of Rinv[I][L] T[L][J]
  const int l0 = PHASE == 0 ? b2 : I;
  const int l1 = PHASE == 0 ? J : b2 - 1;
  const double* Asrc = PHASE == 0 ? R : Rinv;
  const double* Bsrc = PHASE == 0 ? Rinv : T;
  // block pair L's 8 entries per thread, loaded (clamped addresses, entries
  // outside the blocks or below a diagonal block's diagonal zeroed after the
  // load) while pair L - 1 is multiplied
  double av[CM * CM / 256], bv[CM * CM / 256];
  auto fetch = [&](int L) {
#pragma unroll
    for (int q = 0; q < CM * CM / 256; ++q) {
      const int e = t + 256 * q;
      const int r = e / CM, c = e - (e / CM) * CM;
      const int ga = I * CM + r, gl = L * CM + c;  // left block (I, L)
      const int gb = L * CM + r, gj = J * CM + c;  // right block (L, J)
      const double a = Asrc[static_cast<int64_t>(min(ga, k - 1)) * k + min(gl, k - 1)];
      const double b = Bsrc[static_cast<int64_t>(min(gb, k - 1)) * k + min(gj, k - 1)];
      const bool aok = ga < k && gl < k && (PHASE == 0 || L != I || r <= c);
      const bool bok = gb < k && gj < k && (PHASE == 1 || L != J || r <= c);
      av[q] = aok ? a : 0.0;
      bv[q] = bok ? b : 0.0;
    }
  };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  fetch(l0);
  for (int L = l0; L <= l1; ++L) {
#pragma unroll
    for (int q = 0; q < CM * CM / 256; ++q) {
      const int e = t + 256 * q;
      Ab[e / CM][e % CM] = av[q];
      Bb[e / CM][e % CM] = bv[q];
    }
    __syncthreads();
    if (L < l1) fetch(L + 1);
    // (each block's sum in increasing l, then added to the running sum)
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int l = 0; l < CM; ++l) {
      const double b = Bb[l][tx];
#pragma unroll
      for (int u = 0; u < 4; ++u) sum[u] += Ab[ty + 8 * u][l] * b;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += sum[u];
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gr = I * CM + ty + 8 * u, gc = J * CM + tx;
    if (gr < k && gc < k) {
      if (PHASE == 0) T[static_cast<int64_t>(gr) * k + gc] = acc[u];
      else Rinv[static_cast<int64_t>(gr) * k + gc] = -acc[u];
    }
  }
}


__global__ __launch_bounds__(256) void cholm_end_kernel(int k, double* __restrict__ R,
                                                        double* __restrict__ Rinv, int block,
                                                        Ctrl* ctrl, const CholMState* st) {
  const int dec = st->decision, fail = st->fail;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !dec && fail) {
    if (block == 0) atomicOr(&ctrl->flags, CTRL_RANK);
    else atomicMin(&ctrl->q_eff, block - 1);
  }
  const bool zero = dec || fail;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= static_cast<int64_t>(k) * k) return;
  const int r = static_cast<int>(i / k), c = static_cast<int>(i - static_cast<int64_t>(r) * k);
  if (zero || c < r) {
    R[i] = 0.0;
    Rinv[i] = 0.0;
  }
}

__global__ __launch_bounds__(256) void trmm_upper_kernel(int k, const double* A,
                                                         const double* B,
                                                         double* T) {
  for (int idx = threadIdx.x; idx < k * k; idx += 256) {
    const int r = idx / k, c = idx % k;
    double s = 0.0;
    for (int l = r; l <= c; ++l) s += A[r * k + l] * B[l * k + c];
    T[idx] = (c >= r) ? s : 0.0;
  }
}

// dst (cols x rows, ldd) = src (rows x cols, lds)^T through a 32 x 33 tile.
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void transpose_kernel(const TS* __restrict__ src, int64_t lds,
                                                        TD* __restrict__ dst, int64_t ldd,
                                                        int64_t rows, int64_t cols) {
  __shared__ double tile[32][33];
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 32, c0 = static_cast<int64_t>(blockIdx.x) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? static_cast<double>(src[r * lds + c]) : 0.0;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) dst[c * ldd + r] = static_cast<TD>(tile[tx][i]);
  }
}

// out = copyltu(-S): the symmetric matrix whose lower triangle is -S's.
__global__ __launch_bounds__(256) void copyltu_neg_kernel(int k, const double* S, double* out) {
  for (int idx = threadIdx.x; idx < k * k; idx += 256) {
    const int i = idx / k, j = idx % k;
    out[idx] = (i >= j) ? -S[i * k + j] : -S[j * k + i];
  }
}

// Eigen adjoint core: G (m x k) with G[j][j] = theta_bar_j and, for i >= k,
// G[i][j] = H[i][j] / (theta_j - theta_i); entries with i, j < k stay zero
// (they cancel for losses invariant under rotations inside span Z).
__global__ __launch_bounds__(256) void eig_adjoint_kernel(int64_t m, int k, const double* theta,
                                                          const double* H, const double* ritz,
                                                          const double* ritz_bar, double* G) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= m * k) return;
  const int64_t i = idx / k;
  const int j = static_cast<int>(idx - i * k);
  double v = 0.0;
  if (i == j) {
    const double sb = ritz_bar ? ritz_bar[j] : 0.0;
    v = ritz[j] > 0.0 ? sb / (2.0 * ritz[j]) : 0.0;  // d sigma / d theta
  } else if (i >= k) {
    const double gap = theta[j] - theta[i];
    if (fabs(gap) > 1e-14 * fabs(theta[0])) v = H[idx] / gap;
  }
  G[idx] = v;
}

__global__ __launch_bounds__(256) void symmetrize_kernel(int64_t m, double* M) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx / m, j = idx - i * m;
  if (j <= i) return;
  const double v = 0.5 * (M[i * m + j] + M[j * m + i]);
  M[i * m + j] = v;
  M[j * m + i] = v;
}

// out = (R^-1)^T for an upper-triangular k x k R (one workgroup).
__global__ __launch_bounds__(256) void trinv_t_kernel(int k, const double* R, double* Ri,
                                                      double* out) {
  for (int i = threadIdx.x; i < k * k; i += 256) Ri[i] = 0.0;
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double rii = R[i * k + i];
    for (int j = i + threadIdx.x; j < k; j += 256) {
      if (j == i) {
        Ri[i * k + i] = rii != 0.0 ? 1.0 / rii : 0.0;
      } else {
        double s = 0.0;
        for (int l = i + 1; l <= j; ++l) s += R[i * k + l] * Ri[l * k + j];
        Ri[i * k + j] = rii != 0.0 ? -s / rii : 0.0;
      }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < k * k; idx += 256) {
    const int i = idx / k, j = idx % k;
    out[idx] = Ri[j * k + i];
  }
}

// U (m x m, ld m) = eigenvectors in descending order: column c is column
// order[c] of V, times sign[c] for c < k (the signs applied to Z).
__global__ __launch_bounds__(256) void gather_vectors_kernel(const double* Vc, int64_t ldc,
                                                             int64_t m, const int32_t* order,
                                                             const double* sign, int k,
                                                             double* U) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t r = idx / m, c = idx - r * m;
  int64_t j = order[c];
  j = j < 0 ? 0 : (j >= m ? m - 1 : j);
  const double sg = (c < k && sign) ? sign[c] : 1.0;
  U[idx] = sg * Vc[j * ldc + r];
}

template <typename T>
__global__ __launch_bounds__(256) void col_sign_kernel(const T* Z, int64_t n,
                                                       int64_t ldz,
                                                       double* sign) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  double best = -1.0;
  int64_t bidx = n;
  // eight rows per thread in flight (clamped, unconditional loads), then
  // compared in increasing row order: the first maximum is kept
  for (int64_t r0 = t; r0 < n; r0 += 256 * 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = r0 + 256 * u;
      const double x = fabs(static_cast<double>(Z[(r < n ? r : n - 1) * ldz + c]));
      a[u] = r < n ? x : -1.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (a[u] > best) {
        best = a[u];
        bidx = r0 + 256 * u;
      }
    }
  }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      const double o = bv[t + w];
      const int64_t oi = bi[t + w];
      if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
        bv[t] = o;
        bi[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    double sg = 1.0;
    if (bi[0] < n && static_cast<double>(Z[bi[0] * ldz + c]) < 0.0) sg = -1.0;
    sign[c] = sg;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void apply_sign_kernel(T* Z, int64_t n, int k,
                                                         int64_t ldz, double* U,
                                                         int64_t m, int64_t ldu,
                                                         const double* sign) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nz = n * k;
  if (i < nz) {
    const int64_t r = i / k;
    const int c = static_cast<int>(i - r * k);
    if (sign[c] < 0.0) Z[r * ldz + c] = -Z[r * ldz + c];
  } else if (U && i < nz + m * k) {
    const int64_t j = i - nz;
    const int64_t r = j / k;
    const int c = static_cast<int>(j - r * k);
    if (sign[c] < 0.0) U[r * ldu + c] = -U[r * ldu + c];
  }
}

}  // namespace

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) fill_kernel<double><<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(p, n, v);
}
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n > 0) fill_kernel<float><<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(p, n, v);
}
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) fill_kernel<int32_t><<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(p, n, v);
}

void launch_copy2d(const void* src, bool src_f64, int64_t lds, void* dst,
                   bool dst_f64, int64_t ldd, int64_t rows, int64_t cols,
                   hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  const unsigned g = static_cast<unsigned>(cdiv(rows * cols, 256));
  if (src_f64 && dst_f64)
    copy2d_kernel<double, double><<<g, 256, 0, s>>>(
        static_cast<const double*>(src), lds, static_cast<double*>(dst), ldd, rows, cols);
  else if (src_f64)
    copy2d_kernel<double, float><<<g, 256, 0, s>>>(
        static_cast<const double*>(src), lds, static_cast<float*>(dst), ldd, rows, cols);
  else if (dst_f64)
    copy2d_kernel<float, double><<<g, 256, 0, s>>>(
        static_cast<const float*>(src), lds, static_cast<double*>(dst), ldd, rows, cols);
  else
    copy2d_kernel<float, float><<<g, 256, 0, s>>>(
        static_cast<const float*>(src), lds, static_cast<float*>(dst), ldd, rows, cols);
}

void launch_axpy_f64(const double* x, double* y, int64_t n, hipStream_t s) {
  if (n > 0) axpy_kernel<<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(x, y, n);
}

void launch_ctrl_init(Ctrl* c, int32_t q, hipStream_t s) {
  ctrl_init_kernel<<<1, 64, 0, s>>>(c, q);
}
void launch_ctrl_reset_off(Ctrl* c, hipStream_t s) {
  ctrl_reset_off_kernel<<<1, 64, 0, s>>>(c);
}

void launch_chol(int k, const double* G, const double* Gpre, int mode, int block,
                 double tau, double shift_coef, double* R, double* Rinv,
                 double* work, Ctrl* ctrl, hipStream_t s) {
  // Both k x k factors in LDS when they fit (k <= 96: 144 KB of 160 KB).
  const size_t need = static_cast<size_t>(2) * k * k * sizeof(double);
  const int use_lds = k <= 96 ? 1 : 0;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(chol_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    attr_set = true;
  }
  // k <= 64: the factor lives in the registers of one wavefront
#define BK_CHOL_WAVE(KK)                                                                   \
  if (k <= KK) {                                                                           \
    chol_wave_kernel<KK><<<1, 64, 0, s>>>(k, G, Gpre, mode, block, tau, shift_coef, R, Rinv, \
                                          ctrl);                                          \
    return;                                                                                \
  }
  BK_CHOL_WAVE(8)
  BK_CHOL_WAVE(16)
  BK_CHOL_WAVE(24)
  BK_CHOL_WAVE(32)
  BK_CHOL_WAVE(48)
  BK_CHOL_WAVE(64)
#undef BK_CHOL_WAVE
  if (k <= kCholBlockedMax) {
    double* S = work;
    CholMState* st = reinterpret_cast<CholMState*>(work + static_cast<int64_t>(k) * k);
    const int nb = (k + CM - 1) / CM;
    cholm_scan_kernel<<<CM_SCAN_WG, 256, 0, s>>>(k, G, Gpre, mode, st, S);
    cholm_decide_kernel<<<1, 256, 0, s>>>(k, mode, block, tau, shift_coef, ctrl, st, S);
    auto factor = [&]() {
      for (int p = 0; p < nb; ++p) {
        const int o = p * CM, bs = std::min(CM, k - o);
        cholm_diag_kernel<<<1, 64, 0, s>>>(k, o, S, R, Rinv, st);
        const int rest = k - o - bs;
        if (rest > 0) {
          const int nt = (rest + CM - 1) / CM;
          cholm_update_kernel<<<nt * (nt + 1) / 2, 256, 0, s>>>(k, o, bs, S, R, Rinv, st);
        }
      }
    };
    factor();
    if (mode == CHOL_FIRST_BLOCK0) {
      cholm_rank_kernel<<<1, 256, 0, s>>>(k, G, tau, shift_coef, ctrl, st, S);
      factor();
    }
    // R^-1 above the diagonal blocks by doubling: log2(nb) levels of two
    // launches
    for (int nbb = 1; nbb < nb; nbb *= 2) {
      const int pairs = (nb + 2 * nbb - 1) / (2 * nbb);
      const unsigned g = static_cast<unsigned>(pairs * nbb * nbb);
      cholm_invlevel_kernel<0><<<g, 256, 0, s>>>(k, nbb, R, Rinv, S, st);
      cholm_invlevel_kernel<1><<<g, 256, 0, s>>>(k, nbb, R, Rinv, S, st);
    }
    cholm_end_kernel<<<static_cast<unsigned>(cdiv(static_cast<int64_t>(k) * k, 256)), 256, 0, s>>>(
        k, R, Rinv, block, ctrl, st);
    return;
  }
  chol_kernel<<<1, 256, use_lds ? need : 0, s>>>(k, G, Gpre, mode, block, tau, shift_coef, R,
                                                 Rinv, work, ctrl, use_lds);
}

void launch_trmm_upper(int k, const double* A, const double* B, double* T,
                       hipStream_t s) {
  trmm_upper_kernel<<<1, 256, 0, s>>>(k, A, B, T);
}

namespace {
constexpr int CQR_ROWS = 256;   // rows per chunk (one per thread)
constexpr int CQR_MAX_WG = 64;  // workgroups (and Gram partials) per pass

// One CholeskyQR pass for k <= 32 in one launch.  Every workgroup
//  1. adds the P Gram partials Gin[p k k] in a fixed order (the same G in
//     every workgroup);
//  2. factors G [+ shift] in wavefront 0 with the mode logic of
//     chol_wave_kernel (workgroup 0 reports to ctrl and writes R);
//  3. for each chunk of 256 rows of its range: Y R = X by forward
//     substitution, one thread per row (no R^-1 is formed), the rows stored
//     in the working type, and their Gram accumulated in FP64 from the
//     stored values; the workgroup's Gram goes to gout[blockIdx.x k k]
//     (nullable).
// A dropped block (zero factor) gives Y = 0.  X may be Y.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

// VEC: rows are copied with 16-byte accesses (k, ldx, ldy multiples of the
// vector width and X, Y 16-byte aligned).
template <typename T, int K, bool VEC>
__global__ __launch_bounds__(256) void cqr_pass_kernel(
    int64_t n, int k, const double* __restrict__ Gin, int P, const double* __restrict__ Gpre,
    int mode, int block, double tau, double shift_coef, double* __restrict__ R, Ctrl* ctrl,
    const T* X, int64_t ldx, T* Y, int64_t ldy, int64_t rows_per_wg, double* __restrict__ gout,
    double skip_tol, const float* __restrict__ mu, double* __restrict__ mupart) {
  constexpr int LD = K + 1;
  constexpr int TPR = (K == 24) ? 32 : K;  // threads per row in the tile copies
  constexpr int RPI = 256 / TPR;           // rows per copy step
  constexpr int NC = CQR_ROWS / RPI;       // copy steps per chunk
  using V = typename Vec16<T>::type;
  constexpr int VW = 16 / sizeof(T);       // vector width
  constexpr int NQ = (K + VW - 1) / VW;    // vectors per row, at most
  constexpr int NX = VEC ? NQ : NC;        // copy registers per thread
  constexpr int NE = (K * K + 255) / 256;  // Gram entries per thread in the sum
  constexpr int PB = 24;                   // partials loaded per batch
  constexpr int GB = K / 8;                // Gram block edge per lane (8 x 8 lanes)
  __shared__ double Gs[K * K];
  __shared__ double Rs[K * K];
  __shared__ double rd[K];
  __shared__ double pd[K];
  __shared__ double rb[128];
  __shared__ double Ys[CQR_ROWS * LD];
  __shared__ double mus[CQR_ROWS];
  const int t = threadIdx.x;
  const int kk = k * k;
  const int gc = t % TPR, gr = t / TPR;  // copy layout
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
  const int64_t hi = lo + rows_per_wg < n ? lo + rows_per_wg : n;
  // vector copies: item i = t + 256 q of a chunk is row i / kv, vector
  // i % kv (the quotient by a multiply-high, exact for i < 2^12, kv <= 16)
  const int kv = k / VW;
  const unsigned kvm = VEC ? 0xFFFFFFFFu / static_cast<unsigned>(kv) + 1u : 0u;
  // a chunk's rows: one T (scalar copies) or one V (vector copies) per item
  V xv[NX];
  auto fetch = [&](int64_t c0, int rows) {
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      V v;
      if (VEC) {
        const unsigned i = static_cast<unsigned>(t + 256 * q);
        const int r = static_cast<int>(__umulhi(i, kvm));
        const int cv = static_cast<int>(i) - r * kv;
        if (q < kv && r < rows)
          v = *reinterpret_cast<const V*>(X + (c0 + r) * ldx + cv * VW);
        else
          v = V{};
      } else {
        const int r = gr + q * RPI;
        v = V{};
        v.x = (gc < k && r < rows) ? X[(c0 + r) * ldx + gc] : static_cast<T>(0);
      }
      xv[q] = v;
    }
  };
  auto stage = [&]() {  // the fetched rows into Ys (FP64)
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      if (VEC) {
        const unsigned i = static_cast<unsigned>(t + 256 * q);
        const int r = static_cast<int>(__umulhi(i, kvm));
        const int cv = static_cast<int>(i) - r * kv;
        if (q < kv) {
          const T* e = reinterpret_cast<const T*>(&xv[q]);
#pragma unroll
          for (int w = 0; w < VW; ++w) Ys[r * LD + cv * VW + w] = static_cast<double>(e[w]);
        }
      } else if (gc < K) {
        Ys[(gr + q * RPI) * LD + gc] = static_cast<double>(xv[q].x);
      }
    }
  };
  // the first chunk's rows are requested before the Gram sum and the factor
  fetch(lo, static_cast<int>(hi - lo < CQR_ROWS ? hi - lo : CQR_ROWS));
  const double gpre_d = (mode == CHOL_FIRST && t < k) ? Gpre[t * k + t] : 0.0;
  // G = sum of the partials in index order, PB independent loads in flight
  {
    double sum[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) sum[u] = 0.0;
    for (int p0 = 0; p0 < P; p0 += PB) {
      double v[NE][PB];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = t + 256 * u;
#pragma unroll
        for (int j = 0; j < PB; ++j)
          v[u][j] = (e < kk && p0 + j < P) ? Gin[static_cast<int64_t>(p0 + j) * kk + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NE; ++u)
#pragma unroll
        for (int j = 0; j < PB; ++j) sum[u] += v[u][j];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = t + 256 * u;
      if (e < kk) {
        const int r = e / k;
        Gs[r * K + (e - r * k)] = sum[u];
      }
    }
  }
  __syncthreads();
  if (skip_tol > 0.0) {
    // X already orthonormal to working precision (max |G - I| <= skip_tol,
    // the same decision in every workgroup): R = I, Y = X (in place)
    double dev = 0.0;
    for (int e = t; e < kk; e += 256) {
      const int r = e / k, cc = e - r * k;
      dev = fmax(dev, fabs(Gs[r * K + cc] - (r == cc ? 1.0 : 0.0)));
    }
    for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o));
    if ((t & 63) == 0) pd[t >> 6] = dev;  // (pd is rewritten after the next barrier)
    __syncthreads();
    dev = fmax(fmax(pd[0], pd[1]), fmax(pd[2], pd[3]));
    if (!(dev > skip_tol)) {
      if (blockIdx.x == 0)
        for (int e = t; e < kk; e += 256) R[e] = (e / k == e % k) ? 1.0 : 0.0;
      return;
    }
    __syncthreads();
  }
  if (t < K) pd[t] = gpre_d;
  __syncthreads();
  if (t < 64) {
    const int c = t;
    double g[K];
    int bad = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const double x = (r < k && c < k) ? Gs[r * K + c] : 0.0;
      if (!isfinite(x)) bad = 1;
      g[r] = x;
    }
    // the traces, summed in index order by every lane
    double tr = 0.0, pre = 0.0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      tr += r < k ? Gs[r * K + r] : 0.0;  // (entries beyond k are unset)
      pre += pd[r];
    }
    double a[K], rinv[K];
    const bool zero = chol_wave_factor<K>(k, g, bad, tr, pre, mode, block, tau, shift_coef,
                                          blockIdx.x == 0, ctrl, a, rinv, rb);
    if (c < K) {
      double dinv = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j == c) dinv = rinv[j];
      rd[c] = (zero || c >= k) ? 0.0 : dinv;
#pragma unroll
      for (int r = 0; r < K; ++r)
        Rs[r * K + c] = (zero || c >= k || r > c) ? 0.0 : a[r];
      if (blockIdx.x == 0 && c < k) {
#pragma unroll
        for (int r = 0; r < K; ++r)
          if (r < k) R[r * k + c] = (zero || r > c) ? 0.0 : a[r];
      }
    }
  }
  // wavefront w sums the Gram of rows [64 w, 64 w + 64) of each chunk; lane
  // (la, lb) holds the GB x GB block at (GB la, GB lb)
  const int w = t >> 6, la = (t & 63) >> 3, lb = t & 7;
  double acc[GB][GB];
#pragma unroll
  for (int x = 0; x < GB; ++x)
#pragma unroll
    for (int z = 0; z < GB; ++z) acc[x][z] = 0.0;
  // mu^T Y: lane c of wavefront w sums column c over rows [64 w, 64 w + 64)
  double musum = 0.0;
  const int mc = t & 63;
  for (int64_t r0 = lo; r0 < hi; r0 += CQR_ROWS) {
    const int rows = static_cast<int>(hi - r0 < CQR_ROWS ? hi - r0 : CQR_ROWS);
    if (r0 != lo) fetch(r0, rows);
    if (mupart) mus[t] = t < rows ? static_cast<double>(mu[r0 + t]) : 0.0;
    stage();
    __syncthreads();
    double y[K];
#pragma unroll
    for (int c = 0; c < K; ++c) y[c] = c < k ? Ys[t * LD + c] : 0.0;  // (unset beyond k)
    // right-looking: each solved entry updates the later ones at once, in
    // the same order as the row-by-row sums (short dependency chains); row
    // j + 1 of R is read from LDS while row j is applied
    double rn[K];
#pragma unroll
    for (int c = 1; c < K; ++c) rn[c] = Rs[c];
    rn[0] = rd[0];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double rc[K];
#pragma unroll
      for (int c = j; c < K; ++c) rc[c] = rn[c];
      if (j + 1 < K) {
        rn[j + 1] = rd[j + 1];
#pragma unroll
        for (int c = j + 2; c < K; ++c) rn[c] = Rs[(j + 1) * K + c];
      }
      y[j] *= rc[j];
#pragma unroll
      for (int c = j + 1; c < K; ++c) y[c] -= y[j] * rc[c];
    }
#pragma unroll
    for (int c = 0; c < K; ++c) Ys[t * LD + c] = static_cast<double>(static_cast<T>(y[c]));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      if (VEC) {
        const unsigned i = static_cast<unsigned>(t + 256 * q);
        const int r = static_cast<int>(__umulhi(i, kvm));
        const int cv = static_cast<int>(i) - r * kv;
        if (q < kv && r < rows) {
          V v;
          T* e = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int w = 0; w < VW; ++w) e[w] = static_cast<T>(Ys[r * LD + cv * VW + w]);
          *reinterpret_cast<V*>(Y + (r0 + r) * ldy + cv * VW) = v;
        }
      } else {
        const int r = gr + q * RPI;
        if (gc < k && r < rows) Y[(r0 + r) * ldy + gc] = static_cast<T>(Ys[r * LD + gc]);
      }
    }
    if (mupart && mc < k) {
      // rows past the chunk have mus = 0 (Ys holds whatever was staged)
#pragma unroll 8
      for (int r = 64 * w; r < 64 * w + 64; ++r) musum += mus[r] * Ys[r * LD + mc];
    }
    if (gout) {
#pragma unroll 8
      for (int r = 64 * w; r < 64 * w + 64; ++r) {
        double av[GB], bv[GB];
#pragma unroll
        for (int x = 0; x < GB; ++x) {
          av[x] = Ys[r * LD + GB * la + x];
          bv[x] = Ys[r * LD + GB * lb + x];
        }
#pragma unroll
        for (int x = 0; x < GB; ++x)
#pragma unroll
          for (int z = 0; z < GB; ++z) acc[x][z] += av[x] * bv[z];
      }
    }
    __syncthreads();
  }
  if (mupart) {
    // the four wavefronts' sums in wavefront order (rb is free after the
    // factor: 4 x 32 doubles)
    if (mc < k) rb[w * 32 + mc] = musum;
    __syncthreads();
    if (t < k)
      mupart[static_cast<int64_t>(blockIdx.x) * k + t] =
          ((rb[t] + rb[32 + t]) + rb[64 + t]) + rb[96 + t];
  }
  if (!gout) return;
  // the four wavefronts' sums, added in wavefront order
  double* ws = Ys;  // 4 K x K
#pragma unroll
  for (int x = 0; x < GB; ++x)
#pragma unroll
    for (int z = 0; z < GB; ++z) ws[w * K * K + (GB * la + x) * K + GB * lb + z] = acc[x][z];
  __syncthreads();
  double* g = gout + static_cast<int64_t>(blockIdx.x) * kk;
  for (int e = t; e < kk; e += 256) {
    const int a = e / k, b = e - a * k;
    const int o = a * K + b;
    g[e] = ((ws[o] + ws[K * K + o]) + ws[2 * K * K + o]) + ws[3 * K * K + o];
  }
}

template <typename T, int K>
void cqr_pass_launch(unsigned grid, const CqrPass& a, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  const bool vec = a.k % VW == 0 && a.ldx % VW == 0 && a.ldy % VW == 0 &&
                   reinterpret_cast<uintptr_t>(a.X) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(a.Y) % 16 == 0;
  if (vec)
    cqr_pass_kernel<T, K, true><<<grid, 256, 0, s>>>(
        a.n, a.k, a.Gin, a.P, a.Gpre, a.mode, a.block, a.tau, a.shift_coef, a.R, a.ctrl,
        static_cast<const T*>(a.X), a.ldx, static_cast<T*>(a.Y), a.ldy, a.rows_per_wg, a.gout,
        a.skip_tol, a.mu, a.mupart);
  else
    cqr_pass_kernel<T, K, false><<<grid, 256, 0, s>>>(
        a.n, a.k, a.Gin, a.P, a.Gpre, a.mode, a.block, a.tau, a.shift_coef, a.R, a.ctrl,
        static_cast<const T*>(a.X), a.ldx, static_cast<T*>(a.Y), a.ldy, a.rows_per_wg, a.gout,
        a.skip_tol, a.mu, a.mupart);
}
}  // namespace

int cqr_pass_grid(int64_t n, int64_t* rows_per_wg) {
  int64_t chunks = cdiv(n, CQR_ROWS);
  if (chunks < 1) chunks = 1;
  const int64_t per = cdiv(chunks, CQR_MAX_WG);
  const int64_t g = cdiv(chunks, per);
  if (rows_per_wg) *rows_per_wg = per * CQR_ROWS;
  return static_cast<int>(g);
}

int64_t cqr_pass_partial_elems(int k) {
  return k <= kCqrPassMaxK ? static_cast<int64_t>(CQR_MAX_WG) * k * k : 0;
}

int launch_cqr_pass(const CqrPass& a, hipStream_t s) {
  if (a.n <= 0 || a.k <= 0 || a.k > kCqrPassMaxK || a.P < 1) return 0;
  int64_t per = 0;
  const unsigned g = static_cast<unsigned>(cqr_pass_grid(a.n, &per));
  CqrPass b = a;
  b.rows_per_wg = per;
#define BK_CQR(KK)                                                  \
  if (a.k <= KK) {                                                  \
    if (a.f64) cqr_pass_launch<double, KK>(g, b, s);                \
    else cqr_pass_launch<float, KK>(g, b, s);                       \
    return 1;                                                       \
  }
  BK_CQR(8)
  BK_CQR(16)
  BK_CQR(24)
  BK_CQR(32)
#undef BK_CQR
  return 0;
}

void launch_transpose(const void* src, bool src_f64, int64_t lds, void* dst, bool dst_f64,
                      int64_t ldd, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(cols, 32)), static_cast<unsigned>(cdiv(rows, 32)));
  if (src_f64 && dst_f64)
    transpose_kernel<double, double><<<grid, 256, 0, s>>>(static_cast<const double*>(src), lds,
                                                          static_cast<double*>(dst), ldd, rows, cols);
  else if (src_f64)
    transpose_kernel<double, float><<<grid, 256, 0, s>>>(static_cast<const double*>(src), lds,
                                                         static_cast<float*>(dst), ldd, rows, cols);
  else if (dst_f64)
    transpose_kernel<float, double><<<grid, 256, 0, s>>>(static_cast<const float*>(src), lds,
                                                         static_cast<double*>(dst), ldd, rows, cols);
  else
    transpose_kernel<float, float><<<grid, 256, 0, s>>>(static_cast<const float*>(src), lds,
                                                        static_cast<float*>(dst), ldd, rows, cols);
}

void launch_copyltu_neg(int k, const double* S, double* out, hipStream_t s) {
  copyltu_neg_kernel<<<1, 256, 0, s>>>(k, S, out);
}

void launch_eig_adjoint(int64_t m, int k, const double* theta, const double* H,
                        const double* ritz, const double* ritz_bar, double* G, hipStream_t s) {
  eig_adjoint_kernel<<<static_cast<unsigned>(cdiv(m * k, 256)), 256, 0, s>>>(m, k, theta, H, ritz,
                                                                           ritz_bar, G);
}

void launch_symmetrize(int64_t m, double* M, hipStream_t s) {
  symmetrize_kernel<<<static_cast<unsigned>(cdiv(m * m, 256)), 256, 0, s>>>(m, M);
}

void launch_trinv_t(int k, const double* R, double* work, double* out, hipStream_t s) {
  trinv_t_kernel<<<1, 256, 0, s>>>(k, R, work, out);
}

void launch_gather_vectors(const double* Vc, int64_t ldc, int64_t m, const int32_t* order,
                           const double* sign, int k, double* U, hipStream_t s) {
  gather_vectors_kernel<<<static_cast<unsigned>(cdiv(m * m, 256)), 256, 0, s>>>(Vc, ldc, m, order,
                                                                              sign, k, U);
}

void launch_sign_normalize(void* Z, bool f64, int64_t n, int k, int64_t ldz,
                           double* U, int64_t m, int64_t ldu, double* sign,
                           hipStream_t s) {
  if (k <= 0) return;
  const int64_t tot = n * k + (U ? m * k : 0);
  const unsigned g = static_cast<unsigned>(cdiv(tot, 256));
  if (f64) {
    col_sign_kernel<double><<<k, 256, 0, s>>>(static_cast<const double*>(Z), n, ldz, sign);
    apply_sign_kernel<double><<<g, 256, 0, s>>>(static_cast<double*>(Z), n, k, ldz, U, m,
                                                ldu, sign);
  } else {
    col_sign_kernel<float><<<k, 256, 0, s>>>(static_cast<const float*>(Z), n, ldz, sign);
    apply_sign_kernel<float><<<g, 256, 0, s>>>(static_cast<float*>(Z), n, k, ldz, U, m,
                                               ldu, sign);
  }
}

}  // namespace bk
