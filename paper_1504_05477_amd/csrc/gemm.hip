// Skinny dense products of the Krylov loop (Algorithm 2, steps 2-6):
//   NN:  C = alpha A X + beta C        A n x K, X K x N, N small (<= ~2k)
//   TN:  C = alpha X^T Y + beta C      X L x p, Y L x r, long reduction L
// These generic LDS-tiled kernels cover every element type; the wide FP32 /
// BF16 / FP8 products are routed to the MFMA kernels in gemm_mfma.hip.
#include "kernels.hpp"

namespace bk {

namespace {

constexpr int NN_BM = 64, NN_BN = 32, NN_BK = 32;

// gpart (nullable, N <= NN_BN): after C is written, the workgroup's partial
// Gram of the C rows it wrote, (C_rows)^T C_rows in FP64 of the stored
// values, at gpart[blockIdx.x N N] (the layout of the TN split partials).
template <typename TA, typename TX, typename TC, typename ACC, bool SCALED>
__global__ __launch_bounds__(256) void nn_kernel(
    int64_t n, int64_t K, int N, const TA* __restrict__ A, int64_t lda,
    const float* __restrict__ ascale, int64_t ascale_ld,
    const TX* __restrict__ X, int64_t ldx, TC* __restrict__ C, int64_t ldc,
    ACC alpha, ACC beta, double* __restrict__ gpart, int64_t kchunk,
    double* __restrict__ split_out) {
  // split s = blockIdx.z takes K range [s kchunk, (s + 1) kchunk); with
  // split_out its raw sums go to split_out[(s n + row) N + col] (no epilogue)
  __shared__ ACC As[NN_BK][NN_BM + 1];
  __shared__ ACC Xs[NN_BK][NN_BN];
  const int t = threadIdx.x;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * NN_BM;
  const int col0 = blockIdx.y * NN_BN;
  const int tx = t & 7;   // 8 groups of 4 output columns
  const int ty = t >> 3;  // 32 groups of 2 output rows
  ACC acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = ACC(0);

  const int64_t kb = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  // the next K chunk is loaded into registers while this one is multiplied
  ACC ar[8], xr[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      const int r = e >> 5, kk = e & 31;
      const int64_t gr = row0 + r, gk = k0 + kk;
      ACC v = ACC(0);
      if (gr < n && gk < ke) {
        v = static_cast<ACC>(Elem<TA>::load(A, gr * lda + gk));
        if (SCALED) v *= static_cast<ACC>(ascale[(gr >> 7) * ascale_ld + (gk >> 7)]);
      }
      ar[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = t + 256 * i;
      const int kk = e >> 5, c = e & 31;
      const int64_t gk = k0 + kk;
      const int gc = col0 + c;
      xr[i] = (gk < ke && gc < N) ? static_cast<ACC>(X[gk * ldx + gc]) : ACC(0);
    }
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += NN_BK) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      As[e & 31][e >> 5] = ar[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = t + 256 * i;
      Xs[e >> 5][e & 31] = xr[i];
    }
    __syncthreads();
    if (k0 + NN_BK < ke) load(k0 + NN_BK);
#pragma unroll 8
    for (int kk = 0; kk < NN_BK; ++kk) {
      const ACC a0 = As[kk][ty * 2], a1 = As[kk][ty * 2 + 1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const ACC xv = Xs[kk][tx * 4 + j];
        acc[0][j] += a0 * xv;
        acc[1][j] += a1 * xv;
      }
    }
    __syncthreads();
  }
  if (split_out) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t gr = row0 + ty * 2 + i;
      if (gr >= n) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gc = col0 + tx * 4 + j;
        if (gc < N)
          split_out[(static_cast<int64_t>(blockIdx.z) * n + gr) * N + gc] =
              static_cast<double>(acc[i][j]);
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t gr = row0 + ty * 2 + i;
    if (gr >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + tx * 4 + j;
      if (gc >= N) continue;
      ACC v = alpha * acc[i][j];
      if (beta != ACC(0)) v += beta * static_cast<ACC>(C[gr * ldc + gc]);
      C[gr * ldc + gc] = static_cast<TC>(v);
      acc[i][j] = static_cast<ACC>(static_cast<TC>(v));  // as stored
    }
  }
  if (gpart) {
    ACC* T = &As[0][0];  // NN_BM x NN_BN tile of the stored rows
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bool rok = row0 + ty * 2 + i < n;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tx * 4 + j;
        T[(ty * 2 + i) * NN_BN + c] = (rok && col0 + c < N) ? acc[i][j] : ACC(0);
      }
    }
    __syncthreads();
    double* g = gpart + static_cast<int64_t>(blockIdx.x) * N * N;
    for (int e = t; e < N * N; e += 256) {
      const int a = e / N, b = e - a * N;
      double sum = 0.0;
#pragma unroll 8
      for (int r = 0; r < NN_BM; ++r)
        sum += static_cast<double>(T[r * NN_BN + a]) * static_cast<double>(T[r * NN_BN + b]);
      g[e] = sum;
    }
  }
}

// C = alpha (sum over the S splits, in split order) + beta C, one thread
// per element.
template <typename TC>
__global__ __launch_bounds__(256) void nn_vsplit_reduce_kernel(int64_t n, int N, int S,
                                                               const double* __restrict__ sp,
                                                               TC* __restrict__ C, int64_t ldc,
                                                               double alpha, double beta) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n * N) return;
  const int64_t r = e / N;
  const int c = static_cast<int>(e - r * N);
  double sum = 0.0;
  for (int z = 0; z < S; ++z) sum += sp[static_cast<int64_t>(z) * n * N + e];
  double v = alpha * sum;
  if (beta != 0.0) v += beta * static_cast<double>(C[r * ldc + c]);
  C[r * ldc + c] = static_cast<TC>(v);
}

// NN for a short reduction (K <= NS_KMAX) and N <= 32 with FP32 A, FP64 X
// and FP32 C (the applies of the orthonormalization): a workgroup's whole
// 64 x K block of A and X (as FP32) are requested at once (clamped, in
// bounds addresses; one round of memory latency instead of one per
// 32-wide chunk), staged in LDS, then multiplied; the epilogue is
// nn_kernel's (alpha, beta, optional Gram partial of the stored rows).
constexpr int NS_KMAX = 256;
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <bool VEC>
__global__ __launch_bounds__(256) void nn_smallk_kernel(
    int64_t n, int K, int N, const float* __restrict__ A, int64_t lda,
    const double* __restrict__ X, int64_t ldx, float* __restrict__ C, int64_t ldc,
    float alpha, float beta, double* __restrict__ gpart) {
  __shared__ float As[NS_KMAX][NN_BM + 1];
  __shared__ float Xs[NS_KMAX][NN_BN];
  __shared__ float Cs[2][16 * 64];
  const int t = threadIdx.x;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * NN_BM;
  const int64_t rlast = n - 1;
  // the beta term of this lane's outputs (see the epilogue: rows
  // 32 (w & 1) + 8 (v >> 2) + 4 (lane >> 5) + (v & 3), column lane & 31),
  // requested with the operands (clamped, in-bounds addresses, loaded
  // unconditionally; the values are used only when beta != 0)
  float cpre[16];
  {
    const int wv = t >> 6, ln = t & 63;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gr = row0 + 32 * (wv & 1) + 8 * (v >> 2) + 4 * (ln >> 5) + (v & 3);
      cpre[v] = C[min(gr, rlast) * ldc + min(ln & 31, N - 1)];
    }
  }
  {
    // A: VEC: 64 x K / 4 float4 (at most 16 per thread); else 64 x K
    // floats (at most 64 per thread)
    constexpr int QA = VEC ? 16 : 64;
    const int RW = VEC ? K / 4 : K;
    const int na = NN_BM * RW;
    using VA = typename std::conditional<VEC, float4, float>::type;
    VA av[QA];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = min(t + 256 * q, na - 1);
      const int r = e / RW, c = e - r * RW;
      const int64_t gr = min(row0 + r, rlast);
      if constexpr (VEC)
        av[q] = *reinterpret_cast<const float4*>(A + gr * lda + 4 * c);
      else
        av[q] = A[gr * lda + c];
    }
    // X: K x 32 (columns past N are zero), at most 32 per thread
    double xv[32];
    const int nx = K * NN_BN;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int e = min(t + 256 * q, nx - 1);
      const int kk = e >> 5, c = e & 31;
      xv[q] = X[static_cast<int64_t>(kk) * ldx + min(c, N - 1)];
    }
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = t + 256 * q;
      if (e < na) {
        const int r = e / RW, c = e - r * RW;
        const bool ok = row0 + r < n;
        if constexpr (VEC) {
          As[4 * c + 0][r] = ok ? av[q].x : 0.f;
          As[4 * c + 1][r] = ok ? av[q].y : 0.f;
          As[4 * c + 2][r] = ok ? av[q].z : 0.f;
          As[4 * c + 3][r] = ok ? av[q].w : 0.f;
        } else {
          As[c][r] = ok ? av[q] : 0.f;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int e = t + 256 * q;
      if (e < nx) Xs[e >> 5][e & 31] = (e & 31) < N ? static_cast<float>(xv[q]) : 0.f;
    }
  }
  // the reduction padded with zero rows to KP, a multiple of 16 (<= NS_KMAX),
  // so that each wavefront's share is a whole number of 4-step groups
  const int KP = (K + 15) & ~15;
  for (int i = t; i < (KP - K) * (NN_BM + 1); i += 256) As[K + i / (NN_BM + 1)][i % (NN_BM + 1)] = 0.f;
  for (int i = t; i < (KP - K) * NN_BN; i += 256) Xs[K + i / NN_BN][i % NN_BN] = 0.f;
  __syncthreads();
  // matrix cores: wavefront w takes the 32-row half w & 1 of the block and
  // the half w >> 1 of the reduction pairs; 32 x 32 x 2 FP32 steps, lane
  // (rh, cl) supplying A[32 rt + cl][kk] and X[kk][cl], kk = 2 pair + rh
  const int w = t >> 6, lane = t & 63, rh = lane >> 5, cl = lane & 31;
  const int rt = w & 1, kh = w >> 1;
  const int hp = KP >> 2;  // pairs per wavefront (a multiple of 4)
  const int p_lo = kh * hp, p_hi = p_lo + hp;
  f32x16_t c32;
#pragma unroll
  for (int v = 0; v < 16; ++v) c32[v] = 0.f;
  const float* pa = &As[0][0] + 32 * rt + cl;
  const float* pb = &Xs[0][0] + cl;
  for (int pp = p_lo; pp < p_hi; pp += 4) {
    float a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = 2 * (pp + u) + rh;
      a[u] = pa[kk * (NN_BM + 1)];
      b[u] = pb[kk * NN_BN];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], c32, 0, 0, 0);
  }
  // the second reduction half added to the first, in that order
  if (kh == 1)
#pragma unroll
    for (int v = 0; v < 16; ++v) Cs[rt][v * 64 + lane] = c32[v];
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      c32[v] += Cs[rt][v * 64 + lane];
      const int64_t gr = row0 + 32 * rt + 8 * (v >> 2) + 4 * rh + (v & 3);
      float val = alpha * c32[v];
      if (beta != 0.f) val += beta * cpre[v];
      if (gr < n && cl < N) C[gr * ldc + cl] = val;
      c32[v] = val;  // as stored
    }
  }
  if (gpart) {
    float* T = &As[0][0];  // NN_BM x NN_BN tile of the stored rows
    if (kh == 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * rt + 8 * (v >> 2) + 4 * rh + (v & 3);
        T[row * NN_BN + cl] = (row0 + row < n && cl < N) ? c32[v] : 0.f;
      }
    }
    __syncthreads();
    double* g = gpart + static_cast<int64_t>(blockIdx.x) * N * N;
    for (int e = t; e < N * N; e += 256) {
      const int a = e / N, b = e - a * N;
      double sum = 0.0;
#pragma unroll 8
      for (int r = 0; r < NN_BM; ++r)
        sum += static_cast<double>(T[r * NN_BN + a]) * static_cast<double>(T[r * NN_BN + b]);
      g[e] = sum;
    }
  }
}

constexpr int TN_BP = 64, TN_BR = 32, TN_BL = 32;

// Partial sums over the rows [s*Ls, (s+1)*Ls) of split s = blockIdx.z:
// FP32 (or FP64) products summed over 32-row chunks, chunk sums added in FP64.
template <typename TX, typename TY, typename ACC, bool SCALED>
__global__ __launch_bounds__(256) void tn_kernel(
    int64_t L, int64_t p, int r, const TX* __restrict__ X, int64_t ldx,
    const float* __restrict__ xscale, int64_t xscale_ld,
    const TY* __restrict__ Y, int64_t ldy, double* __restrict__ partial,
    int64_t Ls, int sym) {
  __shared__ ACC Xs[TN_BL][TN_BP];
  __shared__ ACC Ys[TN_BL][TN_BR];
  const int t = threadIdx.x;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * TN_BP;
  const int r0 = blockIdx.y * TN_BR;
  if (sym && p0 > r0 + TN_BR - 1) return;  // below the diagonal: mirrored
  const int64_t s = blockIdx.z;
  const int64_t lb = s * Ls;
  const int64_t le = (lb + Ls < L) ? lb + Ls : L;
  const int tp = t >> 3;  // 32 groups of 2 p-rows
  const int tr = t & 7;   // 8 groups of 4 r-columns
  double dacc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) dacc[i][j] = 0.0;

  // the next chunk is loaded into registers while this one is multiplied
  ACC xr[8], yr[4];
  auto load = [&](int64_t l0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      const int ll = e >> 6, pp = e & 63;
      const int64_t gl = l0 + ll, gp = p0 + pp;
      ACC v = ACC(0);
      if (gl < le && gp < p) {
        v = static_cast<ACC>(Elem<TX>::load(X, gl * ldx + gp));
        if (SCALED) v *= static_cast<ACC>(xscale[(gl >> 7) * xscale_ld + (gp >> 7)]);
      }
      xr[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = t + 256 * i;
      const int ll = e >> 5, rr = e & 31;
      const int64_t gl = l0 + ll;
      const int gr = r0 + rr;
      yr[i] = (gl < le && gr < r) ? static_cast<ACC>(Y[gl * ldy + gr]) : ACC(0);
    }
  };
  if (lb < le) load(lb);
  for (int64_t l0 = lb; l0 < le; l0 += TN_BL) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      Xs[e >> 6][e & 63] = xr[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = t + 256 * i;
      Ys[e >> 5][e & 31] = yr[i];
    }
    __syncthreads();
    if (l0 + TN_BL < le) load(l0 + TN_BL);
    ACC acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = ACC(0);
#pragma unroll 8
    for (int ll = 0; ll < TN_BL; ++ll) {
      const ACC x0 = Xs[ll][tp * 2], x1 = Xs[ll][tp * 2 + 1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const ACC yv = Ys[ll][tr * 4 + j];
        acc[0][j] += x0 * yv;
        acc[1][j] += x1 * yv;
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) dacc[i][j] += static_cast<double>(acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t gp = p0 + tp * 2 + i;
    if (gp >= p) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = r0 + tr * 4 + j;
      if (gr >= r) continue;
      partial[(s * p + gp) * r + gr] = dacc[i][j];
    }
  }
}

// sym: X = Y, only partials on or above the diagonal exist; (gp, gr) below
// it takes the sums of (gr, gp), so C is exactly symmetric.
template <typename TC>
__global__ __launch_bounds__(256) void tn_reduce_kernel(
    int S, int64_t p, int r, const double* __restrict__ partial,
    TC* __restrict__ C, int64_t ldc, double alpha, double beta, int sym) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= p * r) return;
  const int64_t gp = idx / r;
  const int gr = static_cast<int>(idx - gp * r);
  const int64_t src = (sym && gp > gr) ? static_cast<int64_t>(gr) * r + gp : gp * r + gr;
  double acc = 0.0;
  for (int i = 0; i < S; ++i) acc += partial[i * p * r + src];
  double v = alpha * acc;
  if (beta != 0.0) v += beta * static_cast<double>(C[gp * ldc + gr]);
  C[gp * ldc + gr] = static_cast<TC>(v);
}

// Same reduction with one wavefront per output: lane l adds partials
// l, l+64, ... in order, then a fixed butterfly combines the lanes.
template <typename TC>
__global__ __launch_bounds__(256) void tn_reduce_wave_kernel(
    int S, int64_t p, int r, const double* __restrict__ partial,
    TC* __restrict__ C, int64_t ldc, double alpha, double beta, int sym) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (idx >= p * r) return;
  const int lane = threadIdx.x & 63;
  const int64_t gp = idx / r;
  const int gr = static_cast<int>(idx - gp * r);
  const int64_t src = (sym && gp > gr) ? static_cast<int64_t>(gr) * r + gp : gp * r + gr;
  double acc = 0.0;
  for (int i = lane; i < S; i += 64) acc += partial[i * p * r + src];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) {
    double v = alpha * acc;
    if (beta != 0.0) v += beta * static_cast<double>(C[gp * ldc + gr]);
    C[gp * ldc + gr] = static_cast<TC>(v);
  }
}

// Splits of K for the vector NN when its tiles leave most of the chip idle
// (~256 workgroups, at least four 32-wide chunks per split).
int nn_vec_splits(int64_t n, int64_t K, int N) {
  const int64_t tiles = cdiv(n, NN_BM) * cdiv(N, NN_BN);
  if (tiles >= 128 || K < 8 * NN_BK) return 1;
  int64_t S = cdiv(256, tiles);
  const int64_t smax = cdiv(K, 4 * NN_BK);
  if (S > smax) S = smax;
  return static_cast<int>(S < 1 ? 1 : S);
}

template <typename TA, typename TX, typename TC, typename ACC>
int nn_dispatch_scaled(const NNArgs& a, hipStream_t s) {
  const int64_t tiles = cdiv(a.n, NN_BM) * cdiv(a.N, NN_BN);
  const int S = a.gram_partial ? 1 : nn_vec_splits(a.n, a.K, a.N);
  const bool split = S > 1 && a.split_work &&
                     static_cast<int64_t>(S) * a.n * a.N <= a.split_work_elems;
  const int64_t kchunk = split ? cdiv(cdiv(a.K, S), NN_BK) * NN_BK : (a.K > 0 ? a.K : 1);
  const int Sx = split ? static_cast<int>(cdiv(a.K, kchunk)) : 1;
  const dim3 grid(static_cast<unsigned>(cdiv(a.n, NN_BM)),
                  static_cast<unsigned>(cdiv(a.N, NN_BN)), static_cast<unsigned>(Sx));
  (void)tiles;
  const TA* A = static_cast<const TA*>(a.A);
  const TX* X = static_cast<const TX*>(a.X);
  TC* C = static_cast<TC*>(a.C);
  double* so = split ? a.split_work : nullptr;
  if (a.ascale)
    nn_kernel<TA, TX, TC, ACC, true><<<grid, 256, 0, s>>>(
        a.n, a.K, a.N, A, a.lda, a.ascale, a.ascale_ld, X, a.ldx, C, a.ldc,
        static_cast<ACC>(a.alpha), static_cast<ACC>(a.beta), a.gram_partial, kchunk, so);
  else
    nn_kernel<TA, TX, TC, ACC, false><<<grid, 256, 0, s>>>(
        a.n, a.K, a.N, A, a.lda, nullptr, 0, X, a.ldx, C, a.ldc,
        static_cast<ACC>(a.alpha), static_cast<ACC>(a.beta), a.gram_partial, kchunk, so);
  if (!split) return 1;
  nn_vsplit_reduce_kernel<TC><<<static_cast<unsigned>(cdiv(a.n * a.N, 256)), 256, 0, s>>>(
      a.n, a.N, Sx, so, C, a.ldc, a.alpha, a.beta);
  return 2;
}

template <typename TA>
int nn_dispatch_lowp(const NNArgs& a, hipStream_t s) {
  // FP32-accumulating paths: X FP64 or FP32, C FP32 (or FP64)
  if (a.x_f64) {
    if (a.c_f64) return nn_dispatch_scaled<TA, double, double, float>(a, s);
    return nn_dispatch_scaled<TA, double, float, float>(a, s);
  }
  if (a.c_f64) return nn_dispatch_scaled<TA, float, double, float>(a, s);
  return nn_dispatch_scaled<TA, float, float, float>(a, s);
}

template <typename TX, typename ACC>
void tn_dispatch(const TNArgs& a, int S, int64_t Ls, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(cdiv(a.p, TN_BP)),
                  static_cast<unsigned>(cdiv(a.r, TN_BR)),
                  static_cast<unsigned>(S));
  const TX* X = static_cast<const TX*>(a.X);
  if (a.y_f64) {
    const double* Y = static_cast<const double*>(a.Y);
    if (a.xscale)
      tn_kernel<TX, double, ACC, true><<<grid, 256, 0, s>>>(
          a.L, a.p, a.r, X, a.ldx, a.xscale, a.xscale_ld, Y, a.ldy, a.partial, Ls, a.sym ? 1 : 0);
    else
      tn_kernel<TX, double, ACC, false><<<grid, 256, 0, s>>>(
          a.L, a.p, a.r, X, a.ldx, nullptr, 0, Y, a.ldy, a.partial, Ls, a.sym ? 1 : 0);
  } else {
    const float* Y = static_cast<const float*>(a.Y);
    if (a.xscale)
      tn_kernel<TX, float, ACC, true><<<grid, 256, 0, s>>>(
          a.L, a.p, a.r, X, a.ldx, a.xscale, a.xscale_ld, Y, a.ldy, a.partial, Ls, a.sym ? 1 : 0);
    else
      tn_kernel<TX, float, ACC, false><<<grid, 256, 0, s>>>(
          a.L, a.p, a.r, X, a.ldx, nullptr, 0, Y, a.ldy, a.partial, Ls, a.sym ? 1 : 0);
  }
}

}  // namespace

int64_t nn_gram_partial_elems(int64_t n, int N) {
  return N <= NN_BN ? cdiv(n, NN_BM) * N * N : 0;
}

int launch_gram_reduce(int64_t n, int N, const double* gpart, double* G, hipStream_t s) {
  const int S = static_cast<int>(cdiv(n, NN_BM));
  const int64_t outs = static_cast<int64_t>(N) * N;
  if (S >= 16 && outs <= (int64_t(1) << 16))
    tn_reduce_wave_kernel<double><<<static_cast<unsigned>(cdiv(outs, 4)), 256, 0, s>>>(
        S, N, N, gpart, G, N, 1.0, 0.0, 0);
  else
    tn_reduce_kernel<double><<<static_cast<unsigned>(cdiv(outs, 256)), 256, 0, s>>>(
        S, N, N, gpart, G, N, 1.0, 0.0, 0);
  return 1;
}

int launch_nn(const NNArgs& a, hipStream_t s) {
  if (a.n <= 0 || a.N <= 0) return 0;  // K = 0 gives C = beta C below
  if (a.gram_partial && a.N > NN_BN) return 0;
  int mfma = 0;
  if (!a.gram_partial) launch_nn_mfma_if(a, s, &mfma);
  if (mfma) return mfma;
  if (a.a_type == BK_F32 && !a.ascale && a.x_f64 && !a.c_f64 && a.N <= NN_BN && a.K > 0 &&
      a.K <= NS_KMAX) {
    const bool vec = a.K % 4 == 0 && a.lda % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(a.A) % 16 == 0;
    const unsigned g = static_cast<unsigned>(cdiv(a.n, NN_BM));
    const int K = static_cast<int>(a.K);
    const float* A = static_cast<const float*>(a.A);
    const double* X = static_cast<const double*>(a.X);
    float* C = static_cast<float*>(a.C);
    const float al = static_cast<float>(a.alpha), be = static_cast<float>(a.beta);
    if (vec)
      nn_smallk_kernel<true><<<g, 256, 0, s>>>(a.n, K, a.N, A, a.lda, X, a.ldx, C, a.ldc, al,
                                               be, a.gram_partial);
    else
      nn_smallk_kernel<false><<<g, 256, 0, s>>>(a.n, K, a.N, A, a.lda, X, a.ldx, C, a.ldc, al,
                                                be, a.gram_partial);
    return 1;
  }
  switch (a.a_type) {
    case BK_F64:
      return nn_dispatch_scaled<double, double, double, double>(a, s);
    case BK_F32:
      return nn_dispatch_lowp<float>(a, s);
    case BK_BF16:
      return nn_dispatch_lowp<bf16_t>(a, s);
    case BK_FP8_E4M3:
      return nn_dispatch_lowp<fp8_t>(a, s);
    default:
      return 0;
  }
}

int tn_splits(int64_t L, int64_t p, int r) {
  const int64_t tiles = cdiv(p, TN_BP) * cdiv(r, TN_BR);
  int64_t S = cdiv(2048, tiles);
  const int64_t smax = cdiv(L, 64);
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  if (S > 4096) S = 4096;
  // each split a whole number of 32-row chunks
  int64_t Ls = align_up(static_cast<size_t>(cdiv(L, S)), TN_BL);
  S = cdiv(L, Ls);
  return static_cast<int>(S < 1 ? 1 : S);
}

int64_t tn_partial_elems(int64_t L, int64_t p, int r) {
  const int S = std::max(tn_splits(L, p, r), tn_mfma_splits(L, p, r));
  return static_cast<int64_t>(S) * p * r;
}

int launch_tn(const TNArgs& a, hipStream_t s) {
  if (a.p <= 0 || a.r <= 0) return 0;
  int S = 0;
  launch_tn_mfma_if(a, s, &S);
  const bool mfma = S > 0;
  if (!mfma) S = a.L > 0 ? tn_splits(a.L, a.p, a.r) : 1;
  int64_t Ls = a.L > 0 ? static_cast<int64_t>(align_up(cdiv(a.L, S), TN_BL)) : 0;
  if (mfma) {
    // partials written by the matrix-core kernel
  } else if (a.L <= 0) {
    launch_fill_f64(a.partial, a.p * a.r, 0.0, s);
  } else {
    switch (a.x_type) {
      case BK_F64:
        tn_dispatch<double, double>(a, S, Ls, s);
        break;
      case BK_F32:
        tn_dispatch<float, float>(a, S, Ls, s);
        break;
      case BK_BF16:
        tn_dispatch<bf16_t, float>(a, S, Ls, s);
        break;
      case BK_FP8_E4M3:
        tn_dispatch<fp8_t, float>(a, S, Ls, s);
        break;
      default:
        return 0;
    }
  }
  // kernels before the reduction: fill, VALU split kernel, or pack + MFMA
  const int before = mfma ? (a.x_type == BK_F32 ? 1 : 2) : 1;
  const int sym = (a.sym && a.L > 0) ? 1 : 0;
  const int64_t outs = a.p * a.r;
  if (S >= 16 && outs <= (int64_t(1) << 16)) {
    const unsigned g = static_cast<unsigned>(cdiv(outs, 4));
    if (a.c_f64)
      tn_reduce_wave_kernel<double><<<g, 256, 0, s>>>(S, a.p, a.r, a.partial,
                                                      static_cast<double*>(a.C), a.ldc,
                                                      a.alpha, a.beta, sym);
    else
      tn_reduce_wave_kernel<float><<<g, 256, 0, s>>>(S, a.p, a.r, a.partial,
                                                     static_cast<float*>(a.C), a.ldc,
                                                     a.alpha, a.beta, sym);
    return before + 1;
  }
  const unsigned g = static_cast<unsigned>(cdiv(outs, 256));
  if (a.c_f64)
    tn_reduce_kernel<double><<<g, 256, 0, s>>>(S, a.p, a.r, a.partial,
                                               static_cast<double*>(a.C), a.ldc,
                                               a.alpha, a.beta, sym);
  else
    tn_reduce_kernel<float><<<g, 256, 0, s>>>(S, a.p, a.r, a.partial,
                                              static_cast<float*>(a.C), a.ldc,
                                              a.alpha, a.beta, sym);
  return before + 1;
}

}  // namespace bk
