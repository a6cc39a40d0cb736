// Matrix-core (MFMA) forms of the dense block products of the Krylov loop
// (Algorithm 2, steps 2-6) and of the wide reductions around them:
//   NN:  C (n x N, FP32) = A X,   A n x K row-major in FP32 / BF16 / FP8 e4m3
//   TN:  partial_s (p x r, FP64) = sum over rows of split s of X^T Y,
//        X L x p row-major in FP32 / BF16 / FP8, Y L x r
// Element types and instructions (lane layouts checked on gfx950):
//   FP32  v_mfma_f32_32x32x2_f32        1 value per lane and step
//   BF16  v_mfma_f32_32x32x16_bf16      8 values per lane and step
//   FP8   v_mfma_scale_f32_32x32x64_f8f6f4  32 values (OCP e4m3) per lane and
//         step, block scales at 1
// The reduction dimension is walked in chunks of 128 bytes per row (32 FP32,
// 64 BF16 or 128 FP8 values; for FP8 one chunk is one 128-wide scale tile).
// Inside a chunk, lanes 0-31 supply bytes 0-63 and lanes 32-63 bytes
// 64-127 of their row; A and B operands use the same assignment, so each
// chunk is summed exactly once.  Partial sums of a chunk are formed in FP32
// and, for FP8, multiplied by the product of the two operand scales before
// they are added to the running sum.  The TN running sum is FP64 (as the
// VALU kernels do over 32-row chunks).
#include "kernels.hpp"

namespace bk {
namespace {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;

constexpr int LDS_ROW = 36;  // 32-bit words per staged row: 128 bytes + 16 pad
// Buffer descriptor word 3 of a raw (unswizzled, 32-bit data format) buffer.
constexpr int kBufferFlags = 0x00020000;

template <typename T>
struct Mf;
template <>
struct Mf<float> {
  static constexpr int KC = 32;     // values per 128-byte chunk
  static constexpr int STEPS = 16;  // MFMA steps per chunk
  static constexpr int LW = 1;      // 32-bit words per lane and step
};
template <>
struct Mf<bf16_t> {
  static constexpr int KC = 64;
  static constexpr int STEPS = 4;
  static constexpr int LW = 4;
};
template <>
struct Mf<fp8_t> {
  static constexpr int KC = 128;
  static constexpr int STEPS = 2;
  static constexpr int LW = 8;
};

template <typename T>
__device__ __forceinline__ f32x16 mfma_step(const uint32_t* a, const uint32_t* b, f32x16 c);
template <>
__device__ __forceinline__ f32x16 mfma_step<float>(const uint32_t* a, const uint32_t* b,
                                                   f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[0]), __uint_as_float(b[0]), c,
                                              0, 0, 0);
}
template <>
__device__ __forceinline__ f32x16 mfma_step<bf16_t>(const uint32_t* a, const uint32_t* b,
                                                    f32x16 c) {
  const uint4 ua = make_uint4(a[0], a[1], a[2], a[3]);
  const uint4 ub = make_uint4(b[0], b[1], b[2], b[3]);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ua),
                                                 __builtin_bit_cast(bf16x8, ub), c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f32x16 mfma_step<fp8_t>(const uint32_t* a, const uint32_t* b,
                                                   f32x16 c) {
  // gfx950's 32 x 32 x 64 FP8 step (both operands OCP e4m3, format 0), with
  // the block scales at 2^0 (E8M0 127): the FP32 tile scales are applied
  // to the chunk sums instead
  i32x8 va, vb;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    va[i] = static_cast<int>(a[i]);
    vb[i] = static_cast<int>(b[i]);
  }
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, c, 0, 0, 0, 127, 0, 127);
}

// LDS words of the lane's operand for step q: row `row` of a staged tile.
template <typename T>
__device__ __forceinline__ void lds_operand(const uint32_t* tile, int row, int h, int q,
                                            uint32_t* out) {
  const uint32_t* p = tile + row * LDS_ROW + 16 * h + q * Mf<T>::LW;
  if constexpr (Mf<T>::LW == 8) {
    const uint4 v0 = *reinterpret_cast<const uint4*>(p);
    const uint4 v1 = *reinterpret_cast<const uint4*>(p + 4);
    out[0] = v0.x;
    out[1] = v0.y;
    out[2] = v0.z;
    out[3] = v0.w;
    out[4] = v1.x;
    out[5] = v1.y;
    out[6] = v1.z;
    out[7] = v1.w;
  } else if constexpr (Mf<T>::LW == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else if constexpr (Mf<T>::LW == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    out[0] = v.x;
    out[1] = v.y;
  } else {
    out[0] = p[0];
  }
}

// Workgroups go to the eight XCDs in turn (id mod 8).  The column blocks
// of one row block read the same rows of A, so they get ids on the same
// XCD, one after another (its L2 then serves the second read):
// id = 8 (rb_local * ncb + cb) + rb mod 8 with rb_local = rb / 8.  One
// column block gives id = rb.  Ids past the last row block do nothing.
__device__ __forceinline__ bool xcd_tile(int64_t id, int64_t nrb, int64_t ncb, int64_t* rb,
                                         int64_t* cb) {
  const int64_t xcd = id & 7, slot = id >> 3;
  *rb = (slot / ncb) * 8 + xcd;
  *cb = slot % ncb;
  return *rb < nrb;
}
inline int64_t xcd_grid(int64_t nrb, int64_t ncb) { return ((nrb + 7) / 8) * 8 * ncb; }

// Output element (row, col) of a 32 x 32 tile held by lane `lane` in
// accumulator register v.
__device__ __forceinline__ int out_row(int lane, int v) {
  return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

// ------------------------------------------------------------------ NN --
// Workgroup: 128 rows of C x 128 columns (4 wavefronts of 32 rows); the
// rows of A go straight from memory into the operand registers (the next
// chunk in flight while the current one is multiplied), the packed X^T
// chunk (128 columns x 128 bytes) is staged in LDS, double-buffered.
// WN = 2 (N > 128, BF16 / FP8): 512 threads, 256 columns of C, wavefront
// (w, cw) with cw = t / 256 taking columns 128 cw ..: every row of A is then
// fetched from memory once (with two 128-column workgroups per row block
// the second fetch only partly hits L2: 6.1 GB read per FP8 A^T.Y of 4.3 GB).
template <typename T, bool SCALED, int PD, int NT, int WN>
__global__ __launch_bounds__(256 * WN, WN == 1 ? 2 : 1) void nn_mfma_kernel(
    int64_t n, int64_t K, int N, const T* __restrict__ A, int64_t lda,
    const float* __restrict__ ascale, int64_t ascale_ld, const T* __restrict__ Xt,
    int64_t ldxt, const float* __restrict__ xscale, float* __restrict__ C, int64_t ldc,
    int64_t cps, float alpha, float beta) {
  constexpr int KC = Mf<T>::KC, STEPS = Mf<T>::STEPS, LW = Mf<T>::LW;
  constexpr int CB = 128 * WN;  // columns of C per workgroup
  __shared__ uint32_t Bs[2][CB * LDS_ROW];
  const int t = threadIdx.x, lane = t & 63, w = (t >> 6) & 3, h = lane >> 5, r32 = lane & 31;
  const int cw = t >> 8;
  int64_t rb, cb;
  if (!xcd_tile(blockIdx.x, (n + 127) / 128, (N + CB - 1) / CB, &rb, &cb)) return;
  // split blockIdx.y takes chunks [c0, c0 + nch) of K; with several splits
  // C is its n x N (ld N) slice of FP32 partials
  const int64_t nall = K / KC;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * cps;
  if (c0 >= nall) return;
  const int64_t nch = (c0 + cps < nall) ? cps : nall - c0;
  if (gridDim.y > 1) {
    C += static_cast<int64_t>(blockIdx.y) * n * N;
    ldc = N;
  }
  const int64_t row0 = rb * 128;
  const int64_t col0 = cb * CB + 128 * cw;  // the wavefront's first column
  // NT output tiles of 32 columns (compile time: no branch between the
  // matrix-core steps); tiles past the valid columns multiply what is
  // staged for them and are not stored
  const int64_t vtb = (N - cb * CB + 31) / 32;
  const int ntb = static_cast<int>(vtb < NT * WN ? vtb : NT * WN);  // the workgroup's
  const int64_t row = row0 + 32 * w + r32;
  const uint4* arow =
      reinterpret_cast<const uint4*>(A + (row < n ? row : n - 1) * lda) + 4 * h + c0 * 8;
  const int bc = t >> 1, bh = t & 1;  // staging: packed column bc, half bh
  const bool bload = bc < 32 * ntb;
  const uint4* xrow =
      reinterpret_cast<const uint4*>(Xt + (cb * CB + (bload ? bc : 0)) * ldxt) + 4 * bh + c0 * 8;
  f32x16 acc[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) acc[tt] = f32x16{};
  // A chunks in a ring of R = PD + 1 register sets, PD chunks in flight
  // ahead of the one multiplied (a chunk of BF16 / FP8 is a few hundred
  // cycles of matrix-core work, far below one memory latency); the packed
  // X^T chunk goes through LDS one chunk ahead; FP8 chunk scales travel with
  // the A chunks.  No load is conditional and no branch separates the
  // chunks (either would make the wait-count pass assume the prefetches
  // unfinished): chunks go in rounds of R, and a chunk past the split's
  // last re-reads the last one and is not multiplied.
  constexpr int R = PD + 1;
  uint4 abuf[R][4], bst[4];
  float scr[R];
  auto aload = [&](int slot, int64_t c) {
    const int64_t cc = c < nch ? c : nch - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) abuf[slot][i] = arow[cc * 8 + i];
    if (SCALED) {
      // 32-row groups never straddle a 128-row scale tile; chunk c is
      // scale column c0 + c
      scr[slot] = ascale[((row0 + 32 * w) >> 7) * ascale_ld + c0 + cc] * xscale[c0 + cc];
    }
  };
  auto bload_ = [&](int64_t c) {
    const int64_t cc = c < nch ? c : nch - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) bst[i] = xrow[cc * 8 + i];
  };
  // (no masking: a chunk past the split's last is never multiplied, and a
  // column past the valid ones, which holds column 0's values, only feeds
  // output columns that are not stored)
  auto bstore = [&](int buf, int64_t c) {
    (void)c;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<uint4*>(&Bs[buf][bc * LDS_ROW + 16 * bh + 4 * i]) =
          make_uint4(bst[i].x, bst[i].y, bst[i].z, bst[i].w);
  };
#pragma unroll
  for (int u = 0; u < PD; ++u) aload(u, u);
  bload_(0);
  bstore(0, 0);
  __syncthreads();
  for (int64_t cb0 = 0; cb0 < nch; cb0 += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t c = cb0 + u;
      // X^T first: the wait before its store then leaves the A chunks in
      // flight (the wait counter drains in issue order)
      bload_(c + 1);
      aload((u + PD) % R, c + PD);
      __builtin_amdgcn_sched_barrier(0);
      if (c < nch) {  // (uniform; no memory operation inside)
      uint32_t aw[16];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        aw[4 * i] = abuf[u][i].x;
        aw[4 * i + 1] = abuf[u][i].y;
        aw[4 * i + 2] = abuf[u][i].z;
        aw[4 * i + 3] = abuf[u][i].w;
      }
      const uint32_t* tile = Bs[c & 1];
      f32x16 tmp[4];
      if (SCALED) {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) tmp[tt] = f32x16{};
      }
#pragma unroll
      for (int q = 0; q < STEPS; ++q) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          uint32_t bw[LW];
          lds_operand<T>(tile, 128 * cw + 32 * tt + r32, h, q, bw);
          if (SCALED) tmp[tt] = mfma_step<T>(aw + q * LW, bw, tmp[tt]);
          else acc[tt] = mfma_step<T>(aw + q * LW, bw, acc[tt]);
        }
      }
      if (SCALED) {
        const float sc = scr[u];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] += sc * tmp[tt];
      }
      }
      __builtin_amdgcn_sched_barrier(0);
      bstore((c + 1) & 1, c + 1);
      __syncthreads();
    }
  }
  // C = alpha acc + beta C (a split's partial: alpha 1, beta 0)
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const int64_t gc = col0 + 32 * tt + r32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gr = row0 + 32 * w + out_row(lane, v);
      if (gr < n && gc < N) {
        float* c = C + gr * ldc + gc;
        *c = beta != 0.0f ? alpha * acc[tt][v] + beta * *c : alpha * acc[tt][v];
      }
    }
  }
}

// ---------------------------------------------------- FP32 as BF16 limbs --
// An FP32 value a splits exactly into three BF16 limbs a = a1 + a2 + a3
// (a1 = RNE_bf16(a), a2 = RNE_bf16(a - a1), a3 = a - a1 - a2: each
// difference is exact in FP32 and the last one has at most 8 significant
// bits).  A product a b is then the sum of nine limb products; the six with
// limb orders adding up to at most 4 are kept (a1 b1, a1 b2, a2 b1, a1 b3,
// a2 b2, a3 b1), the dropped three are below 2^-23 |a b| together, and the
// BF16 matrix-core step multiplies limbs exactly and sums in FP32.  Six
// 32 x 32 x 16 BF16 steps (32 cycles each) replace eight 32 x 32 x 2 FP32
// steps (64 cycles each) for 16 values of the reduction.  Finite inputs
// below the BF16 overflow threshold (about 3.39e38) only.
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
// two FP32 values rounded to BF16 (RNE) in one register, low half first
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
// Limbs of 8 values, two at a time in packed registers (no element moves):
// the BF16 halves widen back to FP32 by a shift or a mask.
__device__ __forceinline__ void split3(const float* x, bf16x8& l1, bf16x8& l2, bf16x8& l3) {
  uint32_t w1[4], w2[4], w3[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float a = x[2 * q], b = x[2 * q + 1];
    const uint32_t p1 = bf16_pair(a, b);
    const float ra = a - __uint_as_float(p1 << 16), rb = b - __uint_as_float(p1 & 0xFFFF0000u);
    const uint32_t p2 = bf16_pair(ra, rb);
    const float sa = ra - __uint_as_float(p2 << 16), sb = rb - __uint_as_float(p2 & 0xFFFF0000u);
    w1[q] = p1;
    w2[q] = p2;
    w3[q] = bf16_pair(sa, sb);
  }
  l1 = __builtin_bit_cast(bf16x8, make_uint4(w1[0], w1[1], w1[2], w1[3]));
  l2 = __builtin_bit_cast(bf16x8, make_uint4(w2[0], w2[1], w2[2], w2[3]));
  l3 = __builtin_bit_cast(bf16x8, make_uint4(w3[0], w3[1], w3[2], w3[3]));
}


// Words per staged column of one limb: 32 BF16 (one 32-value chunk) + 16
// bytes of padding, so that the 8 lanes of a 16-byte LDS read pass hit
// distinct banks.
constexpr int X3_COL = 20;
// Rows per split of the limb X^T Y kernel, whose sums over a split are FP32
// (the A X kernel sums 32768 values in FP32 likewise).
constexpr int64_t kX3SplitRows = 16384;

// FP32 A X (A n x K row-major, X^T packed as three BF16 limb planes, see
// pack_t_x3): workgroup 128 rows x 128 columns of C as in nn_mfma_kernel;
// the rows of A go from memory into registers (the next chunk in flight)
// and are split into limbs there, the X^T limbs of a chunk go through LDS.
// Chunks of 32 values: two steps of 16.
template <int NT, int WN>
__global__ __launch_bounds__(256 * WN) void nn_x3_kernel(
    int64_t n, int64_t K, int N, const float* __restrict__ A, int64_t lda,
    const bf16_t* __restrict__ Xt, int64_t ldxt, int64_t plane, float* __restrict__ C,
    int64_t ldc, int64_t cps, float alpha, float beta) {
  constexpr int CB = 128 * WN;  // columns of C per workgroup
  __shared__ uint32_t Bs[2][3][CB * X3_COL];
  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, r32 = lane & 31;
  // wavefront (w, cw): rows 32 w .. 32 w + 31 x columns 128 cw .. 128 cw +
  // 127 of the block; the WN wavefronts of one row group load the same rows
  // of A at the same time (served once from memory)
  const int w = (t >> 6) & 3, cw = t >> 8;
  int64_t rb, cb;
  if (!xcd_tile(blockIdx.x, (n + 127) / 128, (N + CB - 1) / CB, &rb, &cb)) return;
  const int64_t nall = K / 32;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * cps;
  if (c0 >= nall) return;
  const int64_t nch = (c0 + cps < nall) ? cps : nall - c0;
  if (gridDim.y > 1) {
    C += static_cast<int64_t>(blockIdx.y) * n * N;
    ldc = N;
  }
  const int64_t row0 = rb * 128;
  const int64_t colb = cb * CB;              // the block's first column
  const int64_t col0 = colb + 128 * cw;      // the wavefront's first column
  const int ntb = static_cast<int>((N - colb + 31) / 32 < NT * WN ? (N - colb + 31) / 32
                                                                   : NT * WN);
  const int64_t row = row0 + 32 * w + r32;
  // lane (i, h) holds values 8 h .. 8 h + 7 of each 16-value step
  const uint4* arow =
      reinterpret_cast<const uint4*>(A + (row < n ? row : n - 1) * lda) + 2 * h + c0 * 8;
  const int bc = t >> 1, bh = t & 1;  // staging: packed column bc, half bh
  const bool bload = bc < 32 * ntb;
  const uint4* xrow =
      reinterpret_cast<const uint4*>(Xt + (colb + (bload ? bc : 0)) * ldxt) + 2 * bh + c0 * 4;
  const int64_t pl4 = plane / 8;  // limb plane stride in uint4
  f32x16 acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = f32x16{};
  // A: chunks c+1 and c+2 in flight while chunk c is multiplied (slots mod
  // 3); X^T limbs of chunk c+1 staged after it.  Unconditional loads (a
  // chunk past the split's last re-reads the last one; its X^T is staged as
  // zeros and its steps are skipped).
  uint4 abuf[3][4], bst[2][3][2];
  auto aload = [&](int slot, int64_t c) {
    const int64_t cc = c < nch ? c : nch - 1;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      abuf[slot][2 * s2] = arow[cc * 8 + 4 * s2];
      abuf[slot][2 * s2 + 1] = arow[cc * 8 + 4 * s2 + 1];
    }
  };
  auto bload_ = [&](int slot, int64_t c) {
    const int64_t cc = c < nch ? c : nch - 1;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      bst[slot][l][0] = xrow[l * pl4 + cc * 4];
      bst[slot][l][1] = xrow[l * pl4 + cc * 4 + 1];
    }
  };
  // (no masking: a chunk past the end is never multiplied, and a column
  // past the valid ones, which holds column 0's limbs, only feeds output
  // columns that are not stored; the K tail is zero in the packed limbs)
  auto bstore = [&](int slot, int buf, int64_t c) {
    (void)c;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int i = 0; i < 2; ++i)
        *reinterpret_cast<uint4*>(&Bs[buf][l][bc * X3_COL + 8 * bh + 4 * i]) =
            make_uint4(bst[slot][l][i].x, bst[slot][l][i].y, bst[slot][l][i].z,
                       bst[slot][l][i].w);
  };
  aload(0, 0);
  aload(1, 1);
  bload_(0, 0);
  bload_(1, 1);
  bstore(0, 0, 0);
  __syncthreads();
  // rounds of 6 chunks: A in slots mod 3, X^T limbs in slots mod 2
  for (int64_t cb0 = 0; cb0 < nch; cb0 += 6) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int64_t c = cb0 + u;
      // X^T of chunk c+2 into the slot that chunk c's limbs left (staged at
      // the end of the previous chunk); then A of chunk c+2
      bload_(u & 1, c + 2);
      aload((u + 2) % 3, c + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (c < nch) {  // (uniform; no memory operation but LDS reads inside)
        const uint32_t* tile = &Bs[c & 1][0][0];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          float av[8];
          const uint4 a0 = abuf[u % 3][2 * s2], a1v = abuf[u % 3][2 * s2 + 1];
          av[0] = __uint_as_float(a0.x);
          av[1] = __uint_as_float(a0.y);
          av[2] = __uint_as_float(a0.z);
          av[3] = __uint_as_float(a0.w);
          av[4] = __uint_as_float(a1v.x);
          av[5] = __uint_as_float(a1v.y);
          av[6] = __uint_as_float(a1v.z);
          av[7] = __uint_as_float(a1v.w);
          bf16x8 al[3];
          split3(av, al[0], al[1], al[2]);
          // limb-major, as in tn_x3_kernel
          auto bfrag = [&](int l, int tt) {
            return __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4*>(
                            tile + l * CB * X3_COL + (128 * cw + 32 * tt + r32) * X3_COL +
                            8 * s2 + 4 * h));
          };
          bf16x8 b3[NT], b2[NT], b1[NT];
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b3[tt] = bfrag(2, tt);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b2[tt] = bfrag(1, tt);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt)
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b3[tt], acc[tt], 0, 0, 0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b1[tt] = bfrag(0, tt);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[1], b2[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b2[tt], acc[tt], 0, 0, 0);
          }
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[2], b1[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[1], b1[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b1[tt], acc[tt], 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      bstore((u + 1) & 1, (c + 1) & 1, c + 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int64_t gc = col0 + 32 * tt + r32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gr = row0 + 32 * w + out_row(lane, v);
      if (gr < n && gc < N) {
        float* cp = C + gr * ldc + gc;
        *cp = beta != 0.0f ? alpha * acc[tt][v] + beta * *cp : alpha * acc[tt][v];
      }
    }
  }
}

// C (n x N, ldc) = alpha (sum over the S splits of the FP32 partials, in
// split order) + beta C.
__global__ __launch_bounds__(256) void nn_split_reduce_kernel(int S, int64_t n, int64_t N,
                                                              const float* __restrict__ part,
                                                              float* __restrict__ C,
                                                              int64_t ldc, float alpha,
                                                              float beta) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= n * N) return;
  float acc = 0.0f;
  for (int sp = 0; sp < S; ++sp) acc += part[sp * n * N + idx];
  const int64_t r = idx / N;
  float* c = C + r * ldc + (idx - r * N);
  *c = beta != 0.0f ? alpha * acc + beta * *c : alpha * acc;
}

// ------------------------------------------------------------------ TN --
// Transposing load of one chunk (KC rows x 128 columns) of a row-major
// L x cols matrix into the staged layout [column][128 bytes of rows]; rows
// at or beyond `le` read as zero, columns beyond `cols` are clamped (they
// only feed outputs that are not stored).  Thread t holds row group t mod
// 16 of column group t / 16: the 16 lanes of one LDS store pass write 16
// consecutive 8-byte words of one staged column (no bank conflict; the
// loads of a wavefront take 16 row segments of 64 or 32 bytes).
template <typename T>
struct TLoad;
template <>
struct TLoad<bf16_t> {  // thread: 4 rows x 8 columns
  uint4 v[4];
  uint32_t mk[4];  // rows at or past `le`: re-read the last row, stored as zeros
  __device__ void load(const bf16_t* X, int64_t ldx, int64_t l0, int64_t le, int64_t c0,
                       int64_t cols, int t) {
    const int cg = t >> 4, rg = t & 15;
    int64_t c = c0 + 8 * cg;
    if (c + 8 > cols) c = cols - 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t l = l0 + 4 * rg + i;
      v[i] = *reinterpret_cast<const uint4*>(X + (l < le ? l : le - 1) * ldx + c);
      mk[i] = l < le ? 0xFFFFFFFFu : 0u;
    }
  }
  __device__ void store(uint32_t* tile, int t) const {
    const int cg = t >> 4, rg = t & 15;
    uint32_t w[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w[i][0] = v[i].x & mk[i];
      w[i][1] = v[i].y & mk[i];
      w[i][2] = v[i].z & mk[i];
      w[i][3] = v[i].w & mk[i];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int sh = (e & 1) * 16;
      uint32_t h16[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h16[i] = (w[i][e >> 1] >> sh) & 0xFFFFu;
      *reinterpret_cast<uint2*>(&tile[(8 * cg + e) * LDS_ROW + 2 * rg]) =
          make_uint2(h16[0] | (h16[1] << 16), h16[2] | (h16[3] << 16));
    }
  }
};
template <>
struct TLoad<fp8_t> {  // thread: 8 rows x 8 columns
  uint2 v[8];
  uint32_t mk[8];  // rows at or past `le`: re-read the last row, stored as zeros
  __device__ void load(const fp8_t* X, int64_t ldx, int64_t l0, int64_t le, int64_t c0,
                       int64_t cols, int t) {
    const int cg = t >> 4, rg = t & 15;
    int64_t c = c0 + 8 * cg;
    if (c + 8 > cols) c = cols - 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t l = l0 + 8 * rg + i;
      v[i] = *reinterpret_cast<const uint2*>(X + (l < le ? l : le - 1) * ldx + c);
      mk[i] = l < le ? 0xFFFFFFFFu : 0u;
    }
  }
  __device__ void store(uint32_t* tile, int t) const {
    const int cg = t >> 4, rg = t & 15;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int sh = (e & 3) * 8;
      uint32_t b[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) b[i] = ((((e < 4) ? v[i].x : v[i].y) & mk[i]) >> sh) & 0xFFu;
      *reinterpret_cast<uint2*>(&tile[(8 * cg + e) * LDS_ROW + 2 * rg]) =
          make_uint2(b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24),
                     b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24));
    }
  }
};

// Direct load of one chunk of a packed operand (rows of 128 bytes along the
// reduction): thread t stages half bh of row bc.
struct PLoad {
  uint4 v[4];
  // unconditional (the caller clamps the row and the chunk); `ok` false
  // stages zeros
  __device__ void load(const uint4* rowp, int64_t chunk) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = rowp[chunk * 8 + i];
  }
  __device__ void store(uint32_t* tile, int bc, int bh, bool ok) const {
    const uint32_t mk = ok ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<uint4*>(&tile[bc * LDS_ROW + 16 * bh + 4 * i]) =
          make_uint4(v[i].x & mk, v[i].y & mk, v[i].z & mk, v[i].w & mk);
  }
};

// Workgroup: 128 columns of X (4 wavefronts of 32) x up to 128 columns of Y,
// rows [s Ls, (s+1) Ls) of split s = blockIdx.y; BF16 / FP8 X through the
// transposing load, Y packed (r_pad x L_pad in T, zero padded, with FP8
// scales per 128 rows).
template <typename T, bool SCALED, int NT>
__global__ __launch_bounds__(256, 2) void tn_mfma_kernel(
    int64_t L, int64_t p, int r, const T* __restrict__ X, int64_t ldx,
    const float* __restrict__ xscale, int64_t xscale_ld, const T* __restrict__ Yt,
    int64_t ldyt, const float* __restrict__ yscale, double* __restrict__ partial, int64_t Ls,
    int sym) {
  constexpr int KC = Mf<T>::KC, STEPS = Mf<T>::STEPS, LW = Mf<T>::LW;
  __shared__ uint32_t As[2][128 * LDS_ROW];
  __shared__ uint32_t Bs[2][128 * LDS_ROW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, r32 = lane & 31;
  int64_t pb, rbk;
  if (!xcd_tile(blockIdx.x, (p + 127) / 128, (r + 127) / 128, &pb, &rbk)) return;
  if (sym && pb > rbk) return;  // below the diagonal: mirrored by the reduction
  const int64_t p0 = pb * 128;
  const int64_t r0 = rbk * 128;
  const int64_t sidx = blockIdx.y;
  const int64_t lb = sidx * Ls;
  const int64_t le = (lb + Ls < L) ? lb + Ls : L;
  // NT output tiles of 32 columns at compile time (tiles past the valid
  // columns multiply the zeros staged for them and are not stored)
  const int nt = static_cast<int>((r - r0 + 31) / 32 < NT ? (r - r0 + 31) / 32 : NT);
  const int64_t nch = (le - lb + KC - 1) / KC;
  // FP32 running sums: the operands' rounding (~2^-9 / 2^-4) is far above
  // FP32 summation error
  f32x16 acc[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) acc[tt] = f32x16{};
  // X and Y of chunk c+1 (and its FP8 scale) are loaded while chunk c is
  // multiplied out of LDS, then staged for the next chunk.  Loads are never
  // conditional and no branch separates the chunks (either makes the
  // wait-count pass treat the loads in flight as due): the chunk after the
  // last re-reads the last one and stages zeros.
  TLoad<T> xr;
  PLoad yp;
  const int bc = t >> 1, bh = t & 1;
  const bool bload = bc < 32 * nt;
  const uint4* yrow =
      reinterpret_cast<const uint4*>(Yt + (r0 + (bload ? bc : 0)) * ldyt + lb) + 4 * bh;
  auto scale_of = [&](int64_t c) {
    const int64_t lt = (lb + (c < nch ? c : nch - 1) * KC) >> 7;  // 128-row scale tile
    return xscale[lt * xscale_ld + (p0 >> 7)] * yscale[lt];
  };
  float sc_next = 1.0f;
  if (SCALED) sc_next = scale_of(0);
  xr.load(X, ldx, lb, le, p0, p, t);
  yp.load(yrow, 0);
  xr.store(As[0], t);
  yp.store(Bs[0], bc, bh, bload);
  __syncthreads();
  for (int64_t c = 0; c < nch; ++c) {
    const float sc = sc_next;
    if (SCALED) sc_next = scale_of(c + 1);
    yp.load(yrow, c + 1 < nch ? c + 1 : nch - 1);
    xr.load(X, ldx, lb + (c + 1) * KC, le, p0, p, t);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t* at = As[c & 1];
    const uint32_t* bt = Bs[c & 1];
    f32x16 tmp[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) tmp[tt] = f32x16{};
#pragma unroll
    for (int q = 0; q < STEPS; ++q) {
      uint32_t aw[LW];
      lds_operand<T>(at, 32 * w + r32, h, q, aw);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        uint32_t bw[LW];
        lds_operand<T>(bt, 32 * tt + r32, h, q, bw);
        tmp[tt] = mfma_step<T>(aw, bw, tmp[tt]);
      }
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[tt] += sc * tmp[tt];
    __builtin_amdgcn_sched_barrier(0);
    xr.store(As[(c + 1) & 1], t);
    yp.store(Bs[(c + 1) & 1], bc, bh, bload && c + 1 < nch);
    __syncthreads();
  }
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const int64_t gc = r0 + 32 * tt + r32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gp = p0 + 32 * w + out_row(lane, v);
      if (tt < nt && gp < p && gc < r)
        partial[(sidx * p + gp) * r + gc] = static_cast<double>(acc[tt][v]);
    }
  }
}

// FP32 X^T Y.  Workgroup: 128 columns of X (4 wavefronts of 32) x RB =
// 32 NT columns of Y.  X (row-major L x p) goes straight from memory into
// the operand registers: lane (i, h) of wavefront w holds column
// p0 + 32 w + i and, at step q, row 2 q + h of the 32-row chunk, so each
// load of a wavefront takes two 128-byte row segments and nothing is
// transposed.  The Y chunk (32 rows x RB columns) is staged in LDS in its
// own row order, rows RB + 32 words apart: the two rows one step reads
// (2 q and 2 q + 1) sit 32 banks apart, and a lane reads its column of row
// 2 q + h.  Sums over three 32-row chunks are FP32 (the matrix-core
// steps), added into FP64 running sums.  NT = 2 (64 columns of Y) keeps the FP64 sums,
// two chunks of X and the staging in registers without spills; X is then
// read once per 64 columns of Y, the repeats served by L2 (the column
// blocks of one row block run one after another on one XCD).
template <int NT>
__global__ __launch_bounds__(256, 2) void tn_f32_kernel(int64_t L, int64_t p, int r,
                                                        const float* __restrict__ X,
                                                        int64_t ldx,
                                                        const float* __restrict__ Y,
                                                        int64_t ldy,
                                                        double* __restrict__ partial,
                                                        int64_t Ls, int sym) {
  constexpr int RB = 32 * NT;           // columns of Y per workgroup
  constexpr int YS = RB + 32;           // LDS words per staged row
  constexpr int YQ = RB / 4;            // staging threads per row (16 bytes each)
  constexpr int YR = 256 / YQ;          // rows staged per pass
  constexpr int NP = 32 / YR;           // passes per chunk
  __shared__ float Ys[2][32 * YS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, r32 = lane & 31;
  int64_t pb, rbk;
  if (!xcd_tile(blockIdx.x, (p + 127) / 128, (r + RB - 1) / RB, &pb, &rbk)) return;
  const int64_t p0 = pb * 128;
  const int64_t r0 = rbk * RB;
  if (sym && p0 > r0 + RB - 1) return;  // below the diagonal: mirrored by the reduction
  const int64_t sidx = blockIdx.y;
  const int64_t lb = sidx * Ls;
  const int64_t le = (lb + Ls < L) ? lb + Ls : L;
  const int nt = static_cast<int>((r - r0 + 31) / 32 < NT ? (r - r0 + 31) / 32 : NT);
  const int64_t nch = (le - lb + 31) / 32;
  // this lane's column of X (clamped: columns past p only feed outputs
  // that are not stored); addresses are a uniform row base plus a 32-bit
  // lane offset
  const int64_t xc = (p0 + 32 * w + r32 < p) ? p0 + 32 * w + r32 : p - 1;
  const uint32_t xob = static_cast<uint32_t>((xc + h * ldx) * 4);  // bytes

  // Y staging: thread t moves 16 bytes at columns 4 (t mod YQ) of rows
  // t / YQ + YR i, i < NP (columns past r clamped as above)
  const int yq = t % YQ, yr = t / YQ;
  const bool ycol = 4 * yq < 32 * nt;
  int64_t yc = r0 + 4 * yq;
  if (yc + 4 > r) yc = r - 4;
  const uint32_t yob = static_cast<uint32_t>((yr * ldy + yc) * 4);
  // Loads are never conditional (a load whose register may instead be
  // zeroed forces a wait for every load in flight where the paths meet):
  // rows past the split's end re-read its last row; Y's copies of them are
  // stored as zeros, so they add nothing.
  const int64_t lrel = le - 1 - lb;  // last row of the split, relative
  // whole chunks through buffer loads: the chunk's base in a descriptor
  // (scalar registers), the row in the scalar offset, the lane's column in
  // one vector register (no per-load address arithmetic)
  auto xload = [&](float* xv, int64_t c) {
    if (32 * (c + 1) <= lrel + 1) {  // (uniform) a whole chunk
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(X + (lb + 32 * c) * ldx), 0, -1, kBufferFlags);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        xv[q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
            rs, xob, static_cast<int>(2 * q * ldx * 4), 0));
    } else {  // rows clamped to the split's last (base: the chunk's first
              // row, or the last row for a chunk past the end)
      const int64_t cbase = 32 * c < lrel ? 32 * c : lrel;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(X + (lb + cbase) * ldx), 0, -1, kBufferFlags);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t rr = (32 * c + 2 * q + h < lrel) ? 32 * c + 2 * q + h : lrel;
        xv[q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
            rs, static_cast<uint32_t>(xc * 4 + (rr - cbase) * ldx * 4), 0, 0));
      }
    }
  };
  auto yload_ = [&](uint4* yv, int64_t c) {
    if (32 * (c + 1) <= lrel + 1) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(Y + (lb + 32 * c) * ldy), 0, -1, kBufferFlags);
#pragma unroll
      for (int i = 0; i < NP; ++i)
        yv[i] = __builtin_bit_cast(
            uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, yob, static_cast<int>(YR * i * ldy * 4), 0));
    } else {
      const int64_t cbase = 32 * c < lrel ? 32 * c : lrel;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(Y + (lb + cbase) * ldy), 0, -1, kBufferFlags);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const int64_t rr = (32 * c + yr + YR * i < lrel) ? 32 * c + yr + YR * i : lrel;
        yv[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                              rs, static_cast<uint32_t>(yc * 4 + (rr - cbase) * ldy * 4),
                                              0, 0));
      }
    }
  };
  auto ystore = [&](const uint4* yv, int buf, int64_t c) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      // zeros by a mask, not a branch (a store skipped on some lanes leaves
      // the loads before it looking unfinished to the next chunk)
      const uint32_t mk = (ycol && 32 * c + yr + YR * i <= lrel) ? 0xFFFFFFFFu : 0u;
      *reinterpret_cast<uint4*>(&Ys[buf][(yr + YR * i) * YS + 4 * yq]) =
          make_uint4(yv[i].x & mk, yv[i].y & mk, yv[i].z & mk, yv[i].w & mk);
    }
  };
  double acc[NT][16];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[tt][v] = 0.0;
  // Two chunks in flight ahead of the one multiplied (a chunk is 16 NT
  // matrix-core steps of 64 cycles per wavefront, two wavefronts per SIMD:
  // about one memory latency): X and Y of chunk c+2 are loaded into register
  // slot (c+2) mod 3 while chunk c is multiplied, and Y of chunk c+1 (loaded
  // a chunk earlier) is staged in LDS after it.  Chunks go in rounds of
  // three with no branch around a memory operation: chunks past the last
  // re-read the split's last row and stage zeros (their steps are skipped).
  float xv[3][16];
  uint4 yv[3][NP];
  if (nch == 0) return;  // (uniform; no partials: a split is never empty)
  yload_(yv[0], 0);
  xload(xv[0], 0);
  yload_(yv[1], 1);
  xload(xv[1], 1);
  ystore(yv[0], 0, 0);
  __syncthreads();
  // FP32 sums of a round of chunks (96 rows) per tile, then into FP64
  f32x16 tmp[NT];
  for (int64_t cb0 = 0; cb0 < nch; cb0 += 3) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) tmp[tt] = f32x16{};
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int64_t c = cb0 + u;
      const int s2 = (u + 2) % 3, s1 = (u + 1) % 3;
      // Y first: the wait before the store of Y(c+1) then leaves chunk
      // c+2 in flight (the wait counter drains in issue order)
      yload_(yv[s2], c + 2);
      xload(xv[s2], c + 2);
      // keep the loads here (the scheduler would otherwise sink them
      // next to their uses)
      __builtin_amdgcn_sched_barrier(0);
      if (c < nch) {  // (uniform; no memory operation but LDS reads inside)
        const float* yt = Ys[c & 1] + h * YS + r32;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          // the tile's 16 Y operands first, then its 16 steps
          float yb[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) yb[q] = yt[2 * q * YS + 32 * tt];
#pragma unroll
          for (int q = 0; q < 16; ++q)
            tmp[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[u][q], yb[q], tmp[tt], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      ystore(yv[s1], (c + 1) & 1, c + 1);
      __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tt][v] += static_cast<double>(tmp[tt][v]);
  }
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int64_t gc = r0 + 32 * tt + r32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gp = p0 + 32 * w + out_row(lane, v);
      if (tt < nt && gp < p && gc < r) partial[(sidx * p + gp) * r + gc] = acc[tt][v];
    }
  }
}

// FP32 X^T Y through BF16 limbs: X as in tn_f32_kernel (columns straight
// from memory into registers, here split into limbs there), Y^T packed as
// three limb planes (pack_t_x3) and staged in LDS as in nn_x3_kernel.
// Lane (i, h) of wavefront w holds column p0 + 32 w + i and, at step s of a
// 32-row chunk, rows 16 s + 8 h .. 16 s + 8 h + 7.  Workgroup: 128 columns
// of X x 128 of Y.  FP32 sums over the split (at most kX3SplitRows rows, as
// long as the FP32 sums of the A X products), whose partials the reduction
// adds in FP64.
template <int WN>
__global__ __launch_bounds__(256 * WN) void tn_x3_kernel(int64_t L, int64_t p, int r,
                                                         const float* __restrict__ X,
                                                         int64_t ldx,
                                                         const bf16_t* __restrict__ Yt,
                                                         int64_t ldyt, int64_t plane,
                                                         double* __restrict__ partial,
                                                         int64_t Ls, int sym) {
  constexpr int NT = 4, RB = 128 * WN;  // columns of Y per workgroup
  __shared__ uint32_t Bs[2][3][RB * X3_COL];
  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, r32 = lane & 31;
  // wavefront (w, cw): columns 32 w .. of X x columns 128 cw .. of Y; the
  // WN wavefronts of one X column group load the same rows at the same time
  const int w = (t >> 6) & 3, cw = t >> 8;
  int64_t pb, rbk;
  if (!xcd_tile(blockIdx.x, (p + 127) / 128, (r + RB - 1) / RB, &pb, &rbk)) return;
  const int64_t p0 = pb * 128;
  const int64_t rblk = rbk * RB;          // the block's first column of Y
  const int64_t r0 = rblk + 128 * cw;     // the wavefront's
  if (sym && p0 > rblk + RB - 1) return;  // below the diagonal: mirrored by the reduction
  const int64_t sidx = blockIdx.y;
  const int64_t lb = sidx * Ls;
  const int64_t le = (lb + Ls < L) ? lb + Ls : L;
  const int nt = static_cast<int>((r - r0 + 31) / 32 < NT ? (r - r0 + 31) / 32 : NT);
  const int ntb = static_cast<int>((r - rblk + 31) / 32 < NT * WN ? (r - rblk + 31) / 32
                                                                   : NT * WN);
  const int64_t nch = (le - lb + 31) / 32;
  if (nch == 0) return;  // (uniform; a split is never empty)
  const int64_t xc = (p0 + 32 * w + r32 < p) ? p0 + 32 * w + r32 : p - 1;
  const uint32_t xob = static_cast<uint32_t>((xc + 8 * h * ldx) * 4);
  const int64_t lrel = le - 1 - lb;  // last row of the split, relative
  // X rows of chunk c: whole chunks by buffer loads (row in the scalar
  // offset); a chunk reaching past the split clamps its rows to the last
  // one (their Y limbs are staged as zeros)
  auto xload = [&](float* xv, int64_t c) {
    if (32 * (c + 1) <= lrel + 1) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(X + (lb + 32 * c) * ldx), 0, -1, kBufferFlags);
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          xv[8 * s2 + j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              rs, xob, static_cast<int>((16 * s2 + j) * ldx * 4), 0));
    } else {
      const int64_t cbase = 32 * c < lrel ? 32 * c : lrel;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(X + (lb + cbase) * ldx), 0, -1, kBufferFlags);
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t rr0 = 32 * c + 16 * s2 + 8 * h + j;
          const int64_t rr = rr0 < lrel ? rr0 : lrel;
          xv[8 * s2 + j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              rs, static_cast<uint32_t>(xc * 4 + (rr - cbase) * ldx * 4), 0, 0));
        }
    }
  };
  // Y^T limb staging: thread t moves 32 bytes (16 values) of packed column
  // t / 2, half t mod 2 of the chunk, for each limb
  const int bc = t >> 1, bh = t & 1;
  const bool bload = bc < 32 * ntb;
  const uint4* yrow =
      reinterpret_cast<const uint4*>(Yt + (rblk + (bload ? bc : 0)) * ldyt + lb) + 2 * bh;
  const int64_t pl4 = plane / 8;
  auto yload_ = [&](uint4 (*yv)[2], int64_t c) {
    const int64_t cc = c < nch ? c : nch - 1;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      yv[l][0] = yrow[l * pl4 + cc * 4];
      yv[l][1] = yrow[l * pl4 + cc * 4 + 1];
    }
  };
  // (no masking: a chunk past the end is never multiplied, a column past
  // the valid ones, which holds column 0's limbs, only feeds output columns
  // that are not stored, and rows past the split are zero in the packing)
  auto ystore = [&](const uint4 (*yv)[2], int buf, int64_t c) {
    (void)c;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int i = 0; i < 2; ++i)
        *reinterpret_cast<uint4*>(&Bs[buf][l][bc * X3_COL + 8 * bh + 4 * i]) =
            make_uint4(yv[l][i].x, yv[l][i].y, yv[l][i].z, yv[l][i].w);
  };
  f32x16 acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = f32x16{};
  // X and the Y limbs: two chunks in flight ahead of the one multiplied (X
  // in slots mod 3, Y in slots mod 2); chunk c+1's Y limbs are staged after
  // chunk c.  Rounds of six chunks.
  float xv[3][16];
  uint4 yv[2][3][2];
  yload_(yv[0], 0);
  yload_(yv[1], 1);
  xload(xv[0], 0);
  xload(xv[1], 1);
  ystore(yv[0], 0, 0);
  __syncthreads();
  for (int64_t cb0 = 0; cb0 < nch; cb0 += 6) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int64_t c = cb0 + u;
      yload_(yv[u & 1], c + 2);
      xload(xv[(u + 2) % 3], c + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (c < nch) {  // (uniform; no memory operation but LDS reads inside)
        const uint32_t* tile = &Bs[c & 1][0][0];
        // limb-major: the NT tiles' fragments of one B limb requested
        // together, the next limb's while these are used (the products of a
        // tile in the order a1 b3, a2 b2, a1 b2, a3 b1, a2 b1, a1 b1)
        auto bfrag = [&](int l, int st, int tt) {
          return __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const uint4*>(
                          tile + l * RB * X3_COL + (128 * cw + 32 * tt + r32) * X3_COL +
                          8 * st + 4 * h));
        };
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          bf16x8 al[3];
          split3(&xv[u % 3][8 * st], al[0], al[1], al[2]);
          bf16x8 b3[NT], b2[NT], b1[NT];
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b3[tt] = bfrag(2, st, tt);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b2[tt] = bfrag(1, st, tt);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt)
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b3[tt], acc[tt], 0, 0, 0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) b1[tt] = bfrag(0, st, tt);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[1], b2[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b2[tt], acc[tt], 0, 0, 0);
          }
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[2], b1[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[1], b1[tt], acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[0], b1[tt], acc[tt], 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      ystore(yv[(u + 1) & 1], (c + 1) & 1, c + 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int64_t gc = r0 + 32 * tt + r32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gp = p0 + 32 * w + out_row(lane, v);
      if (tt < nt && gp < p && gc < r)
        partial[(sidx * p + gp) * r + gc] = static_cast<double>(acc[tt][v]);
    }
  }
}

// ---------------------------------------------------------------- pack --
// Dst (cols_pad x rows_pad, T, ld rows_pad) = Src^T for Src rows x cols
// FP32, or FP64 rounded to FP32 (ld lds), zero padded; FP8: one scale per
// 128 source rows, s = amax / 448 over those rows and all columns, values
// e4m3(x / s).
template <typename T>
__device__ __forceinline__ T to_elem(float x, float inv_unused);
template <>
__device__ __forceinline__ float to_elem<float>(float x, float) { return x; }
template <>
__device__ __forceinline__ bf16_t to_elem<bf16_t>(float x, float) { return f32_to_bf16(x); }

template <typename T, typename TS>
__global__ __launch_bounds__(256) void pack_t_kernel(const TS* __restrict__ src, int64_t lds,
                                                     int64_t rows, int64_t cols,
                                                     T* __restrict__ dst, int64_t rows_pad,
                                                     int64_t cols_pad, float* __restrict__ scales) {
  __shared__ float tile[128][33];
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * 128;
  float sc = 1.0f;
  if constexpr (sizeof(T) == 1) {
    float am = 0.0f;
    for (int64_t i = t; i < 128 * cols; i += 256) {
      const int64_t rr = rb + i / cols, cc = i % cols;
      if (rr < rows) am = fmaxf(am, fabsf(static_cast<float>(src[rr * lds + cc])));
    }
    red[t] = am;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if (t < s2) red[t] = fmaxf(red[t], red[t + s2]);
      __syncthreads();
    }
    sc = red[0] > 0.0f ? __fdiv_rn(red[0], 448.0f) : 1.0f;
    if (t == 0) scales[blockIdx.x] = sc;
  }
  for (int64_t c0 = 0; c0 < cols_pad; c0 += 32) {
    // load 128 rows x 32 columns (coalesced along columns)
    for (int i = t; i < 128 * 32; i += 256) {
      const int rr = i >> 5, cc = i & 31;
      const int64_t gr = rb + rr, gc = c0 + cc;
      tile[rr][cc] = (gr < rows && gc < cols) ? static_cast<float>(src[gr * lds + gc]) : 0.0f;
    }
    __syncthreads();
    // write 32 destination rows of 128 values (coalesced along rows)
    for (int i = t; i < 128 * 32; i += 256) {
      const int cc = i >> 7, rr = i & 127;
      const float x = tile[rr][cc];
      T y;
      if constexpr (sizeof(T) == 1) y = f32_to_e4m3(__fdiv_rn(x, sc));
      else y = to_elem<T>(x, 0.0f);
      dst[(c0 + cc) * rows_pad + rb + rr] = y;
    }
    __syncthreads();
  }
}

// Dst (three planes of cols_pad x rows_pad BF16, plane stride `plane`,
// zero padded) = the limbs of Src^T (Src rows x cols FP32, or FP64 rounded
// to FP32 first), for the split FP32 products.
template <typename TS>
__global__ __launch_bounds__(256) void pack_t_x3_kernel(const TS* __restrict__ src, int64_t lds,
                                                        int64_t rows, int64_t cols,
                                                        bf16_t* __restrict__ dst,
                                                        int64_t rows_pad, int64_t cols_pad,
                                                        int64_t plane) {
  __shared__ float tile[128][33];
  const int t = threadIdx.x;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * 128;
  // blockIdx.y: the first of this workgroup's 32-column chunks (gridDim.y
  // chunks apart)
  for (int64_t c0 = 32 * static_cast<int64_t>(blockIdx.y); c0 < cols_pad;
       c0 += 32 * static_cast<int64_t>(gridDim.y)) {
    for (int i = t; i < 128 * 32; i += 256) {
      const int rr = i >> 5, cc = i & 31;
      const int64_t gr = rb + rr, gc = c0 + cc;
      tile[rr][cc] = (gr < rows && gc < cols) ? static_cast<float>(src[gr * lds + gc]) : 0.0f;
    }
    __syncthreads();
    for (int i = t; i < 128 * 32; i += 256) {
      const int cc = i >> 7, rr = i & 127;
      const float x = tile[rr][cc];
      const __bf16 h1 = static_cast<__bf16>(x);
      const float r1 = x - static_cast<float>(h1);
      const __bf16 h2 = static_cast<__bf16>(r1);
      const __bf16 h3 = static_cast<__bf16>(r1 - static_cast<float>(h2));
      const int64_t o = (c0 + cc) * rows_pad + rb + rr;
      dst[o] = __builtin_bit_cast(bf16_t, h1);
      dst[plane + o] = __builtin_bit_cast(bf16_t, h2);
      dst[2 * plane + o] = __builtin_bit_cast(bf16_t, h3);
    }
    __syncthreads();
  }
}

int esize(int type) { return type == BK_F32 ? 4 : (type == BK_BF16 ? 2 : 1); }
int chunk_vals(int type) { return 128 / esize(type); }

// ------------------------------------------------------------ M = W^T W --
// Symmetric Gram of a narrow FP32 block (m <= 384 columns, long L): the
// upper triangle in 32 x 32 tiles; a workgroup of 8 wavefronts takes a tile
// group (up to 40 tiles, 5 per wavefront) over one of S contiguous row
// splits.  Rows arrive in 32-row chunks (contiguous 16-byte loads when m,
// ldw and W allow) into two LDS buffers: while chunk c is multiplied,
// chunk c + 1 goes from registers into the other buffer and chunk c + 2 is
// requested; a chunk's tile is summed in FP32 by 16 MFMA
// steps of two rows and added to the wavefront's FP64 running sums.  The G
// groups of one split run on one XCD (adjacent slots of that XCD), so
// their re-reads of the rows hit its L2.  Output: part[(split T + tile)
// 1024 + v 64 + lane], accumulator register v of lane `lane` (see out_row).
constexpr int GS_CH = 32;    // rows per chunk
constexpr int GS_TPW = 5;    // tiles per wavefront
constexpr int GS_WAVES = 8;  // wavefronts per workgroup
constexpr int GS_TPG = GS_TPW * GS_WAVES;

__device__ __forceinline__ void gs_tile(int ti, int MT, int* bi, int* bj) {
  int b = 0, rem = ti;
  while (rem >= MT - b) {
    rem -= MT - b;
    ++b;
  }
  *bi = b;
  *bj = b + rem;
}

template <bool VEC>
__global__ __launch_bounds__(512) void gram_sym_mfma_kernel(int64_t L, int m,
                                                            const float* __restrict__ W,
                                                            int64_t ldw, int S, int G,
                                                            int64_t per, double* __restrict__ part) {
  extern __shared__ float Wsm[];
  const int MT = (m + 31) >> 5;
  const int T = MT * (MT + 1) / 2;
  const int LDW = MT * 32 + 4;  // (rows 4 banks apart)
  const int BUF = GS_CH * LDW;
  const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
  const int split = (slot / G) * 8 + xcd, g = slot % G;
  if (split >= S) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int bi[GS_TPW], bj[GS_TPW];
  int nt = 0;
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u) {
    const int ti = g * GS_TPG + u * GS_WAVES + w;
    bi[u] = bj[u] = 0;
    if (ti < T) {
      gs_tile(ti, MT, &bi[u], &bj[u]);
      nt = u + 1;
    }
  }
  const int64_t r_lo = static_cast<int64_t>(split) * per;
  const int64_t r_hi = r_lo + per < L ? r_lo + per : L;
  const int64_t nch = (r_hi - r_lo + GS_CH - 1) / GS_CH;
  // chunk copy: VEC: MT * 8 float4 per padded row, NQ = MT / 2 rounded up per
  // thread; else MT * 32 floats per row, 2 MT per thread
  const int RW = VEC ? MT * 8 : MT * 32;
  const int NQ = (GS_CH * RW + 511) / 512;
  constexpr int NQM = VEC ? 6 : 8;  // (MT <= 12; scalar copies: MT <= 4)
  using X = typename std::conditional<VEC, float4, float>::type;
  X xr[NQM];
  auto fetch = [&](int64_t ch, X (&xr)[NQM]) {
    const int64_t c0 = r_lo + ch * GS_CH;
    const int rows = static_cast<int>(r_hi - c0 < GS_CH ? r_hi - c0 : GS_CH);
#pragma unroll
    for (int q = 0; q < NQM; ++q) {
      if (q < NQ) {
        const int e = t + 512 * q;
        const int r = e / RW, c = e - r * RW;
        if constexpr (VEC)
          xr[q] = (r < rows && 4 * c < m)
                      ? *reinterpret_cast<const float4*>(W + (c0 + r) * ldw + 4 * c)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
        else
          xr[q] = (r < rows && c < m) ? W[(c0 + r) * ldw + c] : 0.f;
      }
    }
  };
  auto stage = [&](int64_t ch, const X (&xr)[NQM]) {
    float* buf = Wsm + (ch & 1) * BUF;
#pragma unroll
    for (int q = 0; q < NQM; ++q) {
      if (q < NQ) {
        const int e = t + 512 * q;
        const int r = e / RW, c = e - r * RW;
        if (r < GS_CH) {
          if constexpr (VEC)
            *reinterpret_cast<float4*>(buf + r * LDW + 4 * c) = xr[q];
          else
            buf[r * LDW + c] = xr[q];
        }
      }
    }
  };
  double acc[GS_TPW][16];
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[u][v] = 0.0;
  const int rh = lane >> 5, cl = lane & 31;
  // prologue: chunk 0 staged, chunk 1 in registers
  fetch(0, xr);
  stage(0, xr);
  if (nch > 1) fetch(1, xr);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ++ch) {
    // chunk ch + 1 (registers) into its buffer, then chunk ch + 2 requested
    // into the same registers (that buffer was last read in step ch - 1,
    // which ended with a barrier)
    if (ch + 1 < nch) stage(ch + 1, xr);
    if (ch + 2 < nch) fetch(ch + 2, xr);
    const float* B = Wsm + (ch & 1) * BUF;
#pragma unroll
    for (int u = 0; u < GS_TPW; ++u) {
      if (u < nt) {
        f32x16 c32;
#pragma unroll
        for (int v = 0; v < 16; ++v) c32[v] = 0.f;
        const float* pa = B + rh * LDW + 32 * bi[u] + cl;
        const float* pb = B + rh * LDW + 32 * bj[u] + cl;
#pragma unroll
        for (int st = 0; st < GS_CH / 2; ++st)
          c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[2 * st * LDW], pb[2 * st * LDW], c32,
                                                     0, 0, 0);
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[u][v] += static_cast<double>(c32[v]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u) {
    if (u < nt) {
      const int ti = g * GS_TPG + u * GS_WAVES + w;
      double* o = part + (static_cast<int64_t>(split) * T + ti) * 1024;
#pragma unroll
      for (int v = 0; v < 16; ++v) o[v * 64 + lane] = acc[u][v];
    }
  }
}

// M (m x m FP64, ld ldm, both triangles) = sum over the S splits, in split
// order, of the upper tiles; a diagonal tile supplies its upper half.
__global__ __launch_bounds__(256) void gram_sym_reduce_kernel(int m, int S,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ M,
                                                              int64_t ldm) {
  const int MT = (m + 31) >> 5;
  const int T = MT * (MT + 1) / 2;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(T) * 1024) return;
  const int ti = static_cast<int>(e >> 10), rest = static_cast<int>(e & 1023);
  const int v = rest >> 6, lane = rest & 63;
  int bi, bj;
  gs_tile(ti, MT, &bi, &bj);
  const int i = 32 * bi + out_row(lane, v), j = 32 * bj + (lane & 31);
  if (i >= m || j >= m || (bi == bj && i > j)) return;
  double sum = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < S; ++sp) sum += part[(static_cast<int64_t>(sp) * T + ti) * 1024 + rest];
  M[static_cast<int64_t>(i) * ldm + j] = sum;
  M[static_cast<int64_t>(j) * ldm + i] = sum;
}

}  // namespace

int64_t mfma_pack_bytes(int64_t lred, int64_t cols, int type) {
  const int64_t lp = align_up(static_cast<size_t>(lred), 128);
  const int64_t cp = align_up(static_cast<size_t>(cols), 32);
  return static_cast<int64_t>(align_up(static_cast<size_t>(cp * lp * esize(type)), 256)) +
         (lp / 128) * 4 + 256;
}

// Splits of the limb X^T Y kernel: whole rounds of resident workgroups (one
// per CU with 256-column workgroups, whose staged limbs take 122 KB of LDS,
// two with 128-column ones), one round when the FP32 sum length allows: a
// count just past a round leaves a second round nearly empty (a 1792 x 256
// projection Gram over 131072 rows: 19 splits made 266 workgroups, two
// rounds; 18 make 252).  Never more than tn_mfma_splits, which sizes the
// partials.
static int x3_tn_splits(int64_t L, int64_t p, int r, hipStream_t s) {
  static int cus_cached[64] = {0};
  int dev = 0;
  int cus = 256;
  if (hipStreamGetDevice(s, &dev) == hipSuccess && dev >= 0 && dev < 64) {
    if (cus_cached[dev] == 0) {
      int c = 0;
      cus_cached[dev] =
          (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
           c > 0) ? c : 256;
    }
    cus = cus_cached[dev];
  }
  const int wn = r > 128 ? 2 : 1;
  const int64_t slots = static_cast<int64_t>(cus) * (wn == 2 ? 1 : 2);
  const int64_t nwg = cdiv(p, 128) * cdiv(r, 128 * wn);
  int64_t S = std::max<int64_t>(1, slots / nwg);
  S = std::max<int64_t>(S, cdiv(L, kX3SplitRows));
  S = std::min<int64_t>(S, tn_mfma_splits(L, p, r));
  const int64_t Ls = align_up(static_cast<size_t>(cdiv(L, S)), 128);
  return static_cast<int>(cdiv(L, Ls));
}

int tn_mfma_splits(int64_t L, int64_t p, int r) {
  const int64_t tiles = cdiv(p, 128) * cdiv(r, 128);
  int64_t S = cdiv(512, tiles);
  // FP32 sums of the limb kernel over at most kX3SplitRows rows
  S = std::max<int64_t>(S, cdiv(L, kX3SplitRows));
  const int64_t smax = std::max<int64_t>(1, cdiv(L, 128));
  if (S > smax) S = smax;
  if (S > 64) S = 64;
  if (S < 1) S = 1;
  const int64_t Ls = align_up(static_cast<size_t>(cdiv(L, S)), 128);
  return static_cast<int>(cdiv(L, Ls));
}

// Packs Y (L x cols FP32) for a TN product or X^T for an NN product (X
// FP32, or FP64 coefficients rounded to FP32 when src_f64).
template <typename T>
static void pack_t(const void* src, bool src_f64, int64_t lds, int64_t rows, int64_t cols,
                   void* work, int64_t* rows_pad, int64_t* cols_pad, float** scales,
                   hipStream_t s) {
  *rows_pad = align_up(static_cast<size_t>(rows), 128);
  *cols_pad = align_up(static_cast<size_t>(cols), 32);
  T* dst = static_cast<T*>(work);
  const size_t body = align_up(static_cast<size_t>(*rows_pad * *cols_pad) * sizeof(T), 256);
  *scales = reinterpret_cast<float*>(static_cast<char*>(work) + body);
  const unsigned g = static_cast<unsigned>(*rows_pad / 128);
  if (src_f64)
    pack_t_kernel<T, double><<<g, 256, 0, s>>>(static_cast<const double*>(src), lds, rows, cols,
                                                dst, *rows_pad, *cols_pad, *scales);
  else
    pack_t_kernel<T, float><<<g, 256, 0, s>>>(static_cast<const float*>(src), lds, rows, cols,
                                               dst, *rows_pad, *cols_pad, *scales);
}

// Bytes of the three BF16 limb planes of an lred x cols FP32 operand.
int64_t x3_pack_bytes(int64_t lred, int64_t cols) {
  const int64_t lp = align_up(static_cast<size_t>(lred), 128);
  const int64_t cp = align_up(static_cast<size_t>(cols), 32);
  return static_cast<int64_t>(align_up(static_cast<size_t>(3 * cp * lp * 2), 256)) + 256;
}

// FP32 A X on the BF16 matrix cores through limbs (nn_x3_kernel).
static int nn_run_x3(const NNArgs& a, hipStream_t s) {
  const int64_t kp = align_up(static_cast<size_t>(a.K), 128);
  const int64_t np = align_up(static_cast<size_t>(a.N), 32);
  const int64_t plane = kp * np;
  bf16_t* xt = static_cast<bf16_t*>(a.work);
  const dim3 g(static_cast<unsigned>(kp / 128), static_cast<unsigned>(np / 32));
  if (a.x_f64)
    pack_t_x3_kernel<double><<<g, 256, 0, s>>>(static_cast<const double*>(a.X), a.ldx, a.K, a.N,
                                               xt, kp, np, plane);
  else
    pack_t_x3_kernel<float><<<g, 256, 0, s>>>(static_cast<const float*>(a.X), a.ldx, a.K, a.N,
                                              xt, kp, np, plane);
  const int S = nn_mfma_splits(a.n, a.K, a.N, BK_F32);
  const int64_t nch = a.K / 32;
  const int64_t cps = cdiv(nch, S);
  float* part = S > 1 ? reinterpret_cast<float*>(static_cast<char*>(a.work) +
                                                 x3_pack_bytes(a.K, a.N))
                      : static_cast<float*>(a.C);
  // N > 128: one workgroup of 512 takes 256 columns, so every row of A is
  // read from memory once (two 128-column workgroups drift apart and read
  // it twice)
  const int WN = a.N > 128 ? 2 : 1;
  const dim3 grid(static_cast<unsigned>(xcd_grid(cdiv(a.n, 128), cdiv(a.N, 128 * WN))),
                  static_cast<unsigned>(S));
  const float al = static_cast<float>(a.alpha), be = static_cast<float>(a.beta);
#define BK_NNX_LAUNCH(NTV, WNV)                                                             \
  nn_x3_kernel<NTV, WNV><<<grid, 256 * WNV, 0, s>>>(                                        \
      a.n, a.K, a.N, static_cast<const float*>(a.A), a.lda, xt, kp, plane, part,             \
      S > 1 ? a.N : a.ldc, cps, S > 1 ? 1.0f : al, S > 1 ? 0.0f : be)
  if (WN == 2) BK_NNX_LAUNCH(4, 2);
  else if (a.N <= 32) BK_NNX_LAUNCH(1, 1);
  else if (a.N <= 64) BK_NNX_LAUNCH(2, 1);
  else BK_NNX_LAUNCH(4, 1);
#undef BK_NNX_LAUNCH
  if (S == 1) return 2;
  nn_split_reduce_kernel<<<static_cast<unsigned>(cdiv(a.n * a.N, 256)), 256, 0, s>>>(
      S, a.n, a.N, part, static_cast<float*>(a.C), a.ldc, al, be);
  return 3;
}

template <typename T, bool SCALED>
static int nn_run(const NNArgs& a, int type, hipStream_t s) {
  int64_t kp = 0, np = 0;
  float* xs = nullptr;
  pack_t<T>(a.X, a.x_f64, a.ldx, a.K, a.N, a.work, &kp, &np, &xs, s);
  const int S = nn_mfma_splits(a.n, a.K, a.N, type);
  const int64_t nch = a.K / Mf<T>::KC;
  const int64_t cps = cdiv(nch, S);
  float* part = S > 1 ? reinterpret_cast<float*>(static_cast<char*>(a.work) +
                                                 mfma_pack_bytes(a.K, a.N, type))
                      : static_cast<float*>(a.C);
  const float al = static_cast<float>(a.alpha), be = static_cast<float>(a.beta);
  // chunks of A in flight: one for FP32 (a chunk is ~4000 cycles of
  // matrix-core work), three for BF16 and FP8
  constexpr int PD = sizeof(T) == 4 ? 1 : 3;
  // BF16 / FP8 with N > 128: 256-column workgroups (A read once)
  const int wn = (sizeof(T) < 4 && a.N > 128) ? 2 : 1;
  const dim3 grid(static_cast<unsigned>(xcd_grid(cdiv(a.n, 128), cdiv(a.N, 128 * wn))),
                  static_cast<unsigned>(S));
#define BK_NN_LAUNCH(NTV, WNV)                                                             \
  nn_mfma_kernel<T, SCALED, PD, NTV, WNV><<<grid, 256 * WNV, 0, s>>>(                      \
      a.n, a.K, a.N, static_cast<const T*>(a.A), a.lda, a.ascale, a.ascale_ld,             \
      static_cast<const T*>(a.work), kp, xs, part, S > 1 ? a.N : a.ldc, cps,               \
      S > 1 ? 1.0f : al, S > 1 ? 0.0f : be)
  if (a.N <= 32) BK_NN_LAUNCH(1, 1);
  else if (a.N <= 64) BK_NN_LAUNCH(2, 1);
  else if constexpr (sizeof(T) < 4) {
    if (wn == 2) BK_NN_LAUNCH(4, 2);
    else BK_NN_LAUNCH(4, 1);
  } else {
    BK_NN_LAUNCH(4, 1);
  }
#undef BK_NN_LAUNCH
  if (S == 1) return 2;
  nn_split_reduce_kernel<<<static_cast<unsigned>(cdiv(a.n * a.N, 256)), 256, 0, s>>>(
      S, a.n, a.N, part, static_cast<float*>(a.C), a.ldc, al, be);
  return 3;
}

int nn_mfma_splits(int64_t n, int64_t K, int64_t N, int type) {
  // target 512 workgroups; every split at least 8 chunks of K, at most 16
  const int64_t tiles = cdiv(n, 128) * cdiv(N, 128);
  const int64_t nch = K / chunk_vals(type);
  int64_t S = cdiv(512, tiles);
  S = std::min<int64_t>(S, std::min<int64_t>(16, nch / 8));
  if (S < 2) return 1;
  return static_cast<int>(cdiv(nch, cdiv(nch, S)));  // no empty split
}

int64_t mfma_nn_work_bytes(int64_t n, int64_t K, int64_t N, int type) {
  const int S = nn_mfma_splits(n, K, N, type);
  // FP32: the larger of the FP32 packing and the three BF16 limb planes
  const int64_t pk = type == BK_F32 ? std::max(mfma_pack_bytes(K, N, type), x3_pack_bytes(K, N))
                                    : mfma_pack_bytes(K, N, type);
  return pk +
         (S > 1 ? static_cast<int64_t>(align_up(static_cast<size_t>(S * n * N) * 4, 256)) : 0);
}

void launch_nn_mfma_if(const NNArgs& a, hipStream_t s, int* launches) {
  *launches = 0;
  // FP64 X (coefficients of the orthonormalization and of Z = Q U_k) only
  // with an FP32 A: X is rounded to FP32 in the packing, the sums are FP32
  // as on the vector path
  if (!a.work || a.c_f64 || (a.x_f64 && a.a_type != BK_F32)) return;
  if (a.x_f64 && a.N <= 32) return;  // the small-K vector apply is faster there
  if (a.a_type != BK_F32 && a.a_type != BK_BF16 && a.a_type != BK_FP8_E4M3) return;
  const int es = esize(a.a_type);
  if (a.K <= 0 || a.K % chunk_vals(a.a_type) != 0 || (a.lda * es) % 16 != 0 ||
      (reinterpret_cast<uintptr_t>(a.A) & 15) != 0)
    return;
  if (a.a_type == BK_FP8_E4M3 && !a.ascale) return;
  if (static_cast<int64_t>(a.work_bytes) < mfma_nn_work_bytes(a.n, a.K, a.N, a.a_type)) return;
  // only products large enough to pay for the packing launch
  if (2.0 * static_cast<double>(a.n) * static_cast<double>(a.K) * a.N < 1e8) return;
  switch (a.a_type) {
    case BK_F32:
      *launches = a.fp32_cores ? nn_run<float, false>(a, BK_F32, s) : nn_run_x3(a, s);
      break;
    case BK_BF16:
      *launches = nn_run<bf16_t, false>(a, BK_BF16, s);
      break;
    default:
      *launches = nn_run<fp8_t, true>(a, BK_FP8_E4M3, s);
      break;
  }
}

template <typename T, bool SCALED>
static void tn_run(const TNArgs& a, int S, int64_t Ls, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(xcd_grid(cdiv(a.p, 128), cdiv(a.r, 128))),
                  static_cast<unsigned>(S));
  if constexpr (sizeof(T) == 4) {
    if (!a.fp32_cores && a.work &&
        static_cast<int64_t>(a.work_bytes) >= x3_pack_bytes(a.L, a.r)) {
      // BF16 limbs: Y^T packed in three planes, 64 columns of Y per workgroup
      const int64_t lp = align_up(static_cast<size_t>(a.L), 128);
      const int64_t rp = align_up(static_cast<size_t>(a.r), 32);
      const int64_t plane = lp * rp;
      bf16_t* yt = static_cast<bf16_t*>(a.work);
      pack_t_x3_kernel<float><<<dim3(static_cast<unsigned>(lp / 128),
                                     static_cast<unsigned>(rp / 32)),
                                256, 0, s>>>(static_cast<const float*>(a.Y), a.ldy, a.L, a.r,
                                             yt, lp, rp, plane);
      // r > 128: a workgroup of 512 takes 256 columns of Y, so that X is
      // read from memory once
      if (a.r > 128) {
        const dim3 gridx(static_cast<unsigned>(xcd_grid(cdiv(a.p, 128), cdiv(a.r, 256))),
                         static_cast<unsigned>(S));
        tn_x3_kernel<2><<<gridx, 512, 0, s>>>(a.L, a.p, a.r, static_cast<const float*>(a.X),
                                              a.ldx, yt, lp, plane, a.partial, Ls,
                                              a.sym ? 1 : 0);
      } else {
        const dim3 gridx(static_cast<unsigned>(xcd_grid(cdiv(a.p, 128), cdiv(a.r, 128))),
                         static_cast<unsigned>(S));
        tn_x3_kernel<1><<<gridx, 256, 0, s>>>(a.L, a.p, a.r, static_cast<const float*>(a.X),
                                              a.ldx, yt, lp, plane, a.partial, Ls,
                                              a.sym ? 1 : 0);
      }
      return;
    }
    // 64 columns of Y per workgroup (32 for narrower Y)
    const int NTV = a.r <= 32 ? 1 : 2;
    const dim3 gridf(static_cast<unsigned>(xcd_grid(cdiv(a.p, 128), cdiv(a.r, 32 * NTV))),
                     static_cast<unsigned>(S));
#define BK_TNF_LAUNCH(NTV)                                                                  \
  tn_f32_kernel<NTV><<<gridf, 256, 0, s>>>(a.L, a.p, a.r, static_cast<const float*>(a.X), a.ldx, \
                                           static_cast<const float*>(a.Y), a.ldy, a.partial, Ls,  \
                                           a.sym ? 1 : 0)
    if (NTV == 1) BK_TNF_LAUNCH(1);
    else BK_TNF_LAUNCH(2);
#undef BK_TNF_LAUNCH
  } else {
    float* ys = nullptr;
    int64_t lp = 0, rp = 0;
    pack_t<T>(a.Y, false, a.ldy, a.L, a.r, a.work, &lp, &rp, &ys, s);
    const T* Yt = static_cast<const T*>(a.work);
#define BK_TN_LAUNCH(NTV)                                                                 \
  tn_mfma_kernel<T, SCALED, NTV><<<grid, 256, 0, s>>>(                                    \
      a.L, a.p, a.r, static_cast<const T*>(a.X), a.ldx, a.xscale, a.xscale_ld, Yt, lp, ys, \
      a.partial, Ls, a.sym ? 1 : 0)
    if (a.r <= 32) BK_TN_LAUNCH(1);
    else if (a.r <= 64) BK_TN_LAUNCH(2);
    else BK_TN_LAUNCH(4);
#undef BK_TN_LAUNCH
  }
}

void launch_tn_mfma_if(const TNArgs& a, hipStream_t s, int* splits) {
  *splits = 0;
  if (a.y_f64 || a.L <= 0) return;
  if (a.x_type != BK_F32 && a.x_type != BK_BF16 && a.x_type != BK_FP8_E4M3) return;
  const int es = esize(a.x_type);
  const int vec = 16 / es;  // values per 16-byte load of X
  if (a.p < vec || a.p % vec != 0 || (a.ldx * es) % 16 != 0 ||
      (reinterpret_cast<uintptr_t>(a.X) & 15) != 0)
    return;
  if (a.r < 8) return;
  if (2.0 * static_cast<double>(a.L) * static_cast<double>(a.p) * a.r < 1e9) return;
  const bool packed = a.x_type != BK_F32;
  if (packed) {
    if (!a.work || static_cast<int64_t>(a.work_bytes) < mfma_pack_bytes(a.L, a.r, a.x_type)) return;
    if (a.x_type == BK_FP8_E4M3 && !a.xscale) return;
  } else if (a.r % 4 != 0 || a.ldy % 4 != 0 || (reinterpret_cast<uintptr_t>(a.Y) & 15) != 0 ||
             (a.p + a.ldx) * 4 >= (int64_t(1) << 32) || 32 * a.ldy * 4 >= (int64_t(1) << 32)) {
    return;  // (FP32: lane offsets in bytes must fit 32 bits)
  }
  int S = tn_mfma_splits(a.L, a.p, a.r);
  // FP32: below two workgroups per CU the vector kernel is faster (a 256 x
  // 256 Gram over 131072 rows: 390 us against 660 us on the FP32 matrix
  // cores and 486 us as BF16 limbs, whose limb packing of Y alone writes
  // 200 MB there)
  if (!packed && cdiv(a.p, 128) * cdiv(a.r, 128) * S < 512) return;
  if (!packed && !a.fp32_cores && a.work &&
      static_cast<int64_t>(a.work_bytes) >= x3_pack_bytes(a.L, a.r))
    S = x3_tn_splits(a.L, a.p, a.r, s);
  const int64_t Ls = align_up(static_cast<size_t>(cdiv(a.L, S)), 128);
  switch (a.x_type) {
    case BK_F32:
      tn_run<float, false>(a, S, Ls, s);
      break;
    case BK_BF16:
      tn_run<bf16_t, false>(a, S, Ls, s);
      break;
    default:
      tn_run<fp8_t, true>(a, S, Ls, s);
      break;
  }
  *splits = S;
}

// Splits and tile groups of the symmetric Gram: up to 40 tiles per group
// (the 36 tiles of m = 256 in one group: the 8 wavefronts take 5 or 4, so
// each SIMD's pair takes 9; with 32 per group a second group of 4 tiles
// left half of the workgroups nearly idle),
// enough splits for ~256 workgroups (one per CU), at least 128 rows per
// split.
static void gram_sym_plan(int64_t L, int m, int* S, int* G, int64_t* per) {
  const int MT = static_cast<int>(cdiv(m, 32));
  const int T = MT * (MT + 1) / 2;
  *G = static_cast<int>(cdiv(T, GS_TPG));
  int64_t s_ = cdiv(256, *G);
  const int64_t smax = cdiv(L, 128);
  if (s_ > smax) s_ = smax;
  if (s_ < 1) s_ = 1;
  *per = cdiv(cdiv(L, s_), GS_CH) * GS_CH;
  *S = static_cast<int>(cdiv(L, *per));  // (no empty split)
}

int64_t gram_sym_partial_elems(int64_t L, int m) {
  if (m <= 0 || m > kGramSymMaxM || L < kGramSymMinL) return 0;
  int S, G;
  int64_t per;
  gram_sym_plan(L, m, &S, &G, &per);
  const int64_t MT = cdiv(m, 32);
  return static_cast<int64_t>(S) * (MT * (MT + 1) / 2) * 1024;
}

int launch_gram_sym_mfma(int64_t L, int m, const float* W, int64_t ldw, double* M, int64_t ldm,
                         double* part, hipStream_t s) {
  if (m <= 0 || m > kGramSymMaxM || L < kGramSymMinL) return 0;
  int S, G;
  int64_t per;
  gram_sym_plan(L, m, &S, &G, &per);
  const int MT = static_cast<int>(cdiv(m, 32));
  const int T = MT * (MT + 1) / 2;
  const size_t lds = static_cast<size_t>(2) * GS_CH * (MT * 32 + 4) * sizeof(float);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gram_sym_mfma_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gram_sym_mfma_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  const unsigned grid = static_cast<unsigned>(cdiv(S, 8) * 8 * G);
  const bool vec = m % 4 == 0 && ldw % 4 == 0 && reinterpret_cast<uintptr_t>(W) % 16 == 0;
  if (!vec && m > 128) return 0;  // (scalar copies hold at most 4 tile columns)
  if (vec)
    gram_sym_mfma_kernel<true><<<grid, 512, lds, s>>>(L, m, W, ldw, S, G, per, part);
  else
    gram_sym_mfma_kernel<false><<<grid, 512, lds, s>>>(L, m, W, ldw, S, G, per, part);
  const int64_t outs = static_cast<int64_t>(T) * 1024;
  gram_sym_reduce_kernel<<<static_cast<unsigned>(cdiv(outs, 256)), 256, 0, s>>>(m, S, part, M,
                                                                               ldm);
  return 2;
}

}  // namespace bk
