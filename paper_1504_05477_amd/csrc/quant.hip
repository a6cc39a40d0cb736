// Low-precision copies of A for the block products: BF16 (round to nearest
// even) and OCP e4m3 with one FP32 scale per 128 x 128 tile
// (s = amax / 448, q = RNE-saturate(a / s)).
#include "kernels.hpp"

namespace bk {
namespace {

__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ A,
                                                         int64_t n, int64_t d,
                                                         int64_t lda,
                                                         bf16_t* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n * d) return;
  const int64_t r = i / d, c = i - r * d;
  out[i] = f32_to_bf16(A[r * lda + c]);
}

// One workgroup per 128 x 128 tile (blockIdx.x = tile column, .y = tile row).
__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ A,
                                                        int64_t n, int64_t d,
                                                        int64_t lda,
                                                        fp8_t* __restrict__ out,
                                                        float* __restrict__ scales) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 128;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * 128;
  const int64_t r1 = (r0 + 128 < n) ? r0 + 128 : n;
  const int64_t c1 = (c0 + 128 < d) ? c0 + 128 : d;
  const int64_t w = c1 - c0;
  const int64_t cnt = (r1 - r0) * w;
  float amax = 0.0f;
  for (int64_t i = t; i < cnt; i += 256) {
    const int64_t r = r0 + i / w, c = c0 + i % w;
    amax = fmaxf(amax, fabsf(A[r * lda + c]));
  }
  red[t] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmaxf(red[t], red[t + s]);
    __syncthreads();
  }
  const float am = red[0];
  const float sc = am > 0.0f ? __fdiv_rn(am, 448.0f) : 1.0f;
  if (t == 0) scales[blockIdx.y * gridDim.x + blockIdx.x] = sc;
  for (int64_t i = t; i < cnt; i += 256) {
    const int64_t r = r0 + i / w, c = c0 + i % w;
    out[r * d + c] = f32_to_e4m3(__fdiv_rn(A[r * lda + c], sc));
  }
}

// The same copies stored transposed (out: d x n, ld n; FP8 scales
// [ceil(d/128)][ceil(n/128)]): codes and scales equal those of the copies
// above, element (c, r) of out holding the code of A[r][c].  One workgroup
// per 128 x 128 tile: the tile's codes go through LDS (column-major) so that
// both the reads of A and the writes of out are whole rows.
__global__ __launch_bounds__(256) void quant_fp8_t_kernel(const float* __restrict__ A,
                                                          int64_t n, int64_t d, int64_t lda,
                                                          fp8_t* __restrict__ out,
                                                          float* __restrict__ scales_t) {
  __shared__ float red[256];
  __shared__ uint8_t tile[128][129];  // [column][row] of the tile
  const int t = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 128;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * 128;
  const int64_t r1 = (r0 + 128 < n) ? r0 + 128 : n;
  const int64_t c1 = (c0 + 128 < d) ? c0 + 128 : d;
  const int w = static_cast<int>(c1 - c0), hgt = static_cast<int>(r1 - r0);
  float amax = 0.0f;
  for (int i = t; i < hgt * w; i += 256) {
    const int r = i / w, c = i - r * w;
    amax = fmaxf(amax, fabsf(A[(r0 + r) * lda + c0 + c]));
  }
  red[t] = amax;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) red[t] = fmaxf(red[t], red[t + st]);
    __syncthreads();
  }
  const float am = red[0];
  const float sc = am > 0.0f ? __fdiv_rn(am, 448.0f) : 1.0f;
  if (t == 0) scales_t[static_cast<int64_t>(blockIdx.x) * gridDim.y + blockIdx.y] = sc;
  for (int i = t; i < hgt * w; i += 256) {
    const int r = i / w, c = i - r * w;
    tile[c][r] = f32_to_e4m3(__fdiv_rn(A[(r0 + r) * lda + c0 + c], sc));
  }
  __syncthreads();
  for (int i = t; i < hgt * w; i += 256) {
    const int c = i / hgt, r = i - c * hgt;
    out[(c0 + c) * n + r0 + r] = tile[c][r];
  }
}

__global__ __launch_bounds__(256) void quant_bf16_t_kernel(const float* __restrict__ A,
                                                           int64_t n, int64_t d, int64_t lda,
                                                           bf16_t* __restrict__ out) {
  __shared__ bf16_t tile[64][65];  // [column][row]
  const int t = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 64;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int w = static_cast<int>(((c0 + 64 < d) ? c0 + 64 : d) - c0);
  const int hgt = static_cast<int>(((r0 + 64 < n) ? r0 + 64 : n) - r0);
  for (int i = t; i < hgt * w; i += 256) {
    const int r = i / w, c = i - r * w;
    tile[c][r] = f32_to_bf16(A[(r0 + r) * lda + c0 + c]);
  }
  __syncthreads();
  for (int i = t; i < hgt * w; i += 256) {
    const int c = i / hgt, r = i - c * hgt;
    out[(c0 + c) * n + r0 + r] = tile[c][r];
  }
}

}  // namespace

void launch_quant_t(const float* A, int64_t n, int64_t d, int64_t lda, int to, void* out,
                    float* scales_t, hipStream_t s) {
  if (n * d <= 0) return;
  if (to == BK_FP8_E4M3) {
    const dim3 grid(static_cast<unsigned>(cdiv(d, 128)), static_cast<unsigned>(cdiv(n, 128)));
    quant_fp8_t_kernel<<<grid, 256, 0, s>>>(A, n, d, lda, static_cast<fp8_t*>(out), scales_t);
  } else {
    const dim3 grid(static_cast<unsigned>(cdiv(d, 64)), static_cast<unsigned>(cdiv(n, 64)));
    quant_bf16_t_kernel<<<grid, 256, 0, s>>>(A, n, d, lda, static_cast<bf16_t*>(out));
  }
}

void launch_quant_bf16(const float* A, int64_t n, int64_t d, int64_t lda,
                       bf16_t* out, hipStream_t s) {
  if (n * d <= 0) return;
  quant_bf16_kernel<<<static_cast<unsigned>(cdiv(n * d, 256)), 256, 0, s>>>(A, n, d,
                                                                           lda, out);
}

void launch_quant_fp8(const float* A, int64_t n, int64_t d, int64_t lda,
                      fp8_t* out, float* scales, hipStream_t s) {
  if (n * d <= 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(d, 128)),
                  static_cast<unsigned>(cdiv(n, 128)));
  quant_fp8_kernel<<<grid, 256, 0, s>>>(A, n, d, lda, out, scales);
}

}  // namespace bk
