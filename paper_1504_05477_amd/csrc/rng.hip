// The Gaussian sketch Pi ~ N(0,1)^{d x k} of Algorithm 2, step 1, drawn with
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller in FP64.
#include "kernels.hpp"

namespace bk {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1,
                                              uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed,
                                                       int64_t rows,
                                                       int64_t cols,
                                                       int64_t ld, T* out) {
  const int64_t total = rows * cols;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (2 * j >= total) return;
  uint32_t c0 = static_cast<uint32_t>(j), c1 = static_cast<uint32_t>(j >> 32);
  uint32_t c2 = 0, c3 = 0;
  philox4x32_10(c0, c1, c2, c3, static_cast<uint32_t>(seed),
                static_cast<uint32_t>(seed >> 32));
  // 53-bit uniforms; both products below are exact in FP64.
  const double u1 =
      (static_cast<double>(c0 >> 5) * 67108864.0 + static_cast<double>(c1 >> 6) +
       1.0) * 0x1p-53;
  const double u2 =
      (static_cast<double>(c2 >> 5) * 67108864.0 + static_cast<double>(c3 >> 6)) *
      0x1p-53;
  const double rho = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  const int64_t e0 = 2 * j;
  out[(e0 / cols) * ld + (e0 % cols)] = static_cast<T>(rho * cos(ang));
  if (e0 + 1 < total) {
    const int64_t e1 = e0 + 1;
    out[(e1 / cols) * ld + (e1 % cols)] = static_cast<T>(rho * sin(ang));
  }
}

__global__ __launch_bounds__(256) void philox_raw_kernel(const uint32_t* in,
                                                         int64_t count,
                                                         uint32_t* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c0 = in[6 * i], c1 = in[6 * i + 1], c2 = in[6 * i + 2],
           c3 = in[6 * i + 3];
  philox4x32_10(c0, c1, c2, c3, in[6 * i + 4], in[6 * i + 5]);
  out[4 * i] = c0;
  out[4 * i + 1] = c1;
  out[4 * i + 2] = c2;
  out[4 * i + 3] = c3;
}

}  // namespace

void launch_gaussian(uint64_t seed, int64_t rows, int64_t cols, int64_t ld,
                     bool f64, void* out, hipStream_t s) {
  const int64_t pairs = (rows * cols + 1) / 2;
  if (pairs == 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(pairs, 256)));
  if (f64)
    gaussian_kernel<double><<<grid, 256, 0, s>>>(seed, rows, cols, ld,
                                                 static_cast<double*>(out));
  else
    gaussian_kernel<float><<<grid, 256, 0, s>>>(seed, rows, cols, ld,
                                                static_cast<float*>(out));
}

void launch_philox_raw(const uint32_t* in, int64_t count, uint32_t* out,
                       hipStream_t s) {
  if (count <= 0) return;
  philox_raw_kernel<<<static_cast<unsigned>(cdiv(count, 256)), 256, 0, s>>>(
      in, count, out);
}

}  // namespace bk
