// Reductions behind the error measures of Section 3 (eqs. (1)-(3)): the
// squared Frobenius norm of A, or of the row-centred A - mu 1^T (the PCA
// footnote of Section 1), which the matrix Pythagorean theorem of Section
// 3.2 turns into ||A - Z Z^T A||_F^2 = ||A||_F^2 - ||Z^T A||_F^2.  FP64 sums
// in a fixed order (per-block partials, then the blocks in order).
#include "kernels.hpp"

namespace bk {
namespace {

constexpr int FRO_BLOCKS = 256;

__device__ double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int t = threadIdx.x;
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// Block b sums a[r][c]^2 over rows [b per, (b + 1) per) of a rows x cols
// row-major array (ld).
template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T* __restrict__ a, int64_t rows,
                                                    int64_t cols, int64_t ld, int64_t per,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t r1 = r0 + per < rows ? r0 + per : rows;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r)
    for (int64_t c = threadIdx.x; c < cols; c += 256) {
      const double x = static_cast<double>(a[r * ld + c]);
      s += x * x;
    }
  const double tot = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// CSR rows: sum of v^2 over the row, minus (sum of v)^2 / d with centring
// (||a_r - mean(a_r) 1||^2 = ||a_r||^2 - (1^T a_r)^2 / d).  A wavefront per
// row (coalesced reads of the values), rows dealt to the grid's wavefronts
// in turn; each wavefront adds its rows in order, the block its four
// wavefronts in order.
__global__ __launch_bounds__(256) void csr_sumsq_kernel(const int32_t* __restrict__ rp,
                                                        const float* __restrict__ v,
                                                        int64_t rows, int64_t d, int center,
                                                        double* __restrict__ part) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * 4;
  double acc = 0.0;  // (lane 0's is the wavefront's)
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + w; r < rows; r += nw) {
    double s2 = 0.0, s1 = 0.0;
    for (int32_t j = rp[r] + lane; j < rp[r + 1]; j += 64) {
      const double x = static_cast<double>(v[j]);
      s2 += x * x;
      s1 += x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      s2 += __shfl_xor(s2, o);
      s1 += __shfl_xor(s1, o);
    }
    acc += center ? s2 - s1 * s1 / static_cast<double>(d) : s2;
  }
  if (lane == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    *out = s;
  }
}

// Residual norms of Ritz pairs: block b sums (g_c R[r][c] - theta_c
// Z[r][c])^2 over rows [b per, (b + 1) per) for every column c (a thread
// per column, rows in order), theta_c = sigma_c^2, g_c = rsign[c] (+1 when
// null: a sign applied to Z after R was formed); part is nb x k.
template <typename T>
__global__ __launch_bounds__(256) void ritz_resid_part_kernel(
    const T* __restrict__ R, int64_t ldr, const T* __restrict__ Z, int64_t ldz, int64_t n,
    int k, const double* __restrict__ sigma, const double* __restrict__ rsign, int64_t per,
    double* __restrict__ part) {
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  for (int c = threadIdx.x; c < k; c += 256) {
    const double th = sigma[c] * sigma[c];
    const double g = rsign ? rsign[c] : 1.0;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double e = g * static_cast<double>(R[r * ldr + c]) - th * static_cast<double>(Z[r * ldz + c]);
      s += e * e;
    }
    part[static_cast<int64_t>(blockIdx.x) * k + c] = s;
  }
}

// out[c] = sqrt(sum over blocks, in block order, of part[b][c])
__global__ __launch_bounds__(256) void ritz_resid_final_kernel(const double* __restrict__ part,
                                                               int nb, int k,
                                                               double* __restrict__ out) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < k; c += gridDim.x * 256) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[static_cast<int64_t>(b) * k + c];
    out[c] = sqrt(s);
  }
}

int fro_blocks(int64_t rows) {
  return static_cast<int>(rows < FRO_BLOCKS ? (rows > 0 ? rows : 1) : FRO_BLOCKS);
}

}  // namespace

int64_t fro2_partial_elems() { return FRO_BLOCKS; }

void launch_dense_fro2(const void* A, bool f64, int64_t n, int64_t d, int64_t lda,
                       double* part, double* out, hipStream_t s) {
  const int nb = fro_blocks(n);
  const int64_t per = cdiv(n, nb);
  if (f64)
    sumsq_kernel<double><<<nb, 256, 0, s>>>(static_cast<const double*>(A), n, d, lda, per, part);
  else
    sumsq_kernel<float><<<nb, 256, 0, s>>>(static_cast<const float*>(A), n, d, lda, per, part);
  sum_parts_kernel<<<1, 64, 0, s>>>(part, nb, out);
}

int64_t ritz_resid_partial_elems(int k) { return static_cast<int64_t>(FRO_BLOCKS) * k; }

void launch_ritz_resid(const void* R, int64_t ldr, const void* Z, int64_t ldz, bool f64,
                       int64_t n, int k, const double* sigma, const double* rsign, double* part,
                       double* out, hipStream_t s) {
  const int nb = fro_blocks(n);
  const int64_t per = cdiv(n, nb);
  if (f64)
    ritz_resid_part_kernel<double><<<nb, 256, 0, s>>>(static_cast<const double*>(R), ldr,
                                                      static_cast<const double*>(Z), ldz, n, k,
                                                      sigma, rsign, per, part);
  else
    ritz_resid_part_kernel<float><<<nb, 256, 0, s>>>(static_cast<const float*>(R), ldr,
                                                     static_cast<const float*>(Z), ldz, n, k,
                                                     sigma, rsign, per, part);
  ritz_resid_final_kernel<<<static_cast<int>(cdiv(k, 256)), 256, 0, s>>>(part, nb, k, out);
}

void launch_csr_fro2(const int32_t* rp, const float* v, int64_t n, int64_t d, bool center,
                     double* part, double* out, hipStream_t s) {
  const int nb = fro_blocks(cdiv(n, 4));
  csr_sumsq_kernel<<<nb, 256, 0, s>>>(rp, v, n, d, center ? 1 : 0, part);
  sum_parts_kernel<<<1, 64, 0, s>>>(part, nb, out);
}

}  // namespace bk
