// Sparse (CSR) block products of the Krylov loop: Y = A X costs
// O(nnz(A) k) (Theorem 6's nnz(A) k q term), plus the implicit row centring
// of the PCA footnote in Section 1 (A - mu 1^T applied as a rank-1
// correction, never densified) and a deterministic GPU transpose that gives
// A^T X the same row-split kernel.
#include "kernels.hpp"

namespace bk {
namespace {

__global__ __launch_bounds__(256) void csr_validate_kernel(const int32_t* rp,
                                                           const int32_t* ci,
                                                           int64_t rows,
                                                           int64_t cols,
                                                           int64_t nnz, Ctrl* ctrl) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  int bad = 0;
  if (i < rows) {
    if (rp[i] > rp[i + 1] || rp[i] < 0) bad = 1;
  }
  if (i == 0 && (rp[0] != 0 || static_cast<int64_t>(rp[rows]) != nnz)) bad = 1;
  if (i < nnz) {
    const int32_t c = ci[i];
    if (c < 0 || static_cast<int64_t>(c) >= cols) bad = 1;
  }
  if (bad) atomicAdd(&ctrl->csr_bad, 1);
}

// One wavefront per row.  KC lanes cover KC output columns and the 64 / KC
// lane groups ("slots") walk the row's nonzeros with stride 64 / KC; the
// slots are then added with a fixed butterfly, so the sum order is fixed.
template <int KC>
__global__ __launch_bounds__(256) void csr_spmm_kernel(
    int64_t rows, int k, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const float* __restrict__ v,
    const float* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    const float* __restrict__ rowvec, const double* __restrict__ colvec,
    int long_thr) {
  constexpr int SLOTS = 64 / KC;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  const int slot = lane / KC, c = lane % KC;
  const int32_t beg = rp[row], end = rp[row + 1];
  if (end - beg > long_thr) return;
  const float rv = rowvec ? rowvec[row] : 1.0f;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    float acc = 0.0f;
    if (col < k) {
      int32_t j = beg + slot;
      // two nonzeros in flight per slot
      for (; j + SLOTS < end; j += 2 * SLOTS) {
        const int32_t c1 = ci[j], c2 = ci[j + SLOTS];
        const float v1 = v[j], v2 = v[j + SLOTS];
        const float x1 = X[static_cast<int64_t>(c1) * ldx + col];
        const float x2 = X[static_cast<int64_t>(c2) * ldx + col];
        acc += v1 * x1;
        acc += v2 * x2;
      }
      if (j < end) acc += v[j] * X[static_cast<int64_t>(ci[j]) * ldx + col];
    }
#pragma unroll
    for (int off = KC; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
    if (slot == 0 && col < k) {
      if (colvec) acc -= rv * static_cast<float>(colvec[col]);
      Y[row * ldy + col] = acc;
    }
  }
}

// One 1024-thread workgroup per long row: 16 waves take contiguous segments,
// wave partial sums are added in wave order.
template <int KC>
__global__ __launch_bounds__(1024) void csr_spmm_long_kernel(
    const int32_t* __restrict__ list, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const float* __restrict__ v, int k,
    const float* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    const float* __restrict__ rowvec, const double* __restrict__ colvec) {
  constexpr int SLOTS = 64 / KC;
  __shared__ float part[16][KC];
  const int64_t row = list[blockIdx.x];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int slot = lane / KC, c = lane % KC;
  const int32_t beg = rp[row], end = rp[row + 1];
  const int32_t seg = (end - beg + 15) / 16;
  const int32_t sb = beg + wave * seg;
  const int32_t se = (sb + seg < end) ? sb + seg : end;
  const float rv = rowvec ? rowvec[row] : 1.0f;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    float acc = 0.0f;
    if (col < k)
      for (int32_t j = sb + slot; j < se; j += SLOTS)
        acc += v[j] * X[static_cast<int64_t>(ci[j]) * ldx + col];
#pragma unroll
    for (int off = KC; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
    if (slot == 0) part[wave][c] = acc;
    __syncthreads();
    if (threadIdx.x < KC && c0 + static_cast<int>(threadIdx.x) < k) {
      float s = 0.0f;
      for (int w = 0; w < 16; ++w) s += part[w][threadIdx.x];
      const int cc = c0 + threadIdx.x;
      if (colvec) s -= rv * static_cast<float>(colvec[cc]);
      Y[row * ldy + cc] = s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void csr_long_rows_kernel(const int32_t* rp,
                                                            int64_t rows,
                                                            int long_thr,
                                                            int32_t* list,
                                                            int32_t* count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= rows) return;
  if (rp[i + 1] - rp[i] > long_thr) {
    const int32_t pos = atomicAdd(count, 1);
    list[pos] = static_cast<int32_t>(i);
  }
}

// mu[r] = (sum of row r) / cols, summed in FP64 in a fixed order.
__global__ __launch_bounds__(256) void csr_row_means_kernel(const int32_t* rp,
                                                            const float* v,
                                                            int64_t rows,
                                                            int64_t cols, float* mu) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int32_t j = rp[row] + lane; j < rp[row + 1]; j += 64) s += v[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) mu[row] = static_cast<float>(s / static_cast<double>(cols));
}

// ---------------------------------------------------------- transpose --
__global__ __launch_bounds__(256) void count_cols_kernel(const int32_t* ci,
                                                         int64_t nnz, int32_t* cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < nnz) atomicAdd(&cnt[ci[i]], 1);
}

// Exclusive scan of cnt[0..n) into out[0..n], one 1024-thread workgroup.
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* cnt, int64_t n,
                                                    int32_t* out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = t * per;
  const int64_t e = (b + per < n) ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = t ? part[t - 1] : 0;
  for (int64_t i = b; i < e; ++i) {
    out[i] = static_cast<int32_t>(run);
    run += cnt[i];
  }
  if (t == 1023) out[n] = static_cast<int32_t>(part[1023]);
}

__global__ __launch_bounds__(256) void copy_i32_kernel(const int32_t* a, int32_t* b,
                                                       int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Each nonzero (r, c, v) of A goes to the row c of A^T; its slot in that row
// is taken with an atomic, so the key (r << 32 | bits(v)) is stored and the
// rows are sorted afterwards: the result does not depend on the atomics.
__global__ __launch_bounds__(256) void scatter_kernel(const int32_t* rp,
                                                      const int32_t* ci,
                                                      const float* v, int64_t rows,
                                                      int32_t* cursor,
                                                      unsigned long long* keys) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  for (int32_t j = rp[row] + lane; j < rp[row + 1]; j += 64) {
    const int32_t pos = atomicAdd(&cursor[ci[j]], 1);
    keys[pos] = (static_cast<unsigned long long>(static_cast<uint32_t>(row)) << 32) |
                static_cast<unsigned long long>(__float_as_uint(v[j]));
  }
}

// Bitonic sort of one row of keys (ascending) per workgroup; rows of up to
// 4096 keys in LDS, longer rows in the global scratch area `big`
// (length rounded up to a power of two, padded with all-ones keys).
__global__ __launch_bounds__(256) void sort_rows_kernel(const int32_t* trp,
                                                        int64_t nrows,
                                                        unsigned long long* keys,
                                                        unsigned long long* big,
                                                        int32_t* tci, float* tv) {
  __shared__ unsigned long long sk[4096];
  const int64_t row = blockIdx.x;
  if (row >= nrows) return;
  const int t = threadIdx.x;
  const int32_t beg = trp[row], end = trp[row + 1];
  const int32_t len = end - beg;
  if (len <= 0) return;
  int32_t P = 1;
  while (P < len) P <<= 1;
  unsigned long long* K = (P <= 4096) ? sk : big + 2 * static_cast<int64_t>(beg);
  for (int32_t i = t; i < P; i += 256) K[i] = (i < len) ? keys[beg + i] : ~0ull;
  __syncthreads();
  for (int32_t size = 2; size <= P; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = t; i < P / 2; i += 256) {
        const int32_t lo = 2 * stride * (i / stride) + (i % stride);
        const int32_t hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const unsigned long long a = K[lo], b = K[hi];
        if ((a > b) == asc) {
          K[lo] = b;
          K[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int32_t i = t; i < len; i += 256) {
    const unsigned long long key = K[i];
    tci[beg + i] = static_cast<int32_t>(key >> 32);
    tv[beg + i] = __uint_as_float(static_cast<uint32_t>(key & 0xFFFFFFFFull));
  }
}

int kc_for(int k) {
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  if (k <= 32) return 32;
  return 64;
}

}  // namespace

void launch_csr_validate(const int32_t* rp, const int32_t* ci, int64_t rows,
                         int64_t cols, int64_t nnz, Ctrl* ctrl, hipStream_t s) {
  const int64_t n = (rows > nnz ? rows : nnz) + 1;
  csr_validate_kernel<<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(
      rp, ci, rows, cols, nnz, ctrl);
}

void launch_csr_spmm(const int32_t* rp, const int32_t* ci, const float* v,
                     int64_t rows, int k, const float* X, int64_t ldx, float* Y,
                     int64_t ldy, const float* rowvec, const double* colvec,
                     int long_thr, hipStream_t s) {
  if (rows <= 0 || k <= 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(rows, 4)));
  switch (kc_for(k)) {
    case 8:
      csr_spmm_kernel<8><<<grid, 256, 0, s>>>(rows, k, rp, ci, v, X, ldx, Y, ldy,
                                              rowvec, colvec, long_thr);
      break;
    case 16:
      csr_spmm_kernel<16><<<grid, 256, 0, s>>>(rows, k, rp, ci, v, X, ldx, Y, ldy,
                                               rowvec, colvec, long_thr);
      break;
    case 32:
      csr_spmm_kernel<32><<<grid, 256, 0, s>>>(rows, k, rp, ci, v, X, ldx, Y, ldy,
                                               rowvec, colvec, long_thr);
      break;
    default:
      csr_spmm_kernel<64><<<grid, 256, 0, s>>>(rows, k, rp, ci, v, X, ldx, Y, ldy,
                                               rowvec, colvec, long_thr);
      break;
  }
}

void launch_csr_spmm_long(const int32_t* list, int nlong, const int32_t* rp,
                          const int32_t* ci, const float* v, int k, const float* X,
                          int64_t ldx, float* Y, int64_t ldy, const float* rowvec,
                          const double* colvec, hipStream_t s) {
  if (nlong <= 0 || k <= 0) return;
  switch (kc_for(k)) {
    case 8:
      csr_spmm_long_kernel<8><<<nlong, 1024, 0, s>>>(list, rp, ci, v, k, X, ldx, Y,
                                                     ldy, rowvec, colvec);
      break;
    case 16:
      csr_spmm_long_kernel<16><<<nlong, 1024, 0, s>>>(list, rp, ci, v, k, X, ldx, Y,
                                                      ldy, rowvec, colvec);
      break;
    case 32:
      csr_spmm_long_kernel<32><<<nlong, 1024, 0, s>>>(list, rp, ci, v, k, X, ldx, Y,
                                                      ldy, rowvec, colvec);
      break;
    default:
      csr_spmm_long_kernel<64><<<nlong, 1024, 0, s>>>(list, rp, ci, v, k, X, ldx, Y,
                                                      ldy, rowvec, colvec);
      break;
  }
}

void launch_csr_long_rows(const int32_t* rp, int64_t rows, int long_thr,
                          int32_t* list, int32_t* count, hipStream_t s) {
  launch_fill_i32(count, 1, 0, s);
  if (rows > 0)
    csr_long_rows_kernel<<<static_cast<unsigned>(cdiv(rows, 256)), 256, 0, s>>>(
        rp, rows, long_thr, list, count);
}

void launch_csr_row_means(const int32_t* rp, const float* v, int64_t rows,
                          int64_t cols, float* mu, hipStream_t s) {
  if (rows > 0)
    csr_row_means_kernel<<<static_cast<unsigned>(cdiv(rows, 4)), 256, 0, s>>>(
        rp, v, rows, cols, mu);
}

void launch_csr_transpose(const int32_t* rp, const int32_t* ci, const float* v,
                          int64_t rows, int64_t cols, int64_t nnz, int32_t* trp,
                          int32_t* tci, float* tv, int32_t* cursor,
                          unsigned long long* keys, hipStream_t s) {
  // cursor: cols ints; keys: 3 * nnz (nnz sort keys + 2 * nnz scratch)
  launch_fill_i32(cursor, cols, 0, s);
  if (nnz > 0)
    count_cols_kernel<<<static_cast<unsigned>(cdiv(nnz, 256)), 256, 0, s>>>(ci, nnz,
                                                                           cursor);
  scan_kernel<<<1, 1024, 0, s>>>(cursor, cols, trp);
  if (cols > 0)
    copy_i32_kernel<<<static_cast<unsigned>(cdiv(cols, 256)), 256, 0, s>>>(trp, cursor,
                                                                          cols);
  if (rows > 0)
    scatter_kernel<<<static_cast<unsigned>(cdiv(rows, 4)), 256, 0, s>>>(rp, ci, v, rows,
                                                                       cursor, keys);
  if (cols > 0)
    sort_rows_kernel<<<static_cast<unsigned>(cols), 256, 0, s>>>(trp, cols, keys,
                                                                keys + nnz, tci, tv);
}

}  // namespace bk
