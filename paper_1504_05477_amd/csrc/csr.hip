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

// Lane layout shared by the product kernels: a wavefront is split into
// SLOTS = 64 / KC slots of KC lanes (KC = min(k, 64)); lane c of a slot owns
// output column c0 + c.  A slot walks a run of nonzeros in chunks of KC: the
// chunk's (column id, value) pairs are loaded with one coalesced access (one
// per lane, next chunk prefetched), then broadcast inside the slot with
// shuffles while eight independent X-row gathers are in flight.
__device__ __forceinline__ float slot_run(const int32_t* __restrict__ ci,
                                          const float* __restrict__ v,
                                          const float* __restrict__ X, int64_t ldx,
                                          int32_t b, int32_t e, int32_t step, int KC,
                                          int base, int c, int col, bool colok) {
  float acc = 0.0f;
  int32_t j = b + c;
  int32_t nci = (j < e && c < KC) ? ci[j] : 0;
  float nv = (j < e && c < KC) ? v[j] : 0.0f;
  for (int32_t j0 = b; j0 < e; j0 += step) {
    const int32_t myci = nci;
    const float myv = nv;
    const int cnt = (e - j0 < KC) ? (e - j0) : KC;
    const int32_t jn = j0 + step + c;
    nci = (jn < e) ? ci[jn] : 0;
    nv = (jn < e) ? v[jn] : 0.0f;
    int t = 0;
    for (; t + 8 <= cnt; t += 8) {
      int32_t cc[8];
      float vv[8], xx[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cc[u] = __shfl(myci, base + t + u);
        vv[u] = __shfl(myv, base + t + u);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        xx[u] = colok ? X[static_cast<int64_t>(cc[u]) * ldx + col] : 0.0f;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += vv[u] * xx[u];
    }
    for (; t < cnt; ++t) {
      const int32_t c1 = __shfl(myci, base + t);
      const float v1 = __shfl(myv, base + t);
      const float x1 = colok ? X[static_cast<int64_t>(c1) * ldx + col] : 0.0f;
      acc += v1 * x1;
    }
  }
  return acc;
}

// Rows of at most short_thr nonzeros: one slot per row (SLOTS rows per
// wavefront).  Longer rows are left to the piece kernels.
__global__ __launch_bounds__(256) void csr_spmm_kernel(
    int64_t rows, int k, int KC, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const float* __restrict__ v,
    const float* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    const float* __restrict__ rowvec, const double* __restrict__ colvec,
    int short_thr) {
  const int SLOTS = 64 / KC;
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int s = lane / KC, c = lane - s * KC;
  const int64_t row = wave * SLOTS + s;
  const bool valid = s < SLOTS && row < rows;
  int32_t beg = 0, end = 0;
  bool own = false;
  if (valid) {
    beg = rp[row];
    end = rp[row + 1];
    own = end - beg <= short_thr;
    if (!own) end = beg;  // the piece kernels take this row
  }
  const float rv = (valid && rowvec) ? rowvec[row] : 1.0f;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    const bool colok = valid && col < k;
    float acc = slot_run(ci, v, X, ldx, beg, end, KC, KC, s * KC, c, col, colok);
    if (own && col < k) {
      if (colvec) acc -= rv * static_cast<float>(colvec[col]);
      Y[row * ldy + col] = acc;
    }
  }
}

// Long rows are cut into pieces of kPiece nonzeros; blockIdx = (long row i,
// piece p), one wavefront.  Its slots take interleaved chunks of the piece
// and are added in slot order; the piece sum goes to part[poff[i] + p].
__global__ __launch_bounds__(64) void csr_pieces_kernel(
    const int32_t* __restrict__ list, const int32_t* __restrict__ npc,
    const int32_t* __restrict__ poff, int k, int KC, int piece,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const float* __restrict__ v, const float* __restrict__ X, int64_t ldx,
    float* __restrict__ part) {
  const int i = blockIdx.x;
  const int p = blockIdx.y;
  if (p >= npc[i]) return;
  const int SLOTS = 64 / KC;
  const int lane = threadIdx.x;
  const int s = lane / KC, c = lane - s * KC;
  const int64_t row = list[i];
  const int32_t b = rp[row] + p * piece;
  const int32_t e = (b + piece < rp[row + 1]) ? b + piece : rp[row + 1];
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    const bool colok = s < SLOTS && col < k;
    const int32_t bs = (s < SLOTS) ? b + s * KC : e;
    float acc = slot_run(ci, v, X, ldx, bs, e, SLOTS * KC, KC, s * KC, c, col, colok);
    float tot = 0.0f;
    for (int ss = 0; ss < SLOTS; ++ss) tot += __shfl(acc, ss * KC + c);
    if (s == 0 && col < k) part[(static_cast<int64_t>(poff[i]) + p) * k + col] = tot;
  }
}

// Y[row] = sum of the row's piece sums in piece order (- centring).
__global__ __launch_bounds__(256) void csr_combine_kernel(
    const int32_t* __restrict__ list, const int32_t* __restrict__ npc,
    const int32_t* __restrict__ poff, int nlong, int k,
    const float* __restrict__ part, float* __restrict__ Y, int64_t ldy,
    const float* __restrict__ rowvec, const double* __restrict__ colvec) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (i >= nlong) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = list[i];
  const float rv = rowvec ? rowvec[row] : 1.0f;
  for (int col = lane; col < k; col += 64) {
    float acc = 0.0f;
    for (int p = 0; p < npc[i]; ++p) acc += part[(static_cast<int64_t>(poff[i]) + p) * k + col];
    if (colvec) acc -= rv * static_cast<float>(colvec[col]);
    Y[row * ldy + col] = acc;
  }
}

// Rows longer than short_thr: list them with their piece counts; counters[0]
// = number of listed rows, counters[1] = largest piece count.
__global__ __launch_bounds__(256) void csr_classify_kernel(const int32_t* rp,
                                                           int64_t rows,
                                                           int short_thr, int piece,
                                                           int32_t* list, int32_t* npc,
                                                           int32_t* counters) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (r >= rows) return;
  const int32_t len = rp[r + 1] - rp[r];
  if (len > short_thr) {
    const int32_t pos = atomicAdd(&counters[0], 1);
    const int32_t np = (len + piece - 1) / piece;
    list[pos] = static_cast<int32_t>(r);
    npc[pos] = np;
    atomicMax(&counters[1], np);
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

int kc_for(int k) { return k < 64 ? k : 64; }

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
                     int short_thr, hipStream_t s) {
  if (rows <= 0 || k <= 0) return;
  const int KC = kc_for(k);
  const int64_t waves = cdiv(rows, 64 / KC);
  csr_spmm_kernel<<<static_cast<unsigned>(cdiv(waves, 4)), 256, 0, s>>>(
      rows, k, KC, rp, ci, v, X, ldx, Y, ldy, rowvec, colvec, short_thr);
}

void launch_csr_classify(const int32_t* rp, int64_t rows, int short_thr,
                         int32_t* list, int32_t* npc, int32_t* counters,
                         hipStream_t s) {
  launch_fill_i32(counters, 2, 0, s);
  if (rows > 0)
    csr_classify_kernel<<<static_cast<unsigned>(cdiv(rows, 256)), 256, 0, s>>>(
        rp, rows, short_thr, kCsrPiece, list, npc, counters);
}

void launch_csr_pieces(const CsrPieces& pl, const int32_t* rp, const int32_t* ci,
                       const float* v, int k, const float* X, int64_t ldx, float* Y,
                       int64_t ldy, const float* rowvec, const double* colvec,
                       hipStream_t s) {
  if (pl.nlong <= 0 || k <= 0) return;
  const int KC = kc_for(k);
  const dim3 grid(static_cast<unsigned>(pl.nlong), static_cast<unsigned>(pl.maxp));
  csr_pieces_kernel<<<grid, 64, 0, s>>>(pl.list, pl.npc, pl.poff, k, KC, kCsrPiece, rp, ci,
                                        v, X, ldx, pl.part);
  csr_combine_kernel<<<static_cast<unsigned>(cdiv(pl.nlong, 4)), 256, 0, s>>>(
      pl.list, pl.npc, pl.poff, pl.nlong, k, pl.part, Y, ldy, rowvec, colvec);
}

void launch_scan_i32(const int32_t* cnt, int64_t n, int32_t* out, hipStream_t s) {
  scan_kernel<<<1, 1024, 0, s>>>(cnt, n, out);
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
