// Sparse (CSR) block products of the Krylov loop: Y = A X costs
// O(nnz(A) k) (Theorem 6's nnz(A) k q term), plus the implicit row centring
// of the PCA footnote in Section 1 (A - mu 1^T applied as a rank-1
// correction, never densified) and a deterministic GPU transpose that gives
// A^T X the same row-split kernel.
#include <rocprim/device/device_radix_sort.hpp>

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
// per lane, next chunk prefetched).  BATCH (products whose short rows
// average 16 or more nonzeros, so that most chunks fill a batch):
// the pairs are posted to the wavefront's LDS area (slot s at s * KCP, KCP =
// KC rounded up to 4), every lane of the slot reads them back four at a
// time, and the X-row gathers go out 32 at a time with no branch between
// them: entries past the chunk gather nothing (XBUF: an out-of-range buffer
// offset, which reads zero without a memory access; otherwise row 0,
// selected away) and add exact zeros, so the products are added in index
// order as by a plain loop -- one round trip to the cache per 32
// nonzeros.  Otherwise (short runs) the gathers are issued 16, 8, then one
// at a time: more round trips, but the number of gather instructions, which
// bounds these kernels through the texture address unit, stays at the run
// length.  Both add the same products in the same order.
constexpr int kSlotLds = 288;  // LDS entries per wavefront (>= (SLOTS - 1) KCP + 32)

__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool XBUF, bool BATCH>
__device__ __forceinline__ float slot_run(const int32_t* __restrict__ ci,
                                          const float* __restrict__ v,
                                          const float* __restrict__ X, int64_t ldx,
                                          uint32_t xbytes, int32_t b, int32_t e, int32_t step,
                                          int KC, int base, int lbase, int c, int col,
                                          bool colok, int32_t nci, float nv, int32_t* lci,
                                          float* lv) {
  float acc = 0.0f;
  if constexpr (!BATCH) {
    // runs that mostly stop short of 32: the chunk's pairs broadcast by
    // shuffles, gathers in batches of 16, then 8, then one at a time (a
    // round trip each, but no gather instruction past the run)
    for (int32_t j0 = b; j0 < e; j0 += step) {
      const int32_t myci = nci;
      const float myv = nv;
      const int cnt = (e - j0 < KC) ? (e - j0) : KC;
      const int32_t jn = j0 + step + c;
      nci = (jn < e) ? ci[jn] : 0;
      nv = (jn < e) ? v[jn] : 0.0f;
      int t = 0;
      for (; t + 16 <= cnt; t += 16) {
        int32_t cc[16];
        float vv[16], xx[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          cc[u] = __shfl(myci, base + t + u);
          vv[u] = __shfl(myv, base + t + u);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          xx[u] = colok ? X[static_cast<int64_t>(cc[u]) * ldx + col] : 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += vv[u] * xx[u];
      }
      if (t + 8 <= cnt) {
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
        t += 8;
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
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X), 0, static_cast<int>(xbytes),
                                        0x00020000);
  const uint32_t cofs = static_cast<uint32_t>(colok ? col : 0) * 4u;
  for (int32_t j0 = b; j0 < e; j0 += step) {
    const int cnt = (e - j0 < KC) ? (e - j0) : KC;
    wave_lds_order();  // (the previous chunk's reads come first)
    lci[lbase + c] = nci;
    lv[lbase + c] = nv;
    wave_lds_order();
    const int32_t jn = j0 + step + c;
    nci = (jn < e) ? ci[jn] : 0;
    nv = (jn < e) ? v[jn] : 0.0f;
    for (int t = 0; t < cnt; t += 32) {
      int4 c4[8];
      float4 v4[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        c4[q] = *reinterpret_cast<const int4*>(lci + lbase + t + 4 * q);
        v4[q] = *reinterpret_cast<const float4*>(lv + lbase + t + 4 * q);
      }
      float xx[32], vv[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const int q = u >> 2, w = u & 3;
        const int32_t cu = w == 0 ? c4[q].x : w == 1 ? c4[q].y : w == 2 ? c4[q].z : c4[q].w;
        const float vu = w == 0 ? v4[q].x : w == 1 ? v4[q].y : w == 2 ? v4[q].z : v4[q].w;
        const bool in = t + u < cnt && colok;
        vv[u] = in ? vu : 0.0f;
        if constexpr (XBUF) {
          const uint32_t off = in ? static_cast<uint32_t>(cu) * static_cast<uint32_t>(ldx) * 4u + cofs
                                  : 0xFFFFFFF0u;
          xx[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        } else {
          const int64_t row = in ? cu : 0;
          xx[u] = X[row * ldx + (colok ? col : 0)];
          xx[u] = in ? xx[u] : 0.0f;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // (all 32 gathers out before the first sum)
#pragma unroll
      for (int u = 0; u < 32; ++u) acc += vv[u] * xx[u];
    }
  }
  return acc;
}

// Rows of at most short_thr nonzeros: one slot per row (SLOTS rows per
// wavefront).  Longer rows are left to the piece kernels.
template <bool XBUF, bool BATCH>
__global__ __launch_bounds__(256) void csr_spmm_kernel(
    int64_t rows, int k, int KC, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const float* __restrict__ v,
    const float* __restrict__ X, int64_t ldx, uint32_t xbytes, float* __restrict__ Y, int64_t ldy,
    const float* __restrict__ rowvec, const double* __restrict__ colvec,
    int short_thr) {
  __shared__ __align__(16) int32_t s_ci[4 * kSlotLds];
  __shared__ __align__(16) float s_v[4 * kSlotLds];
  const int SLOTS = 64 / KC, KCP = (KC + 3) & ~3;
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  int32_t* lci = s_ci + (threadIdx.x >> 6) * kSlotLds;
  float* lv = s_v + (threadIdx.x >> 6) * kSlotLds;
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
    const int32_t j0 = beg + c;
    float acc = slot_run<XBUF, BATCH>(ci, v, X, ldx, xbytes, beg, end, KC, KC, s * KC, s * KCP, c,
                                      col, colok, (j0 < end && c < KC) ? ci[j0] : 0,
                                      (j0 < end && c < KC) ? v[j0] : 0.0f, lci, lv);
    if (own && col < k) {
      if (colvec) acc -= rv * static_cast<float>(colvec[col]);
      Y[row * ldy + col] = acc;
    }
  }
}

// ------------------------------------------------------------ plan --
constexpr int kPlanRows = 1024;  // rows per plan workgroup (256 threads x 4)

__device__ __forceinline__ int32_t wave_sum_i32(int32_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Per chunk of kPlanRows rows: number of short rows, of long-row pieces and
// of rows cut into more than one piece.
__global__ __launch_bounds__(256) void csr_plan_count_kernel(const int32_t* __restrict__ rp,
                                                             int64_t rows, int piece,
                                                             int32_t* cnt_s, int32_t* cnt_p,
                                                             int32_t* cnt_m, int32_t* cnt_q) {
  __shared__ int32_t red[4][4];
  const int t = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanRows + t * 4;
  int32_t ns = 0, np = 0, nm = 0, nq = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = r0 + u;
    if (r < rows) {
      const int32_t len = rp[r + 1] - rp[r];
      if (len <= kCsrShort) {
        ++ns;
        nq += len;
      } else {
        np += (len + piece - 1) / piece;
        if (len > piece) ++nm;
      }
    }
  }
  ns = wave_sum_i32(ns);
  np = wave_sum_i32(np);
  nm = wave_sum_i32(nm);
  nq = wave_sum_i32(nq);
  if ((t & 63) == 0) {
    red[0][t >> 6] = ns;
    red[1][t >> 6] = np;
    red[2][t >> 6] = nm;
    red[3][t >> 6] = nq;
  }
  __syncthreads();
  if (t == 0) {
    cnt_s[blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    cnt_p[blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    cnt_m[blockIdx.x] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    cnt_q[blockIdx.x] = red[3][0] + red[3][1] + red[3][2] + red[3][3];
  }
}

// Writes, in row order, the short-row list, the piece table and the list
// of rows cut into several pieces (with their first piece).
__global__ __launch_bounds__(256) void csr_plan_write_kernel(
    const int32_t* __restrict__ rp, int64_t rows, int piece, const int32_t* __restrict__ off_s,
    const int32_t* __restrict__ off_p, const int32_t* __restrict__ off_m, int32_t* short_rows,
    int32_t* piece_row, int32_t* piece_first, int32_t* multi_row, int32_t* multi_first) {
  __shared__ int32_t ss[256], sp[256], sm[256];
  const int t = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanRows + t * 4;
  int32_t len[4];
  int32_t ns = 0, np = 0, nm = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = r0 + u;
    len[u] = (r < rows) ? rp[r + 1] - rp[r] : -1;
    if (len[u] >= 0) {
      if (len[u] <= kCsrShort) {
        ++ns;
      } else {
        np += (len[u] + piece - 1) / piece;
        if (len[u] > piece) ++nm;
      }
    }
  }
  ss[t] = ns;
  sp[t] = np;
  sm[t] = nm;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scans
    const int32_t a = t >= off ? ss[t - off] : 0;
    const int32_t b = t >= off ? sp[t - off] : 0;
    const int32_t c = t >= off ? sm[t - off] : 0;
    __syncthreads();
    ss[t] += a;
    sp[t] += b;
    sm[t] += c;
    __syncthreads();
  }
  int32_t os = off_s[blockIdx.x] + ss[t] - ns;
  int32_t op = off_p[blockIdx.x] + sp[t] - np;
  int32_t om = off_m[blockIdx.x] + sm[t] - nm;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (len[u] < 0) continue;
    const int32_t r = static_cast<int32_t>(r0 + u);
    if (len[u] <= kCsrShort) {
      short_rows[os++] = r;
    } else {
      const int32_t npc = (len[u] + piece - 1) / piece;
      for (int32_t j = 0; j < npc; ++j) {
        piece_row[op + j] = r;
        piece_first[op + j] = op;
      }
      if (npc > 1) {
        multi_row[om] = r;
        multi_first[om] = op;
        ++om;
      }
      op += npc;
    }
  }
}

// One product Y = A X (- rowvec c^T, c the centring vector) over a plan.
// Wavefront w < nsw takes SLOTS short rows (one slot each); wavefront
// nsw + p takes piece p: its slots walk interleaved chunks of the piece and
// are added in slot order.  A single-piece row is written at once; the sums
// of a row cut into several pieces go to part[p] and are added by
// csr_combine_kernel.  Y2 (nullable, ld ldy2) receives a second copy of
// every finished row.  OPERAND (0: A, 1: A^T) only names the instance, so
// that profiles tell the two products apart.
template <int OPERAND, bool XBUF, bool BATCH>
__global__ __launch_bounds__(256) void csr_product_kernel(
    int k, int KC, int RPS, int piece, int nshort, int npieces,
    const int32_t* __restrict__ short_rows,
    const int32_t* __restrict__ piece_row, const int32_t* __restrict__ piece_first,
    float* __restrict__ part, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const float* __restrict__ v,
    const float* __restrict__ X, int64_t ldx, uint32_t xbytes, float* __restrict__ Y,
    int64_t ldy, float* __restrict__ Y2, int64_t ldy2, const float* __restrict__ rowvec,
    const double* __restrict__ colvec) {
  __shared__ __align__(16) int32_t s_ci[4 * kSlotLds];
  __shared__ __align__(16) float s_v[4 * kSlotLds];
  const int SLOTS = 64 / KC, KCP = (KC + 3) & ~3;
  const int nsw = (nshort + SLOTS * RPS - 1) / (SLOTS * RPS);
  const int w = static_cast<int>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  int32_t* lci = s_ci + (threadIdx.x >> 6) * kSlotLds;
  float* lv = s_v + (threadIdx.x >> 6) * kSlotLds;
  const int lane = threadIdx.x & 63;
  const int s = lane / KC, c = lane - s * KC;
  if (w < nsw) {
    // slot s takes RPS consecutive entries of the short-row list: lane q of
    // the slot loads row q's id and bounds, shuffled to the slot row by row
    const int idx0 = (w * SLOTS + s) * RPS;
    const bool sok = s < SLOTS;
    int64_t myrow = 0;
    int32_t mybeg = 0, myend = 0;
    if (sok && c < RPS && idx0 + c < nshort) {
      myrow = short_rows[idx0 + c];
      mybeg = rp[myrow];
      myend = rp[myrow + 1];
    }
    const int nrows = (sok && idx0 < nshort) ? min(RPS, nshort - idx0) : 0;
    const int base = s * KC;
    // first chunk of row 0; inside the loop, row q + 1's is loaded before
    // row q is multiplied
    int32_t beg = __shfl(mybeg, sok ? base : 0), end = __shfl(myend, sok ? base : 0);
    if (nrows <= 0) beg = end = 0;
    int32_t fci = (c < KC && beg + c < end) ? ci[beg + c] : 0;
    float fv = (c < KC && beg + c < end) ? v[beg + c] : 0.0f;
    for (int q = 0; q < RPS; ++q) {
      const int src = sok ? base + q : 0;
      const int64_t row = __shfl(myrow, src);
      const bool valid = q < nrows;
      const int srcn = sok ? base + (q + 1 < RPS ? q + 1 : q) : 0;
      int32_t nbeg = __shfl(mybeg, srcn), nend = __shfl(myend, srcn);
      if (q + 1 >= nrows) nbeg = nend = 0;
      const int32_t nci = (c < KC && nbeg + c < nend) ? ci[nbeg + c] : 0;
      const float nv = (c < KC && nbeg + c < nend) ? v[nbeg + c] : 0.0f;
      const float rv = (valid && rowvec) ? rowvec[row] : 1.0f;
      for (int c0 = 0; c0 < k; c0 += KC) {
        const int col = c0 + c;
        const bool colok = valid && col < k;
        float acc = slot_run<XBUF, BATCH>(ci, v, X, ldx, xbytes, valid ? beg : 0,
                                                valid ? end : 0, KC, KC, base, s * KCP, c, col,
                                                colok, fci, fv, lci, lv);
        if (colok) {
          if (colvec) acc -= rv * static_cast<float>(colvec[col]);
          Y[row * ldy + col] = acc;
          if (Y2) Y2[row * ldy2 + col] = acc;
        }
      }
      beg = nbeg;
      end = nend;
      fci = nci;
      fv = nv;
    }
    return;
  }
  const int p = w - nsw;
  if (p >= npieces) return;
  const int64_t row = piece_row[p];
  const int first = piece_first[p];
  const int32_t rb = rp[row], re = rp[row + 1];
  const bool single = re - rb <= piece;
  const int32_t b = rb + (p - first) * piece;
  const int32_t e = (b + piece < re) ? b + piece : re;
  const float rv = rowvec ? rowvec[row] : 1.0f;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    const bool colok = s < SLOTS && col < k;
    const int32_t bs = (s < SLOTS) ? b + s * KC : e;
    const int32_t j0 = bs + c;
    const float acc = slot_run<XBUF, BATCH>(ci, v, X, ldx, xbytes, bs, e, SLOTS * KC, KC, s * KC,
                                           s * KCP, c, col, colok, (j0 < e && c < KC) ? ci[j0] : 0,
                                           (j0 < e && c < KC) ? v[j0] : 0.0f, lci, lv);
    float tot = 0.0f;
    for (int q = 0; q < SLOTS; ++q) tot += __shfl(acc, q * KC + c);
    if (s == 0 && col < k) {
      if (single) {
        if (colvec) tot -= rv * static_cast<float>(colvec[col]);
        Y[row * ldy + col] = tot;
        if (Y2) Y2[row * ldy2 + col] = tot;
      } else {
        part[static_cast<int64_t>(p) * k + col] = tot;
      }
    }
  }
}

// Rows cut into several pieces: Y[row] = sum of the piece sums in piece
// order (- centring), one wavefront per row.
__global__ __launch_bounds__(256) void csr_combine_kernel(
    int nmulti, int k, int piece, const int32_t* __restrict__ multi_row,
    const int32_t* __restrict__ multi_first, const int32_t* __restrict__ rp,
    const float* __restrict__ part, float* __restrict__ Y, int64_t ldy,
    float* __restrict__ Y2, int64_t ldy2, const float* __restrict__ rowvec,
    const double* __restrict__ colvec) {
  const int i = static_cast<int>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (i >= nmulti) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = multi_row[i];
  const int first = multi_first[i];
  const int npc = (rp[row + 1] - rp[row] + piece - 1) / piece;
  const float rv = rowvec ? rowvec[row] : 1.0f;
  for (int col = lane; col < k; col += 64) {
    const float* pp = part + static_cast<int64_t>(first) * k + col;
    float acc = 0.0f;
    int j = 0;
    for (; j + 8 <= npc; j += 8) {  // eight loads in flight, added in order
      float t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = pp[static_cast<int64_t>(j + u) * k];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += t[u];
    }
    for (; j < npc; ++j) acc += pp[static_cast<int64_t>(j) * k];
    if (colvec) acc -= rv * static_cast<float>(colvec[col]);
    Y[row * ldy + col] = acc;
    if (Y2) Y2[row * ldy2 + col] = acc;
  }
}

// Gather copy: xs (rows x kp, kp a multiple of 32 floats, so that every row
// starts on a 128-byte line) = X (rows x k, ld ldx); the padding columns are
// written as zeros.  A thread per four output floats.
__global__ __launch_bounds__(256) void csr_stage_kernel(const float* __restrict__ X,
                                                        int64_t ldx, int64_t rows, int k,
                                                        float* __restrict__ xs, int kp) {
  const int q4 = kp >> 2;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= rows * q4) return;
  const int64_t r = e / q4;
  const int c = 4 * static_cast<int>(e - r * q4);
  const float* x = X + r * ldx;
  float4 o;
  o.x = c < k ? x[c] : 0.0f;
  o.y = c + 1 < k ? x[c + 1] : 0.0f;
  o.z = c + 2 < k ? x[c + 2] : 0.0f;
  o.w = c + 3 < k ? x[c + 3] : 0.0f;
  *reinterpret_cast<float4*>(xs + r * kp + c) = o;
}

// Block partials of the weighted column sums w^T X (FP64): block b sums
// its contiguous row range by slots of KC lanes and adds the slots in slot
// order into colpart[b].
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ X, int64_t ldx,
                                                     int64_t L, int k, int KC,
                                                     const float* __restrict__ w,
                                                     double* __restrict__ colpart) {
  __shared__ double red[4 * 64];
  const int t = threadIdx.x;
  const int SLOTS = 64 / KC;
  const int lane = t & 63;
  const int s = lane / KC, c = lane - s * KC;
  const int slot = (t >> 6) * SLOTS + s;
  const int NSL = 4 * SLOTS;
  const int64_t per = (L + gridDim.x - 1) / gridDim.x;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t re = (rb + per < L) ? rb + per : L;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    const bool ok = s < SLOTS && col < k;
    if (ok) {
      double acc = 0.0;
#pragma unroll 8
      for (int64_t r = rb + slot; r < re; r += NSL) {
        const double wr = w ? static_cast<double>(w[r]) : 1.0;
        acc += wr * static_cast<double>(X[r * ldx + col]);
      }
      red[slot * KC + c] = acc;
    }
    __syncthreads();
    if (t < KC && c0 + t < k) {
      double sum = 0.0;
      for (int q = 0; q < NSL; ++q) sum += red[q * KC + t];
      colpart[static_cast<int64_t>(blockIdx.x) * k + c0 + t] = sum;
    }
    __syncthreads();
  }
}

// colvec[c] = sum of the nb block partials of column c: slots take every
// NSL-th block, then the slots are added in slot order.
__global__ __launch_bounds__(256) void colsum_final_kernel(const double* __restrict__ colpart,
                                                           int nb, int k, int KC,
                                                           double* __restrict__ colvec) {
  __shared__ double red[4 * 64];
  const int t = threadIdx.x;
  const int SLOTS = 64 / KC;
  const int lane = t & 63;
  const int s = lane / KC, c = lane - s * KC;
  const int slot = (t >> 6) * SLOTS + s;
  const int NSL = 4 * SLOTS;
  for (int c0 = 0; c0 < k; c0 += KC) {
    const int col = c0 + c;
    if (s < SLOTS && col < k) {
      double acc = 0.0;
      for (int b = slot; b < nb; b += NSL) acc += colpart[static_cast<int64_t>(b) * k + col];
      red[slot * KC + c] = acc;
    }
    __syncthreads();
    if (t < KC && c0 + t < k) {
      double sum = 0.0;
      for (int q = 0; q < NSL; ++q) sum += red[q * KC + t];
      colvec[c0 + t] = sum;
    }
    __syncthreads();
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
// Exclusive scan of cnt[0..n) into out[0..n] (out[n] = total), one workgroup;
// workgroup b scans cnt + b stride into out + b stride and, with totals,
// also writes its total to totals[b].
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* cnt, int64_t n,
                                                    int32_t* out, int64_t stride = 0,
                                                    int32_t* totals = nullptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  cnt += blockIdx.x * stride;
  out += blockIdx.x * stride;
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
  if (t == 1023) {
    out[n] = static_cast<int32_t>(part[1023]);
    if (totals) totals[blockIdx.x] = static_cast<int32_t>(part[1023]);
  }
}


// Row id and position of every nonzero (the payload of the sort below), a
// wavefront per row.
__global__ __launch_bounds__(256) void expand_rows_kernel(const int32_t* rp, int64_t rows,
                                                          int32_t* rowid, int32_t* pos) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  for (int32_t j = rp[row] + lane; j < rp[row + 1]; j += 64) {
    rowid[j] = static_cast<int32_t>(row);
    pos[j] = j;
  }
}

__global__ __launch_bounds__(256) void copy_keys_kernel(const int32_t* ci, int64_t nnz,
                                                        int32_t* keys) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < nnz) keys[i] = ci[i];
}

// Entry p of A^T (column-major order of A) from the sorted positions.
__global__ __launch_bounds__(256) void gather_t_kernel(const int32_t* src, int64_t nnz,
                                                       const int32_t* rowid,
                                                       const float* v, int32_t* tci,
                                                       float* tv) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (p >= nnz) return;
  const int32_t j = src[p];
  tci[p] = rowid[j];
  tv[p] = v[j];
}

unsigned key_bits(int64_t cols) {
  unsigned b = 1;
  while ((int64_t(1) << b) < cols) ++b;
  return b;
}

int kc_for(int k) { return k < 64 ? k : 64; }

}  // namespace

void launch_csr_validate(const int32_t* rp, const int32_t* ci, int64_t rows,
                         int64_t cols, int64_t nnz, Ctrl* ctrl, hipStream_t s) {
  const int64_t n = (rows > nnz ? rows : nnz) + 1;
  csr_validate_kernel<<<static_cast<unsigned>(cdiv(n, 256)), 256, 0, s>>>(
      rp, ci, rows, cols, nnz, ctrl);
}

// X through a buffer descriptor (range-checked gathers) when its rows span
// less than 2 GB: 32-bit byte offsets, and 0xFFFFFFF0 is out of range.
static uint32_t gather_bytes(int64_t xrows, int64_t ldx) {
  const int64_t b = xrows * ldx * 4;
  return (b > 0 && b <= 0x7FFFFFFF) ? static_cast<uint32_t>(b) : 0u;
}

void launch_csr_spmm(const int32_t* rp, const int32_t* ci, const float* v,
                     int64_t rows, int k, const float* X, int64_t xrows, int64_t ldx, float* Y,
                     int64_t ldy, const float* rowvec, const double* colvec, bool batch,
                     hipStream_t s) {
  if (rows <= 0 || k <= 0) return;
  const int KC = kc_for(k);
  const int64_t waves = cdiv(rows, 64 / KC);
  const uint32_t xb = gather_bytes(xrows, ldx);
  auto kern = xb ? (batch ? csr_spmm_kernel<true, true> : csr_spmm_kernel<true, false>)
                 : (batch ? csr_spmm_kernel<false, true> : csr_spmm_kernel<false, false>);
  kern<<<static_cast<unsigned>(cdiv(waves, 4)), 256, 0, s>>>(
      rows, k, KC, rp, ci, v, X, ldx, xb, Y, ldy, rowvec, colvec, 0x7FFFFFFF);
}

int csr_piece_len(int k) { return (64 / kc_for(k)) * kCsrShort; }

// Short rows per KC-lane slot: up to kCsrSlotRows (at most KC, one lane per
// row for the bounds) when the short rows average at most KC / 2 nonzeros,
// i.e. mostly fit one chunk; otherwise one, so no slot serializes long rows.
int csr_slot_rows(const CsrPlan& pl, int k) {
  const int KC = kc_for(k);
  if (pl.nshort <= 0 || 2 * pl.short_nnz > static_cast<int64_t>(pl.nshort) * KC) return 1;
  return std::min(KC, kCsrSlotRows);
}

int64_t csr_max_pieces(int64_t nnz, int64_t rows) {
  // a row of len > kCsrShort nonzeros has at most len / kCsrShort + 1
  // pieces, and at most nnz / kCsrShort rows are that long
  const int64_t longrows = std::min(rows, nnz / kCsrShort);
  return nnz / kCsrShort + longrows + 1;
}

int64_t csr_plan_chunks(int64_t rows) { return cdiv(rows, kPlanRows); }

void launch_csr_plan(const int32_t* rp, int64_t rows, int k, CsrPlan& pl, int32_t* totals,
                     hipStream_t s) {
  const int64_t nb = csr_plan_chunks(rows);
  int32_t* cnt_s = pl.blk;
  int32_t* cnt_p = pl.blk + (nb + 1);
  int32_t* cnt_m = pl.blk + 2 * (nb + 1);
  int32_t* cnt_q = pl.blk + 3 * (nb + 1);
  int32_t* off_s = pl.blk + 4 * (nb + 1);  // then off_p, off_m, off_q (short nnz)
  int32_t* off_p = pl.blk + 5 * (nb + 1);
  int32_t* off_m = pl.blk + 6 * (nb + 1);
  pl.rows = rows;
  const int piece = csr_piece_len(k);  // pl.operand is set by the caller
  if (nb > 0)
    csr_plan_count_kernel<<<static_cast<unsigned>(nb), 256, 0, s>>>(rp, rows, piece, cnt_s,
                                                                   cnt_p, cnt_m, cnt_q);
  // the four counts in one launch (arrays nb + 1 apart), totals[0..3]
  scan_kernel<<<4, 1024, 0, s>>>(cnt_s, nb, off_s, nb + 1, totals);
  if (nb > 0)
    csr_plan_write_kernel<<<static_cast<unsigned>(nb), 256, 0, s>>>(
        rp, rows, piece, off_s, off_p, off_m, pl.short_rows, pl.piece_row, pl.piece_first,
        pl.multi_row, pl.multi_first);
}

void launch_csr_product(const CsrPlan& pl, const int32_t* rp, const int32_t* ci,
                        const float* v, int k, const float* X, int64_t xrows, int64_t ldx,
                        float* Y, int64_t ldy, float* Y2, int64_t ldy2, const float* rowvec,
                        const double* colvec, hipStream_t s) {
  if (k <= 0) return;
  const int KC = kc_for(k);
  const int rps = csr_slot_rows(pl, k);
  const int64_t nsw = cdiv(pl.nshort, (64 / KC) * rps);
  const int64_t waves = nsw + pl.npieces;
  if (waves <= 0) return;
  const uint32_t xb = gather_bytes(xrows, ldx);
  // gathers 32 at a time when the short rows average 16 or more nonzeros
  // (A X at the term-document workload, document rows: 30.0 -> 25.9 us);
  // else 16 / 8 / 1 at a time (its A^T Y, term rows of ~11 nonzeros: 39.3
  // us, against 45.3 us in batches of 32, whose extra gather instructions
  // load the texture address unit)
  const bool sb = pl.short_nnz >= 16 * static_cast<int64_t>(pl.nshort);
  using K = decltype(&csr_product_kernel<0, true, true>);
  static const K kerns[2][2][2] = {
      {{csr_product_kernel<0, false, false>, csr_product_kernel<0, false, true>},
       {csr_product_kernel<0, true, false>, csr_product_kernel<0, true, true>}},
      {{csr_product_kernel<1, false, false>, csr_product_kernel<1, false, true>},
       {csr_product_kernel<1, true, false>, csr_product_kernel<1, true, true>}}};
  const K kern = kerns[pl.operand ? 1 : 0][xb ? 1 : 0][sb ? 1 : 0];
  kern<<<static_cast<unsigned>(cdiv(waves, 4)), 256, 0, s>>>(
      k, KC, rps, csr_piece_len(k), pl.nshort, pl.npieces, pl.short_rows, pl.piece_row,
      pl.piece_first, pl.part, rp, ci, v, X, ldx, xb, Y, ldy, Y2, ldy2, rowvec, colvec);
}

void launch_csr_combine(const CsrPlan& pl, const int32_t* rp, int k, float* Y, int64_t ldy,
                        float* Y2, int64_t ldy2, const float* rowvec, const double* colvec,
                        hipStream_t s) {
  if (pl.nmulti > 0 && k > 0)
    csr_combine_kernel<<<static_cast<unsigned>(cdiv(pl.nmulti, 4)), 256, 0, s>>>(
        pl.nmulti, k, csr_piece_len(k), pl.multi_row, pl.multi_first, rp, pl.part, Y, ldy,
        Y2, ldy2, rowvec, colvec);
}

int csr_stage_ld(int k) { return static_cast<int>(align_up(static_cast<size_t>(k), 32)); }

void launch_csr_stage(const float* X, int64_t ldx, int64_t rows, int k, float* xs,
                      hipStream_t s) {
  const int kp = csr_stage_ld(k);
  const int64_t total = rows * (kp / 4);
  if (total > 0)
    csr_stage_kernel<<<static_cast<unsigned>(cdiv(total, 256)), 256, 0, s>>>(X, ldx, rows, k,
                                                                            xs, kp);
}

int colsum_blocks(int64_t L) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(kColsumBlocks, cdiv(L, 256))));
}

void launch_colsum(const float* X, int64_t ldx, int64_t L, int k, const float* w,
                   double* colpart, double* colvec, hipStream_t s) {
  if (k <= 0) return;
  const int nb = colsum_blocks(L);
  colsum_kernel<<<static_cast<unsigned>(nb), 256, 0, s>>>(X, ldx, L, k, kc_for(k), w, colpart);
  colsum_final_kernel<<<1, 256, 0, s>>>(colpart, nb, k, kc_for(k), colvec);
}

void launch_colsum_final(const double* colpart, int nb, int k, double* colvec, hipStream_t s) {
  if (k <= 0) return;
  colsum_final_kernel<<<1, 256, 0, s>>>(colpart, nb, k, kc_for(k), colvec);
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

size_t csr_transpose_scratch_bytes(int64_t nnz, int64_t cols) {
  // keys and positions in two buffers each (the sort's double buffers) and
  // the row ids: 20 bytes per nonzero, plus the sort's own storage
  size_t tb = 0;
  rocprim::double_buffer<int32_t> kb(nullptr, nullptr);
  rocprim::double_buffer<int32_t> vb(nullptr, nullptr);
  if (rocprim::radix_sort_pairs(nullptr, tb, kb, vb, static_cast<unsigned>(nnz > 0 ? nnz : 1), 0,
                                key_bits(cols)) != hipSuccess)
    tb = 0;
  return 5 * align_up(static_cast<size_t>(nnz > 0 ? nnz : 1) * 4, 256) + align_up(tb, 256) + 256;
}

int launch_csr_transpose(const int32_t* rp, const int32_t* ci, const float* v, int64_t rows,
                         int64_t cols, int64_t nnz, int32_t* trp, int32_t* tci, float* tv,
                         int32_t* cursor, void* scratch, size_t scratch_bytes, hipStream_t s) {
  // row pointers of A^T: column counts (order-free) and their scan
  launch_fill_i32(cursor, cols, 0, s);
  if (nnz > 0)
    count_cols_kernel<<<static_cast<unsigned>(cdiv(nnz, 256)), 256, 0, s>>>(ci, nnz, cursor);
  scan_kernel<<<1, 1024, 0, s>>>(cursor, cols, trp);
  if (nnz <= 0) return 0;
  // entries: a stable radix sort of the column ids (A's entries come in row
  // order, so each column's entries stay in row order), positions as payload
  const size_t seg = align_up(static_cast<size_t>(nnz) * 4, 256);
  char* b = static_cast<char*>(scratch);
  int32_t* k0 = reinterpret_cast<int32_t*>(b);
  int32_t* k1 = reinterpret_cast<int32_t*>(b + seg);
  int32_t* v0 = reinterpret_cast<int32_t*>(b + 2 * seg);
  int32_t* v1 = reinterpret_cast<int32_t*>(b + 3 * seg);
  int32_t* rowid = reinterpret_cast<int32_t*>(b + 4 * seg);
  void* tmp = b + 5 * seg;
  size_t tb = scratch_bytes > 5 * seg ? scratch_bytes - 5 * seg : 0;
  copy_keys_kernel<<<static_cast<unsigned>(cdiv(nnz, 256)), 256, 0, s>>>(ci, nnz, k0);
  expand_rows_kernel<<<static_cast<unsigned>(cdiv(rows, 4)), 256, 0, s>>>(rp, rows, rowid, v0);
  rocprim::double_buffer<int32_t> kb(k0, k1);
  rocprim::double_buffer<int32_t> vb(v0, v1);
  size_t need = 0;
  if (rocprim::radix_sort_pairs(nullptr, need, kb, vb, static_cast<unsigned>(nnz), 0,
                                key_bits(cols), s) != hipSuccess ||
      need > tb)
    return -1;
  if (rocprim::radix_sort_pairs(tmp, need, kb, vb, static_cast<unsigned>(nnz), 0, key_bits(cols),
                                s) != hipSuccess)
    return -1;
  gather_t_kernel<<<static_cast<unsigned>(cdiv(nnz, 256)), 256, 0, s>>>(vb.current(), nnz,
                                                                       rowid, v, tci, tv);
  return 0;
}

}  // namespace bk
