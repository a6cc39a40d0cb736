// Host driver and C ABI of the Block Krylov library.
//
// One solve (Algorithm 2):
//   Pi (Philox)  ->  B_0 = A Pi  ->  Q_0 = orth(B_0)
//   for i = 1..q:   Y_i = A^T Q_{i-1}      (kept: W = [Y_1 .. Y_{q+1}] = A^T Q)
//                   B_i = A Y_i
//                   B_i <- (I - Q_<i Q_<i^T) B_i   twice (block Gram-Schmidt)
//                   Q_i = orth(B_i)   (shifted CholeskyQR3, FP64 Gram/Cholesky)
//   Y_{q+1} = A^T Q_q;   M = W^T W (FP64)   (= Q^T A A^T Q)
//   Jacobi(M) -> top-k (theta, U_k);   Z = Q U_k;   sigma = sqrt(theta)
// Feeding the orthonormal block Q_{i-1} (not the raw power) into the next
// product keeps every block well scaled (the per-block reorthonormalization
// of Section 4.2), and it makes W = A^T Q a by-product of the loop: forming
// M costs one extra k-wide product instead of an m-wide one.
//
// Breakdown of a block i >= 1 (invariant Krylov space) zeroes that block and
// every later one follows (A A^T 0 = 0), so the Rayleigh-Ritz step over the
// zero-padded basis equals the one over the blocks built so far: no host
// round trip is needed inside the loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace bk {
namespace {

constexpr double kEps64 = 2.220446049250313e-16;
constexpr double kUnit64 = 1.1102230246251565e-16;  // 2^-53

// ------------------------------------------------------------ workspace --
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Options {
  int refine = 0, center = 0, max_sweeps = 40, timing = 0, save = 0, jblock = 0;
  int timing_phases = 0;  // bitmask of timed phases (0: all)
  int p = 0;   // block width (0: k), oversampling of Section 6
  int si = 0;  // 1: simultaneous iteration (Algorithm 1)
  int bl = 0;  // 1: block-tridiagonal Rayleigh-Ritz matrix (block Lanczos)
  double jtol = 0.0, tau = 0.0;
  const void* pi = nullptr;
  double* resid = nullptr;  // device k: residual norms of the Ritz pairs
  const void* at = nullptr;  // transposed low-precision copy of A (nullable)
  int64_t ld_at = 0;
  const float* at_scales = nullptr;
  bool fp32_cores = false;   // FP32 products on the FP32 matrix cores
  bool csr_staged = false;   // CSR products gather from padded copies
};

Options read_options(const bk_options* o, bool f64) {
  Options r;
  if (o && o->struct_size >= static_cast<int32_t>(offsetof(bk_options, timing_phases))) {
    r.refine = o->refine;
    r.center = o->center_rows;
    if (o->max_jacobi_sweeps > 0) r.max_sweeps = o->max_jacobi_sweeps;
    r.jtol = o->jacobi_tol;
    r.tau = o->breakdown_tol;
    r.pi = o->pi;
    r.timing = o->timing;
    r.save = o->save_for_backward;
    r.jblock = o->jacobi_block;
    r.p = o->block_size;
    r.si = o->method == BK_METHOD_SIMULTANEOUS ? 1 : 0;
    r.bl = o->method == BK_METHOD_BLOCK_LANCZOS ? 1 : 0;
    if (o->struct_size >= static_cast<int32_t>(offsetof(bk_options, reserved)))
      r.timing_phases = o->timing_phases;
    if (o->struct_size >= static_cast<int32_t>(offsetof(bk_options, residuals) + sizeof(double*)))
      r.resid = o->residuals;
    if (o->struct_size >= static_cast<int32_t>(offsetof(bk_options, at_scales) + sizeof(float*))) {
      r.at = o->a_transposed;
      r.ld_at = o->ld_at;
      r.at_scales = o->at_scales;
    }
    if (o->struct_size >= static_cast<int32_t>(offsetof(bk_options, fp32_products) + sizeof(int32_t)))
      r.fp32_cores = o->fp32_products == 1;
    if (o->struct_size >= static_cast<int32_t>(offsetof(bk_options, csr_gather) + sizeof(int32_t)))
      r.csr_staged = o->csr_gather == BK_CSR_GATHER_STAGED;
  }
  if (!(r.tau > 0.0)) r.tau = f64 ? 1e-11 : 1e-5;
  return r;
}

double jacobi_tol_for(int64_t m, double user) {
  return user > 0.0 ? user : 10.0 * std::sqrt(static_cast<double>(m)) * kEps64;
}

int jacobi_block_for(int64_t m, int user) {
  return (user == 8 || user == 16) ? user : jacobi_default_block(m);
}

// Largest FP64 partial-sum buffer any TN call of a solve needs.
int64_t partial_need(int64_t n, int64_t d, int k, int q, bool refine, bool csr) {
  const int64_t m = static_cast<int64_t>(q + 1) * k;
  int64_t need = std::max<int64_t>(tn_partial_elems(n, k, k), tn_partial_elems(d, m, static_cast<int>(m)));
  need = std::max(need, tn_partial_elems(d, k, k));  // the last block's Gram (block Lanczos)
  if (!csr) need = std::max(need, tn_partial_elems(n, d, k));
  // projection of block i: [Q_<i, B]^T B (i + 1) k x k, then Q_<i^T B
  for (int i = 1; i <= q + 1; ++i)
    need = std::max(need, tn_partial_elems(n, static_cast<int64_t>(i) * k, k));
  // Gram partials of the fused applies (k <= 32): one k x k per row block;
  // the one-launch CholeskyQR passes alternate between two sets
  need = std::max(need, nn_gram_partial_elems(n, k));
  need = std::max(need, 2 * cqr_pass_partial_elems(k));
  // M = W^T W on the matrix cores (FP32 W, m <= kGramSymMaxM), and the
  // CholeskyQR Grams of the blocks the same way
  need = std::max(need, gram_sym_partial_elems(d, static_cast<int>(m)));
  need = std::max(need, gram_sym_partial_elems(n, k));
  if (refine) {
    need = std::max(need, tn_partial_elems(n, d, k));
    need = std::max(need, tn_partial_elems(d, k, k));
  }
  if (csr) {
    need = std::max(need, tn_partial_elems(d, k, 1));
    need = std::max(need, tn_partial_elems(n, k, 1));
  }
  return need;
}

struct JacobiWs {
  double* Xc = nullptr;
  double* Vc = nullptr;
  double* norms = nullptr;
  double* theta = nullptr;
  int32_t* order = nullptr;
  int64_t ldc = 0, nbp = 0;
  int b = 16;
};

JacobiWs take_jacobi(Arena& ar, int64_t m, int jblock, bool withv) {
  JacobiWs j;
  j.b = jacobi_block_for(m, jblock);
  j.nbp = jacobi_padded_cols(m, j.b);
  j.ldc = m;
  j.Xc = ar.take<double>(static_cast<size_t>(j.nbp * m));
  if (withv) j.Vc = ar.take<double>(static_cast<size_t>(j.nbp * m));
  j.norms = ar.take<double>(static_cast<size_t>(m));
  j.theta = ar.take<double>(static_cast<size_t>(m));
  j.order = ar.take<int32_t>(static_cast<size_t>(m));
  return j;
}

// The Rayleigh-Ritz eigen-solve goes through the tridiagonal reduction for
// moderate m unless every eigenvector is kept (adjoint) or Jacobi is asked
// for explicitly (jacobi_block).
bool use_tridiag(int64_t m, const Options& o) {
  return !o.save && o.jblock == 0 && m <= kTridiagMax;
}

struct Layout {
  Ctrl* ctrl = nullptr;
  void* Pi = nullptr;
  void* Q = nullptr;
  void* W = nullptr;
  void* Bs = nullptr;
  void* Bs2 = nullptr;
  double* partial = nullptr;
  int64_t partial_elems = 0;
  void* pack = nullptr;  // matrix-core operand packing of the dense products
  size_t pack_bytes = 0;
  double *G = nullptr, *Gpre = nullptr, *R = nullptr, *Rinv = nullptr,
         *cholwork = nullptr, *Racc = nullptr, *Rtmp = nullptr;
  double* C = nullptr;
  double* M = nullptr;
  JacobiWs jw;
  double* Uk = nullptr;
  double* tri = nullptr;  // tridiagonal eigen-solve scratch (when used)
  double* sign = nullptr;
  double* Rsave = nullptr;  // (q+1) x k x k, R_i of B_i = Q_i R_i (saved)
  double* ritz_dev = nullptr;
  // block Lanczos: per-block projection coefficients (two passes, stride
  // m k) and CholeskyQR factors (three passes), scratch, the last block
  double *Cband = nullptr, *Rband = nullptr, *Pband = nullptr, *Tqq = nullptr;
  // residual norms of the Ritz pairs: A^T Z (d x block width, the working
  // type) and the norm partials
  void* Wr = nullptr;
  double* rpart = nullptr;
  // refinement
  float* Wk = nullptr;
  double* Gk = nullptr;
  double* Pk = nullptr;
  JacobiWs jk;
  double* trik = nullptr;  // its tridiagonal eigen-solve scratch
  // CSR
  int32_t *trp = nullptr, *tci = nullptr, *cursor = nullptr, *counters = nullptr;
  CsrPlan plan_a, plan_t;       // work plans of A and A^T (shared part)
  double* colpart = nullptr;    // kColsumBlocks x k block sums of the centring
  float* tv = nullptr;
  char* tscratch = nullptr;  // CSR transpose: sort buffers
  size_t tscratch_bytes = 0;
  float* mu = nullptr;
  double* colvec = nullptr;
  float* xs = nullptr;  // staged CSR gathers: d x csr_stage_ld(k), n x ...
  float* ys = nullptr;
  size_t bytes = 0;
};

Layout make_layout(char* base, int64_t n, int64_t d, int64_t nnz, int k, int q,
                   bool f64, const Options& o, bool csr, bool own_transpose) {
  Arena ar;
  ar.base = base;
  Layout L;
  const size_t es = f64 ? 8 : 4;
  const int64_t m = o.si ? k : static_cast<int64_t>(q + 1) * k;  // k: block width here
  L.ctrl = ar.take<Ctrl>(1);
  L.Pi = ar.take<char>(static_cast<size_t>(d * k) * es);
  L.Q = ar.take<char>(static_cast<size_t>(n * m) * es);
  L.W = ar.take<char>(static_cast<size_t>(d * m) * es);
  L.Bs = ar.take<char>(static_cast<size_t>(n * k) * es);
  L.Bs2 = ar.take<char>(static_cast<size_t>(n * k) * es);
  L.partial_elems = partial_need(n, d, k, q, o.refine != 0, csr);
  L.partial = ar.take<double>(static_cast<size_t>(L.partial_elems));
  if (!csr && !f64) {
    // X^T of A X in FP32 (the widest type), Y^T of A^T Y in BF16 / FP8
    int64_t nn = 0;  // A X on the matrix cores: packed X^T (+ split partials)
    for (int t : {BK_F32, BK_BF16, BK_FP8_E4M3}) nn = std::max(nn, mfma_nn_work_bytes(n, d, k, t));
    // A^T Y on a transposed BF16 / FP8 copy: packed Y^T (+ split partials)
    for (int t : {BK_BF16, BK_FP8_E4M3}) nn = std::max(nn, mfma_nn_work_bytes(d, n, k, t));
    // FP32 X^T Y through BF16 limbs: Y's limb planes (A^T Y: n rows; the
    // Grams: n or d rows)
    nn = std::max(nn, x3_pack_bytes(std::max(n, d), k));
    L.pack_bytes = static_cast<size_t>(std::max(nn, mfma_pack_bytes(n, k, BK_BF16)));
    L.pack = ar.take<char>(L.pack_bytes);
  }
  const size_t kk = static_cast<size_t>(k) * k;
  L.G = ar.take<double>(kk);
  L.Gpre = ar.take<double>(kk);
  L.R = ar.take<double>(kk);
  L.Rinv = ar.take<double>(kk);
  L.cholwork = ar.take<double>(static_cast<size_t>(chol_work_doubles(k)));
  L.Racc = ar.take<double>(kk);
  L.Rtmp = ar.take<double>(kk);
  L.C = ar.take<double>(static_cast<size_t>(m * k));
  L.M = ar.take<double>(static_cast<size_t>(m * m));
  L.jw = take_jacobi(ar, m, o.jblock, o.save != 0);
  L.Uk = ar.take<double>(static_cast<size_t>(m * k));
  if (use_tridiag(m, o)) L.tri = ar.take<double>(static_cast<size_t>(tridiag_scratch_doubles(m, k)));
  L.sign = ar.take<double>(static_cast<size_t>(k));
  L.ritz_dev = ar.take<double>(static_cast<size_t>(k));
  if (o.bl && !o.si) {
    L.Cband = ar.take<double>(2 * static_cast<size_t>(q + 1) * static_cast<size_t>(m * k));
    L.Rband = ar.take<double>(3 * static_cast<size_t>(q + 1) * kk);
    L.Pband = ar.take<double>(static_cast<size_t>(q + 1) * kk);
    L.Tqq = ar.take<double>(kk);
  }
  if (o.save) L.Rsave = ar.take<double>(static_cast<size_t>(q + 1) * kk);
  if (o.resid) {
    L.Wr = ar.take<char>(static_cast<size_t>(d * k) * es);
    L.rpart = ar.take<double>(static_cast<size_t>(ritz_resid_partial_elems(k)));
  }
  if (o.refine) {
    L.Wk = ar.take<float>(static_cast<size_t>(d * k));
    L.Gk = ar.take<double>(kk);
    L.Pk = ar.take<double>(kk);
    L.jk = take_jacobi(ar, k, 0, true);
    // the k x k Rayleigh-Ritz of the correction pass: tridiagonal path
    if (k >= 3 && k <= kTridiagMax)
      L.trik = ar.take<double>(static_cast<size_t>(tridiag_scratch_doubles(k, k)));
  }
  if (csr) {
    if (own_transpose) {
      L.trp = ar.take<int32_t>(static_cast<size_t>(d + 1));
      L.tci = ar.take<int32_t>(static_cast<size_t>(nnz));
      L.tv = ar.take<float>(static_cast<size_t>(nnz));
      L.cursor = ar.take<int32_t>(static_cast<size_t>(d));
      L.tscratch_bytes = csr_transpose_scratch_bytes(nnz, d);
      L.tscratch = ar.take<char>(L.tscratch_bytes);
    }
    const int64_t pmax = csr_max_pieces(nnz, std::max(n, d));
    float* part = ar.take<float>(static_cast<size_t>(pmax) * static_cast<size_t>(k));
    CsrPlan* plans[2] = {&L.plan_a, &L.plan_t};
    const int64_t prow[2] = {n, d};
    for (int i = 0; i < 2; ++i) {
      CsrPlan& pl = *plans[i];
      pl.short_rows = ar.take<int32_t>(static_cast<size_t>(prow[i]));
      pl.piece_row = ar.take<int32_t>(static_cast<size_t>(pmax));
      pl.piece_first = ar.take<int32_t>(static_cast<size_t>(pmax));
      pl.multi_row = ar.take<int32_t>(static_cast<size_t>(pmax));
      pl.multi_first = ar.take<int32_t>(static_cast<size_t>(pmax));
      pl.blk = ar.take<int32_t>(static_cast<size_t>(8 * (csr_plan_chunks(prow[i]) + 1)));
      pl.part = part;
    }
    L.counters = ar.take<int32_t>(8);
    L.colpart = ar.take<double>(static_cast<size_t>(kColsumBlocks) * k);
    L.mu = ar.take<float>(static_cast<size_t>(n));
    L.colvec = ar.take<double>(static_cast<size_t>(k));
    if (o.csr_staged) {
      L.xs = ar.take<float>(static_cast<size_t>(d) * csr_stage_ld(k));
      L.ys = ar.take<float>(static_cast<size_t>(n) * csr_stage_ld(k));
    }
  }
  L.bytes = align_up(ar.off, 256);
  return L;
}

// ---------------------------------------------------------------- timer --
// Events are recycled through a per-thread pool: timing a solve costs one
// hipEventRecord per phase boundary, no creation.
struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e;
      // timing only: no system-scope fence (cache write-back) at each record
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
};
thread_local EventPool g_events;

struct Timer {
  bool on = false;
  int mask = 0;  // phases given events (0: all)
  hipStream_t s = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  int launches[BK_NPHASE] = {0};
  int cur = -1;
  size_t pool_mark = 0;
  hipEvent_t start{};
  void begin(int ph) {
    cur = ph;
    start = nullptr;
    if (!on || (mask != 0 && !(mask & (1 << ph)))) return;
    if (marks.empty()) pool_mark = g_events.used;
    start = g_events.get();
    if (start) (void)hipEventRecord(start, s);
  }
  void end(int nlaunch) {
    if (cur >= 0) launches[cur] += nlaunch;
    if (on && start) {
      hipEvent_t stop = g_events.get();
      if (stop) {
        (void)hipEventRecord(stop, s);
        marks.push_back({cur, {start, stop}});
      }
    }
    cur = -1;
  }
  void collect(bk_info* info) {
    if (!info) return;
    for (int i = 0; i < BK_NPHASE; ++i) {
      info->ms[i] = 0.0f;
      info->launches[i] = launches[i];
    }
    for (auto& mk : marks) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, mk.second.first, mk.second.second) == hipSuccess)
        info->ms[mk.first] += ms;
    }
  }
  ~Timer() {
    // the events go back to the pool once their times have been read (the
    // solve synchronizes the stream before collect())
    if (on && !marks.empty()) g_events.used = pool_mark;
  }
};

// ------------------------------------------------------------ operators --
struct Op {
  int64_t n = 0, d = 0;
  bool f64 = false;
  bool fp32_cores = false;  // FP32 products on the FP32 matrix cores
  double* partial = nullptr;
  int64_t partial_elems = 0;  // (free during ax: split-K scratch)
  Timer* tm = nullptr;
  virtual ~Op() = default;
  // Y (n x k, ldy) = A X, X d x k (ldx)
  virtual void ax(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) = 0;
  // Y (d x k, ldy) = A^T X, X n x k (ldx)
  virtual void aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) = 0;
  // ax for an X that aty produced (the Krylov recurrence): operators that
  // are exact on such inputs without a correction term may skip it
  virtual void ax_of_aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy,
                         hipStream_t s) {
    ax(X, ldx, k, Y, ldy, s);
  }
  // Row weights whose weighted column sums w^T X the next aty needs (null:
  // none), and the block partials of them for the X of that next aty, when
  // the orthonormalization that wrote X formed them (nb x k, consumed once).
  virtual const float* aty_row_weights() const { return nullptr; }
  virtual void set_aty_partials(const double*, int) {}
};

struct DenseOp : Op {
  const void* A = nullptr;
  int64_t lda = 0;
  int a_type = BK_F32;
  const float* ascale = nullptr;
  const void* At = nullptr;  // A^T (d x n) in a_type, for the A^T Y products
  int64_t ld_at = 0;
  const float* atscale = nullptr;
  void* pack = nullptr;  // matrix-core operand packing (nullable)
  size_t pack_bytes = 0;
  void ax(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    tm->begin(BK_PH_AX);
    NNArgs a;
    a.n = n;
    a.K = d;
    a.N = k;
    a.A = A;
    a.lda = lda;
    a.a_type = a_type;
    a.ascale = ascale;
    a.ascale_ld = cdiv(d, 128);
    a.X = X;
    a.ldx = ldx;
    a.x_f64 = f64;
    a.C = Y;
    a.ldc = ldy;
    a.c_f64 = f64;
    a.work = pack;
    a.work_bytes = pack_bytes;
    a.split_work = partial;
    a.split_work_elems = partial_elems;
    a.fp32_cores = fp32_cores;
    tm->end(launch_nn(a, s));
  }
  void aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    tm->begin(BK_PH_ATY);
    if (At) {  // A^T Y as an A X-form product on the transposed copy
      NNArgs a;
      a.n = d;
      a.K = n;
      a.N = k;
      a.A = At;
      a.lda = ld_at;
      a.a_type = a_type;
      a.ascale = atscale;
      a.ascale_ld = cdiv(n, 128);
      a.X = X;
      a.ldx = ldx;
      a.x_f64 = f64;
      a.C = Y;
      a.ldc = ldy;
      a.c_f64 = f64;
      a.work = pack;
      a.work_bytes = pack_bytes;
      a.split_work = partial;
      a.split_work_elems = partial_elems;
      tm->end(launch_nn(a, s));
      return;
    }
    TNArgs a;
    a.L = n;
    a.p = d;
    a.r = k;
    a.X = A;
    a.ldx = lda;
    a.x_type = a_type;
    a.xscale = ascale;
    a.xscale_ld = cdiv(d, 128);
    a.Y = X;
    a.ldy = ldx;
    a.y_f64 = f64;
    a.C = Y;
    a.ldc = ldy;
    a.c_f64 = f64;
    a.partial = partial;
    a.work = pack;
    a.work_bytes = pack_bytes;
    a.fp32_cores = fp32_cores;
    tm->end(launch_tn(a, s));
  }
};

struct CsrOp : Op {
  const int32_t *rp = nullptr, *ci = nullptr, *trp = nullptr, *tci = nullptr;
  const float *v = nullptr, *tv = nullptr;
  const CsrPlan* pa = nullptr;  // work plans of A and A^T
  const CsrPlan* pt = nullptr;
  const float* mu = nullptr;    // row means (centring) or null
  double* colpart = nullptr;    // kColsumBlocks x k
  double* colvec = nullptr;     // k
  // Staged gathers (nullable): the right-hand block of every product is
  // gathered from a copy whose rows start on their own 128-byte lines (one
  // line per gathered row instead of two or three at the Krylov slab's
  // stride, and a smaller footprint in each XCD's L2): xs for A X (d rows),
  // ys for A^T Y (n rows).  The product A^T Y leaves its result in xs too,
  // so that the A X of that result that follows it (ax_of_aty) needs no
  // copy; any other A X copies its block first.
  float* xs = nullptr;
  float* ys = nullptr;
  const void* mirror = nullptr;  // the block whose copy xs holds, or null
  int64_t mirror_ld = 0;
  int mirror_k = 0;
  // Centred products (footnote on PCA, Section 1): with Abar = A - mu 1^T,
  //   Abar X   = A X   - mu (1^T X)    and   Abar^T Y = A^T Y - 1 (mu^T Y),
  // the k-vector (1^T X or mu^T Y) first, then the product with the rank-1
  // correction in its epilogue.
  //
  // X = Abar^T Y has 1^T X = (Abar 1)^T Y = 0 (Abar 1 = A 1 - d mu = 0, mu
  // being the row means), so for such an X the correction of Abar X is zero
  // in exact arithmetic (computed, it is rounding far below the product's
  // own) and is skipped (`exact`).
  void product(const int32_t* r_, const int32_t* c_, const float* v_, const CsrPlan& pl,
               int phase, const void* X, int64_t ldx, int k, void* Y, int64_t ldy,
               const float* rowvec, const float* colw, int64_t Lc, hipStream_t s,
               bool exact = false, const double* part = nullptr, int nb = 0,
               const float* Xg = nullptr, float* Y2 = nullptr) {
    if (exact) rowvec = nullptr;
    if (mu && !exact) {
      tm->begin(BK_PH_CENTER);
      if (part) {  // the partials came with X
        launch_colsum_final(part, nb, k, colvec, s);
        tm->end(1);
      } else {
        launch_colsum(static_cast<const float*>(X), ldx, Lc, k, colw, colpart, colvec, s);
        tm->end(2);
      }
    }
    tm->begin(phase);
    const int kp = csr_stage_ld(k);
    launch_csr_product(pl, r_, c_, v_, k, Xg ? Xg : static_cast<const float*>(X), Lc,
                       Xg ? kp : ldx, static_cast<float*>(Y), ldy, Y2, kp, rowvec,
                       (mu && !exact) ? colvec : nullptr, s);
    tm->end(1);
    if (pl.nmulti > 0) {
      tm->begin(BK_PH_LONG);
      launch_csr_combine(pl, r_, k, static_cast<float*>(Y), ldy, Y2, kp, rowvec,
                         (mu && !exact) ? colvec : nullptr, s);
      tm->end(1);
    }
  }
  // the gather copy of an A X operand (d rows): xs, copied unless it is
  // the result of the A^T Y just before (a_of_aty)
  const float* stage_x(const void* X, int64_t ldx, int k, bool of_aty, hipStream_t s) {
    const bool hit = of_aty && X == mirror && ldx == mirror_ld && k == mirror_k;
    mirror = nullptr;
    if (!xs) return nullptr;
    if (!hit) {
      tm->begin(BK_PH_CENTER);
      launch_csr_stage(static_cast<const float*>(X), ldx, d, k, xs, s);
      tm->end(1);
    }
    return xs;
  }
  const double* pre_part = nullptr;  // block partials of mu^T X for the next aty
  int pre_nb = 0;
  const float* aty_row_weights() const override { return mu; }
  void set_aty_partials(const double* part, int nb) override {
    pre_part = part;
    pre_nb = nb;
  }
  void ax(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    const float* xg = stage_x(X, ldx, k, false, s);
    product(rp, ci, v, *pa, BK_PH_AX, X, ldx, k, Y, ldy, mu, nullptr, d, s, false, nullptr, 0,
            xg);
  }
  void ax_of_aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy,
                 hipStream_t s) override {
    const float* xg = stage_x(X, ldx, k, true, s);
    product(rp, ci, v, *pa, BK_PH_AX, X, ldx, k, Y, ldy, mu, nullptr, d, s, true, nullptr, 0,
            xg);
  }
  void aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    mirror = nullptr;
    if (ys) {
      tm->begin(BK_PH_CENTER);
      launch_csr_stage(static_cast<const float*>(X), ldx, n, k, ys, s);
      tm->end(1);
    }
    product(trp, tci, tv, *pt, BK_PH_ATY, X, ldx, k, Y, ldy, nullptr, mu, n, s, false,
            pre_part, pre_nb, ys, xs);
    pre_part = nullptr;
    if (xs) {
      mirror = Y;
      mirror_ld = ldy;
      mirror_k = k;
    }
  }
};

// The residual R = (I - Z Z^T) Abar of a rank-k projection (Section 3.2),
// whose norms eqs. (1) and (2) measure, as an operator over a base one:
//   R X   = Abar X - Z (Z^T Abar X),    R^T Y = Abar^T (Y - Z (Z^T Y)).
// Its largest singular value, ||Abar - Z Z^T Abar||_2, is then the top Ritz
// value of a block Krylov solve on R.  R^T Y lies in the range of Abar^T, so
// the base operator's ax_of_aty shortcut stays valid.
struct ProjOp : Op {
  Op* base = nullptr;
  const void* Z = nullptr;  // n x kz, working type
  int64_t ldz = 0;
  int kz = 0;
  void* tmp = nullptr;      // n x (block width), ld = block width
  double* C = nullptr;      // kz x (block width) FP64
  void forward_state() {
    base->tm = tm;
    base->partial = partial;
    base->partial_elems = partial_elems;
  }
  // Y (n x k, ldy) -= Z (Z^T Y)
  int project(void* Y, int64_t ldy, int k, hipStream_t s) {
    const int zt = f64 ? BK_F64 : BK_F32;
    TNArgs g;
    g.L = n;
    g.p = kz;
    g.r = k;
    g.X = Z;
    g.ldx = ldz;
    g.x_type = zt;
    g.Y = Y;
    g.ldy = ldy;
    g.y_f64 = f64;
    g.C = C;
    g.ldc = k;
    g.c_f64 = true;
    g.partial = partial;
    int nl = launch_tn(g, s);
    NNArgs a;
    a.n = n;
    a.K = kz;
    a.N = k;
    a.A = Z;
    a.lda = ldz;
    a.a_type = zt;
    a.X = C;
    a.ldx = k;
    a.x_f64 = true;
    a.C = Y;
    a.ldc = ldy;
    a.c_f64 = f64;
    a.alpha = -1.0;
    a.beta = 1.0;
    nl += launch_nn(a, s);
    return nl;
  }
  void ax(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    forward_state();
    base->ax(X, ldx, k, Y, ldy, s);
    tm->begin(BK_PH_PROJ);
    tm->end(project(Y, ldy, k, s));
  }
  void ax_of_aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy,
                 hipStream_t s) override {
    forward_state();
    base->ax_of_aty(X, ldx, k, Y, ldy, s);
    tm->begin(BK_PH_PROJ);
    tm->end(project(Y, ldy, k, s));
  }
  void aty(const void* X, int64_t ldx, int k, void* Y, int64_t ldy, hipStream_t s) override {
    forward_state();
    tm->begin(BK_PH_PROJ);
    launch_copy2d(X, f64, ldx, tmp, f64, k, n, k, s);
    tm->end(1 + project(tmp, k, k, s));
    base->aty(tmp, k, k, Y, ldy, s);
  }
};

// --------------------------------------------------------------- solver --
struct Solver {
  Op* op = nullptr;
  Layout* L = nullptr;
  Options o;
  Timer* tm = nullptr;
  hipStream_t s = nullptr;
  int k = 0, q = 0;
  int64_t n = 0, d = 0, m = 0;
  bool f64 = false;
  size_t es = 4;
  int sweeps = 0;
  double offdiag = 0.0;
  bool noconv = false;

  char* qslab(int i) const { return static_cast<char*>(L->Q) + static_cast<size_t>(i) * k * es; }
  char* wslab(int i) const { return static_cast<char*>(L->W) + static_cast<size_t>(i) * k * es; }
  int wtype() const { return f64 ? BK_F64 : BK_F32; }

  // G (p x r FP64, ld r) = X^T Y, X L x p (ldx), Y L x r (ldy), both the
  // working type.
  int gram(const void* X, int64_t ldx, int64_t p, const void* Y, int64_t ldy,
           int r, int64_t Lrows, double* G, double alpha = 1.0, double beta = 0.0,
           bool sym = false) {
    // a plain symmetric Gram of a long narrow FP32 block (the CholeskyQR
    // Grams): upper 32 x 32 tiles on the matrix cores, FP64 sums of FP32
    // chunk sums, when its partials fit
    if (!f64 && sym && X == Y && ldx == ldy && p == r && alpha == 1.0 && beta == 0.0 &&
        gram_sym_partial_elems(Lrows, r) > 0 &&
        gram_sym_partial_elems(Lrows, r) <= L->partial_elems) {
      const int nl = launch_gram_sym_mfma(Lrows, r, static_cast<const float*>(X), ldx, G, r,
                                          L->partial, s);
      if (nl) return nl;
    }
    TNArgs a;
    a.L = Lrows;
    a.p = p;
    a.r = r;
    a.X = X;
    a.ldx = ldx;
    a.x_type = wtype();
    a.Y = Y;
    a.ldy = ldy;
    a.y_f64 = f64;
    a.C = G;
    a.ldc = r;
    a.c_f64 = true;
    a.alpha = alpha;
    a.beta = beta;
    a.partial = L->partial;
    a.sym = sym && X == Y && ldx == ldy && p == r;
    a.work = L->pack;
    a.work_bytes = L->pack_bytes;
    a.fp32_cores = o.fp32_cores;
    return launch_tn(a, s);
  }
  // C (rows x N, ldc) = alpha A (rows x K, lda) Xf (K x N FP64, ldx) + beta C
  int apply(const void* A, int64_t lda, int64_t rows, int64_t K, const double* Xf,
            int64_t ldx, int N, void* C, int64_t ldc, double alpha, double beta,
            double* gram_partial = nullptr) {
    NNArgs a;
    a.n = rows;
    a.K = K;
    a.N = N;
    a.A = A;
    a.lda = lda;
    a.a_type = wtype();
    a.X = Xf;
    a.ldx = ldx;
    a.x_f64 = true;
    a.C = C;
    a.ldc = ldc;
    a.c_f64 = f64;
    a.alpha = alpha;
    a.beta = beta;
    a.gram_partial = gram_partial;
    if (L) {  // wide applies of an FP32 block on the matrix cores
      a.work = L->pack;
      a.work_bytes = L->pack_bytes;
    }
    a.fp32_cores = o.fp32_cores;
    return launch_nn(a, s);
  }
  // k <= 32: the applies of the orthonormalization also leave the partial
  // Grams of the block they write, so no separate Gram product is needed
  bool fuse_gram() const { return nn_gram_partial_elems(n, k) > 0; }

  // Q slab = orth(B), B (n x k, ld ldb: Bs or the slab itself): shifted
  // CholeskyQR3 (Fukaya et al., SIAM J. Sci. Comput. 2020).  Pass 1 factors
  // G + s I with s = 11 (nk + k(k+1)) u ||B||_F^2 so the FP64 Cholesky cannot
  // fail on an ill-conditioned block; passes 2 and 3 are plain CholeskyQR on
  // the already well-conditioned result.  R_i = R3 R2 R1 (saved for the
  // adjoint).  `gpre` has trace ||B before projection||_F^2 (CHOL_FIRST);
  // with have_gram, L->G already holds B^T B.
  void orth_block(int i, int slab, void* B, int64_t ldb, const double* gpre,
                  bool have_gram = false) {
    tm->begin(BK_PH_CHOLQR);
    const double shift_coef = 11.0 * (static_cast<double>(n) * k + static_cast<double>(k) * (k + 1)) * kUnit64;
    const bool fuse = fuse_gram() && k <= kCqrPassMaxK;
    // B -> Bs2 -> Bs -> slab (B may be the slab); fused: B -> Bs2 -> slab,
    // and the third pass in place, skipped on the device when the second
    // already left the block orthonormal to working precision
    void* bufs[4] = {B, L->Bs2, fuse ? qslab(slab) : L->Bs, qslab(slab)};
    const int64_t lds[4] = {ldb, k, fuse ? m : k, m};
    const double unit = f64 ? 0x1p-53 : 0x1p-24;
    const float* muw = (fuse && !f64) ? op->aty_row_weights() : nullptr;
    int nl = 0;
    // k <= 32: each pass is one launch that adds the previous pass's Gram
    // partials, factors, solves the rows against R (no R^-1) and leaves the
    // partials of the next Gram (two buffers, alternating)
    double* part[2] = {L->partial, L->partial + cqr_pass_partial_elems(k)};
    const double* gin = L->G;
    int P = 1;
    for (int pass = 0; pass < 3; ++pass) {
      void* src = bufs[pass];
      const int64_t ls = lds[pass];
      // block Lanczos keeps every pass's factor (the sub-diagonal blocks)
      double* R = L->Rband ? L->Rband + (3 * static_cast<size_t>(i) + pass) * k * k : L->R;
      if (pass == 0 ? !have_gram : !fuse)
        nl += gram(src, ls, k, src, ls, k, n, L->G, 1.0, 0.0, true);
      const int mode = pass ? CHOL_REPEAT : (i == 0 ? CHOL_FIRST_BLOCK0 : CHOL_FIRST);
      if (fuse) {
        CqrPass a;
        a.n = n;
        a.k = k;
        a.Gin = gin;
        a.P = P;
        a.Gpre = gpre;
        a.mode = mode;
        a.block = i;
        a.tau = o.tau;
        a.shift_coef = shift_coef;
        a.R = R;
        a.ctrl = L->ctrl;
        a.X = src;
        a.ldx = ls;
        a.Y = bufs[pass + 1];
        a.ldy = lds[pass + 1];
        a.f64 = f64;
        a.gout = pass < 2 ? part[pass & 1] : nullptr;
        a.skip_tol = pass == 2 ? 64.0 * unit : 0.0;
        // the last two passes write the final block (the third may skip
        // itself): both leave the partials of mu^T Q_i for the next aty
        if (pass >= 1 && muw) {
          a.mu = muw;
          a.mupart = L->colpart;
        }
        nl += launch_cqr_pass(a, s);
        gin = part[pass & 1];
        P = cqr_pass_grid(n, nullptr);
      } else {
        launch_chol(k, L->G, gpre, mode, i, o.tau, shift_coef, R, L->Rinv, L->cholwork,
                    L->ctrl, s);
        ++nl;
        nl += apply(src, ls, n, k, L->Rinv, k, k, bufs[pass + 1], lds[pass + 1], 1.0, 0.0);
      }
      if (o.save) {
        if (pass == 0) {
          launch_copy2d(R, true, k, L->Racc, true, k, k, k, s);
        } else {
          launch_trmm_upper(k, R, L->Racc, L->Rtmp, s);
          launch_copy2d(L->Rtmp, true, k, L->Racc, true, k, k, k, s);
        }
      }
    }
    if (o.save)
      launch_copy2d(L->Racc, true, k, L->Rsave + static_cast<size_t>(i) * k * k, true, k, k,
                    k, s);
    if (muw) op->set_aty_partials(L->colpart, cqr_pass_grid(n, nullptr));
    tm->end(nl + (o.save ? 6 : 0));
  }

  // B <- (I - Q_<i Q_<i^T) B, twice, for the block B held in Q's slab i (so
  // [Q_<i, B] are the first (i+1)k columns of Q): the first TN product gives
  // C = Q_<i^T B and B^T B (whose trace the breakdown test of the first
  // CholeskyQR pass needs) together.  Returns B^T B (k x k, ld k); with
  // fuse_gram() the last apply also leaves the Gram of the projected block
  // in L->G.
  const double* project(int i) {
    tm->begin(BK_PH_PROJ);
    const int64_t p = static_cast<int64_t>(i) * k;
    void* B = qslab(i);
    const bool fuse = fuse_gram();
    // block Lanczos keeps both passes' coefficients of every block
    double* C1 = L->Cband ? L->Cband + 2 * static_cast<size_t>(i) * m * k : L->C;
    double* C2 = L->Cband ? C1 + static_cast<size_t>(m) * k : L->C;
    int nl = gram(L->Q, m, p + k, B, m, k, n, C1);  // rows p.. : B^T B
    nl += apply(L->Q, m, n, p, C1, k, k, B, m, -1.0, 1.0);
    nl += gram(L->Q, m, p, B, m, k, n, C2);         // rows 0 .. p-1 only
    nl += apply(L->Q, m, n, p, C2, k, k, B, m, -1.0, 1.0, fuse ? L->partial : nullptr);
    if (fuse) nl += launch_gram_reduce(n, k, L->partial, L->G, s);
    tm->end(nl);
    return C1 + p * k;
  }

  // Eigen-solve of the FP64 symmetric PSD `Mat` (mm x mm): top `kk`
  // eigenvectors into Uk (ld ldu) and sqrt(theta) into ritz.
  int eig(const double* Mat, int64_t mm, JacobiWs& jw, int kk, double* Uk, int64_t ldu,
          double* ritz, double* tri = nullptr) {
    if (tri) {  // tridiagonal reduction path: top-k only
      launch_tridiag_topk(Mat, mm, mm, kk, tri, jw.theta, Uk, ldu, ritz, L->ctrl, s);
      BK_TRY_LAUNCH();
      return BK_OK;
    }
    const double tol = jacobi_tol_for(mm, o.jtol);
    const int nb = static_cast<int>(jw.nbp / jw.b);
    launch_jacobi_init(Mat, mm, mm, jw.Xc, jw.Vc, jw.ldc, jw.nbp, s);
    bool conv = false;
    int sw = 0;
    double off = 0.0;
    for (sw = 1; sw <= o.max_sweeps; ++sw) {
      launch_ctrl_reset_off(L->ctrl, s);
      for (int r = 0; r < nb - 1; ++r)
        // one inner sweep per round: full inner convergence buys no outer
        // sweeps (measured on the Rayleigh-Ritz matrices of the workloads)
        launch_jacobi_round(jw.b, mm, nb, r, jw.Xc, jw.Vc, jw.ldc, tol, 1, L->ctrl, s);
      Ctrl h;
      BK_TRY(hipMemcpyAsync(&h, L->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
      BK_TRY(hipStreamSynchronize(s));
      long long bits = static_cast<long long>(h.offmax);
      std::memcpy(&off, &bits, sizeof(off));
      if (off <= tol) {
        conv = true;
        break;
      }
    }
    sweeps += std::min(sw, o.max_sweeps);
    offdiag = off;
    if (!conv) noconv = true;
    launch_jacobi_finalize(jw.Xc, jw.Vc, jw.ldc, mm, kk, jw.theta, jw.order, jw.norms, Uk,
                           ldu, ritz, s);
    BK_TRY_LAUNCH();
    return BK_OK;
  }

};

// refine: 0 = default (on for the BF16 / FP8 copies when an FP32 master is
// given), > 0 on, < 0 off; never for the plain FP32 / FP64 paths.
void normalize_refine(Options& o, int a_type, bool has_master) {
  const bool lowp = a_type == BK_BF16 || a_type == BK_FP8_E4M3;
  if (!lowp) o.refine = 0;
  else if (o.refine == 0) o.refine = has_master ? 1 : 0;
  else o.refine = o.refine > 0 ? 1 : 0;
}

int finish_status(const Ctrl& h, bool noconv) {
  if (h.flags & CTRL_STALL) return BK_EHIP;
  if (h.flags & CTRL_NONFINITE) return BK_ENONFINITE;
  if (h.flags & CTRL_RANK) return BK_ERANK;
  if (noconv) return BK_ENOCONV;
  return BK_OK;
}

// The whole solve for an operator; Z is FP64 when op->f64, else FP32.
int solve(Op& op, Layout& L, const Options& o, int k, int q, uint64_t seed,
          const DenseOp* master, void* Z, int64_t ldz, double* ritz, bk_info* info,
          hipStream_t s) {
  Timer tm;
  tm.on = o.timing != 0;
  tm.mask = o.timing_phases;
  tm.s = s;
  op.tm = &tm;
  op.partial = L.partial;
  op.partial_elems = L.partial_elems;
  if (DenseOp* dop = dynamic_cast<DenseOp*>(&op)) {
    dop->pack = L.pack;
    dop->pack_bytes = L.pack_bytes;
  }
  Solver S;
  S.op = &op;
  S.L = &L;
  S.o = o;
  S.tm = &tm;
  S.s = s;
  // p: width of the sketch and of every block (p >= k, Section 6); the
  // Rayleigh-Ritz step below returns the top k
  const int pw = o.p > 0 ? o.p : k;
  S.k = pw;
  S.q = q;
  S.n = op.n;
  S.d = op.d;
  S.f64 = op.f64;
  S.es = op.f64 ? 8 : 4;
  S.m = o.si ? pw : static_cast<int64_t>(q + 1) * pw;
  const int64_t n = op.n, d = op.d, m = S.m;
  const bool f64 = op.f64;

  launch_ctrl_init(L.ctrl, q, s);
  // Step 1: the sketch.
  tm.begin(BK_PH_PI);
  if (o.pi)
    launch_copy2d(o.pi, f64, pw, L.Pi, f64, pw, d, pw, s);
  else
    launch_gaussian(seed, d, pw, pw, f64, L.Pi, s);
  tm.end(1);

  // Step 2-3: Krylov blocks, orthonormalized as they are formed.
  op.ax(L.Pi, pw, pw, L.Bs, pw, s);
  S.orth_block(0, 0, L.Bs, pw, L.Gpre);
  if (!o.si) {
    for (int i = 1; i <= q; ++i) {
      op.aty(S.qslab(i - 1), m, pw, S.wslab(i - 1), m, s);
      op.ax_of_aty(S.wslab(i - 1), m, pw, S.qslab(i), m, s);  // the block in its slab
      const double* gpre = S.project(i);
      S.orth_block(i, i, S.qslab(i), m, gpre, S.fuse_gram());
    }
    op.aty(S.qslab(q), m, pw, S.wslab(q), m, s);
  } else {
    // Algorithm 1: the single block is replaced by orth(A A^T block)
    for (int i = 1; i <= q; ++i) {
      op.aty(S.qslab(0), m, pw, S.wslab(0), m, s);
      op.ax_of_aty(S.wslab(0), m, pw, L.Bs, pw, s);
      tm.begin(BK_PH_PROJ);
      const int nl = S.gram(L.Bs, pw, pw, L.Bs, pw, pw, n, L.Gpre);  // trace for the breakdown test
      tm.end(nl);
      S.orth_block(i, 0, L.Bs, pw, L.Gpre);
    }
    op.aty(S.qslab(0), m, pw, S.wslab(0), m, s);
  }
  BK_TRY_LAUNCH();

  // Step 4: M = W^T W = Q^T A A^T Q in FP64.
  tm.begin(BK_PH_M);
  int mlaunch = 0;
  if (L.Cband) {
    // block Lanczos: the block-tridiagonal T from the recurrence's own
    // coefficients; only the last diagonal block needs a product
    mlaunch = S.gram(S.wslab(q), m, pw, S.wslab(q), m, pw, d, L.Tqq, 1.0, 0.0, true);
    mlaunch += launch_block_tridiag(m, pw, q, L.Cband, m * pw, L.Rband, L.Pband, L.Tqq, L.M, m,
                                    s);
  } else {
    // narrow FP32 W: matrix-core tiles of the upper triangle
    mlaunch = f64 ? 0
                  : launch_gram_sym_mfma(d, static_cast<int>(m), static_cast<const float*>(L.W),
                                         m, L.M, m, L.partial, s);
    if (!mlaunch)
      mlaunch = S.gram(L.W, m, m, L.W, m, static_cast<int>(m), d, L.M, 1.0, 0.0, true);
  }
  tm.end(mlaunch);
  BK_TRY_LAUNCH();

  // Step 5: top-k eigenpairs of M.
  tm.begin(BK_PH_EIG);
  int st = S.eig(L.M, m, L.jw, k, L.Uk, k, L.ritz_dev, L.tri);
  tm.end(0);
  if (st != BK_OK) return st;

  // Step 6: Z = Q U_k.
  tm.begin(BK_PH_Z);
  S.apply(L.Q, m, n, m, L.Uk, k, k, Z, ldz, 1.0, 0.0);
  launch_sign_normalize(Z, f64, n, k, ldz, L.Uk, m, k, L.sign, s);
  tm.end(3);
  BK_TRY_LAUNCH();

  // Correction pass: Rayleigh-Ritz on span(Z) with the FP32 master copy.
  if (o.refine && master) {
    tm.begin(BK_PH_REFINE);
    DenseOp mop = *master;
    mop.partial = L.partial;
    mop.pack = L.pack;
    mop.pack_bytes = L.pack_bytes;
    Timer dummy;
    mop.tm = &dummy;
    mop.aty(Z, ldz, k, L.Wk, k, s);  // W_k = A^T Z (FP32 master)
    TNArgs g;
    g.L = d;
    g.p = k;
    g.r = k;
    g.X = L.Wk;
    g.ldx = k;
    g.x_type = BK_F32;
    g.Y = L.Wk;
    g.ldy = k;
    g.y_f64 = false;
    g.C = L.Gk;
    g.ldc = k;
    g.c_f64 = true;
    g.partial = L.partial;
    g.work = L.pack;
    g.work_bytes = L.pack_bytes;
    g.fp32_cores = o.fp32_cores;
    launch_tn(g, s);
    tm.end(4);
    st = S.eig(L.Gk, k, L.jk, k, L.Pk, k, L.ritz_dev, L.trik);
    if (st != BK_OK) return st;
    tm.begin(BK_PH_REFINE);
    S.apply(Z, ldz, n, k, L.Pk, k, k, L.Bs, k, 1.0, 0.0);
    launch_copy2d(L.Bs, false, k, Z, false, ldz, n, k, s);
    launch_sign_normalize(Z, false, n, k, ldz, nullptr, 0, 0, L.sign, s);
    tm.end(4);
    BK_TRY_LAUNCH();
  }

  // Residual norms r_i = ||A A^T z_i - sigma_i^2 z_i|| of the returned pairs
  // (Bauer-Fike certificate of Lemma 1's Ritz values): W_r = A^T Z -- after
  // the correction pass that is W_k P, already formed with the FP32 master
  // -- then R = A W_r and the column norms of R - Z diag(sigma^2).
  if (o.resid) {
    tm.begin(BK_PH_REFINE);
    int nl = 0;
    Op* rop = &op;
    DenseOp mop;
    Timer dummy;
    // the correction pass signed Z after forming W_k: R then carries the
    // columns before those signs
    const double* rsign = (o.refine && master) ? L.sign : nullptr;
    if (o.refine && master) {
      mop = *master;
      mop.partial = L.partial;
      mop.partial_elems = L.partial_elems;
      mop.pack = L.pack;
      mop.pack_bytes = L.pack_bytes;
      mop.tm = &dummy;
      rop = &mop;
      nl += S.apply(L.Wk, k, d, k, L.Pk, k, k, L.Wr, k, 1.0, 0.0);
    } else {
      rop->aty(Z, ldz, k, L.Wr, k, s);
      ++nl;
    }
    rop->ax_of_aty(L.Wr, k, k, L.Bs, k, s);
    launch_ritz_resid(L.Bs, k, Z, ldz, f64, n, k, L.ritz_dev, rsign, L.rpart, o.resid, s);
    tm.end(nl + 3);
    BK_TRY_LAUNCH();
  }

  launch_copy2d(L.ritz_dev, true, 1, ritz, true, 1, k, 1, s);
  Ctrl h;
  BK_TRY(hipMemcpyAsync(&h, L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  BK_TRY_LAUNCH();
  if (info) {
    tm.collect(info);
    info->q_eff = h.q_eff;
    info->jacobi_sweeps = S.sweeps;
    info->jacobi_offdiag = S.offdiag;
    info->workspace_bytes = static_cast<int64_t>(L.bytes);
  }
  return finish_status(h, S.noconv);
}

// ------------------------------------------------------------- adjoint --
// Reverse mode of the forward above for the plain FP32 / FP64 paths, for a
// loss L(Z, sigma) unchanged by rotations inside span(Z).  With the thin-QR
// adjoint (Q_i R_i = P_i, R_i unused elsewhere):
//   P_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T
// the projection P_i = (I - Q_< Q_<^T) B_i:
//   B_bar = P_bar - Q_< (Q_<^T P_bar),  Q_<bar -= P_bar C^T + B (Q_<^T P_bar)^T
// the symmetric eigen-decomposition M = U diag(theta) U^T:
//   M_bar = sym(U [diag(theta_bar) + F o (U^T U_bar)] U^T),
//   F_ij = 1 / (theta_j - theta_i), zero inside the top-k block
// and W = A^T Q, M = W^T W, B_i = A Y_i, Y_i = A^T Q_{i-1}.  B_i is recomputed
// from the saved Y_i; A_bar is gathered as two n x d x m products.
struct BwdLayout {
  double* partial = nullptr;
  void *Qbar = nullptr, *Wbar = nullptr, *Bbar = nullptr, *Bi = nullptr, *Pbar = nullptr,
       *RtA = nullptr, *RtB = nullptr;
  double *Ufull = nullptr, *Ubk = nullptr, *UkT = nullptr, *H = nullptr, *Gk = nullptr,
         *T1 = nullptr, *Mbar = nullptr, *S = nullptr, *Cu = nullptr, *RinvT = nullptr,
         *work = nullptr, *D = nullptr, *C = nullptr, *DT = nullptr, *CT = nullptr;
  size_t bytes = 0;
};

BwdLayout make_bwd_layout(char* base, int64_t n, int64_t d, int k, int q, bool f64) {
  Arena ar;
  ar.base = base;
  BwdLayout B;
  const size_t es = f64 ? 8 : 4;
  const int64_t m = static_cast<int64_t>(q + 1) * k;
  int64_t need = std::max<int64_t>(tn_partial_elems(n, m, k), tn_partial_elems(m, m, k));
  need = std::max(need, tn_partial_elems(n, k, k));
  need = std::max(need, tn_partial_elems(n, d, k));
  for (int i = 1; i <= q; ++i) need = std::max(need, tn_partial_elems(n, static_cast<int64_t>(i) * k, k));
  B.partial = ar.take<double>(static_cast<size_t>(need));
  B.Qbar = ar.take<char>(static_cast<size_t>(n * m) * es);
  B.Wbar = ar.take<char>(static_cast<size_t>(d * m) * es);
  B.Bbar = ar.take<char>(static_cast<size_t>(n * m) * es);
  B.Bi = ar.take<char>(static_cast<size_t>(n * k) * es);
  B.Pbar = ar.take<char>(static_cast<size_t>(n * k) * es);
  B.RtA = ar.take<char>(static_cast<size_t>(m * d) * es);
  B.RtB = ar.take<char>(static_cast<size_t>(m * d) * es);
  const size_t mm = static_cast<size_t>(m) * m, mk = static_cast<size_t>(m) * k,
               kk = static_cast<size_t>(k) * k;
  B.Ufull = ar.take<double>(mm);
  B.Mbar = ar.take<double>(mm);
  B.Ubk = ar.take<double>(mk);
  B.UkT = ar.take<double>(mk);
  B.H = ar.take<double>(mk);
  B.Gk = ar.take<double>(mk);
  B.T1 = ar.take<double>(mk);
  B.D = ar.take<double>(mk);
  B.C = ar.take<double>(mk);
  B.DT = ar.take<double>(mk);
  B.CT = ar.take<double>(mk);
  B.S = ar.take<double>(kk);
  B.Cu = ar.take<double>(kk);
  B.RinvT = ar.take<double>(kk);
  B.work = ar.take<double>(kk);
  B.bytes = align_up(ar.off, 256);
  return B;
}

Options backward_fwd_options(bool f64) {
  Options o;
  o.save = 1;
  o.tau = f64 ? 1e-11 : 1e-5;
  return o;
}

int backward_dense(const DenseOp& op, int k, int q, const Layout& F, const BwdLayout& B,
                   const void* Zbar, int64_t ldzb, const double* ritz_bar, void* Abar,
                   int64_t ld_bar, hipStream_t s) {
  const int64_t n = op.n, d = op.d, m = static_cast<int64_t>(q + 1) * k;
  const bool f64 = op.f64;
  const size_t es = f64 ? 8 : 4;
  const int wt = f64 ? BK_F64 : BK_F32;
  auto slab = [&](void* base, int i) {
    return static_cast<char*>(base) + static_cast<size_t>(i) * k * es;
  };
  auto cslab = [&](const void* base, int i) {
    return static_cast<const char*>(base) + static_cast<size_t>(i) * k * es;
  };
  // C (rows x N) = alpha A (rows x K) X (K x N) + beta C; xf64 marks X FP64
  auto nn = [&](const void* A, int atype, int64_t lda, int64_t rows, int64_t K, const void* X,
                bool xf64, int64_t ldx, int N, void* C, bool cf64, int64_t ldc, double alpha,
                double beta) {
    NNArgs a;
    a.n = rows;
    a.K = K;
    a.N = N;
    a.A = A;
    a.lda = lda;
    a.a_type = atype;
    a.X = X;
    a.ldx = ldx;
    a.x_f64 = xf64;
    a.C = C;
    a.ldc = ldc;
    a.c_f64 = cf64;
    a.alpha = alpha;
    a.beta = beta;
    launch_nn(a, s);
  };
  // C (p x r) = alpha X^T Y + beta C, X rows x p, Y rows x r
  auto tn = [&](const void* X, int xtype, int64_t ldx, int64_t rows, int64_t p, const void* Y,
                bool yf64, int64_t ldy, int r, void* C, bool cf64, int64_t ldc, double beta) {
    TNArgs a;
    a.L = rows;
    a.p = p;
    a.r = r;
    a.X = X;
    a.ldx = ldx;
    a.x_type = xtype;
    a.Y = Y;
    a.ldy = ldy;
    a.y_f64 = yf64;
    a.C = C;
    a.ldc = ldc;
    a.c_f64 = cf64;
    a.beta = beta;
    a.partial = B.partial;
    launch_tn(a, s);
  };

  Ctrl h;
  BK_TRY(hipMemcpyAsync(&h, F.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  if (h.flags) return BK_EINVAL;  // the forward did not succeed
  const int qe = std::min(std::max(h.q_eff, 0), q);

  // Eigenvectors in the forward's order and signs; U_k^T.
  launch_gather_vectors(F.jw.Vc, F.jw.ldc, m, F.jw.order, F.sign, k, B.Ufull, s);
  launch_transpose(F.Uk, true, k, B.UkT, true, m, m, k, s);
  // Z = Q U_k:  U_k_bar = Q^T Z_bar,  Q_bar = Z_bar U_k^T.
  if (Zbar) {
    tn(F.Q, wt, m, n, m, Zbar, f64, ldzb, k, B.Ubk, true, k, 0.0);
    nn(Zbar, wt, ldzb, n, k, B.UkT, true, m, static_cast<int>(m), B.Qbar, f64, m, 1.0, 0.0);
  } else {
    launch_fill_f64(B.Ubk, m * k, 0.0, s);
    if (f64) launch_fill_f64(static_cast<double*>(B.Qbar), n * m, 0.0, s);
    else launch_fill_f32(static_cast<float*>(B.Qbar), n * m, 0.0f, s);
  }
  // M_bar = sym(U G U_k^T),  G = diag(theta_bar) + F o (U^T U_k_bar).
  tn(B.Ufull, BK_F64, m, m, m, B.Ubk, true, k, k, B.H, true, k, 0.0);
  launch_eig_adjoint(m, k, F.jw.theta, B.H, F.ritz_dev, ritz_bar, B.Gk, s);
  nn(B.Ufull, BK_F64, m, m, m, B.Gk, true, k, k, B.T1, true, k, 1.0, 0.0);
  nn(B.T1, BK_F64, k, m, k, B.UkT, true, m, static_cast<int>(m), B.Mbar, true, m, 1.0, 0.0);
  launch_symmetrize(m, B.Mbar, s);
  // W_bar = 2 W M_bar  (W = [Y_1 .. Y_{q+1}]).
  nn(F.W, wt, m, d, m, B.Mbar, true, m, static_cast<int>(m), B.Wbar, f64, m, 2.0, 0.0);
  // B_bar slots: i - 1 for block i >= 1, q for block 0; unused ones stay 0.
  if (f64) launch_fill_f64(static_cast<double*>(B.Bbar), n * m, 0.0, s);
  else launch_fill_f32(static_cast<float*>(B.Bbar), n * m, 0.0f, s);
  // Y_{qe+1} = A^T Q_qe feeds only W:  Q_qe_bar += A W_bar_qe.
  nn(op.A, op.a_type, op.lda, n, d, cslab(B.Wbar, qe), f64, m, k, slab(B.Qbar, qe), f64, m,
     1.0, 1.0);
  BK_TRY_LAUNCH();

  for (int i = qe; i >= 0; --i) {
    void* Qbi = slab(B.Qbar, i);
    const void* Qi = cslab(F.Q, i);
    // thin-QR adjoint: P_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T
    tn(Qbi, wt, m, n, k, Qi, f64, m, k, B.S, true, k, 0.0);
    launch_copyltu_neg(k, B.S, B.Cu, s);
    nn(Qi, wt, m, n, k, B.Cu, true, k, k, Qbi, f64, m, 1.0, 1.0);
    launch_trinv_t(k, F.Rsave + static_cast<size_t>(i) * k * k, B.work, B.RinvT, s);
    nn(Qbi, wt, m, n, k, B.RinvT, true, k, k, B.Pbar, f64, k, 1.0, 0.0);
    if (i == 0) {  // B_0 = A Pi: A_bar += P_bar Pi^T
      launch_copy2d(B.Pbar, f64, k, slab(B.Bbar, q), f64, m, n, k, s);
      break;
    }
    // recompute B_i = A Y_i from the saved Y_i
    nn(op.A, op.a_type, op.lda, n, d, cslab(F.W, i - 1), f64, m, k, B.Bi, f64, k, 1.0, 0.0);
    const int64_t p = static_cast<int64_t>(i) * k;
    // projection adjoint, C = Q_<^T B_i and D = Q_<^T P_bar
    tn(F.Q, wt, m, n, p, B.Bi, f64, k, k, B.C, true, k, 0.0);
    tn(F.Q, wt, m, n, p, B.Pbar, f64, k, k, B.D, true, k, 0.0);
    launch_transpose(B.C, true, k, B.CT, true, p, p, k, s);
    launch_transpose(B.D, true, k, B.DT, true, p, p, k, s);
    nn(B.Pbar, wt, k, n, k, B.CT, true, p, static_cast<int>(p), B.Qbar, f64, m, -1.0, 1.0);
    nn(B.Bi, wt, k, n, k, B.DT, true, p, static_cast<int>(p), B.Qbar, f64, m, -1.0, 1.0);
    nn(F.Q, wt, m, n, p, B.D, true, k, k, B.Pbar, f64, k, -1.0, 1.0);  // -> B_bar_i
    launch_copy2d(B.Pbar, f64, k, slab(B.Bbar, i - 1), f64, m, n, k, s);
    // B_i = A Y_i:   Y_bar_i = W_bar_{i-1} + A^T B_bar_i
    tn(op.A, op.a_type, op.lda, n, d, B.Pbar, f64, k, k, slab(B.Wbar, i - 1), f64, m, 1.0);
    // Y_i = A^T Q_{i-1}:   Q_bar_{i-1} += A Y_bar_i
    nn(op.A, op.a_type, op.lda, n, d, cslab(B.Wbar, i - 1), f64, m, k, slab(B.Qbar, i - 1), f64,
       m, 1.0, 1.0);
    BK_TRY_LAUNCH();
  }
  // A_bar = Q [Y_bar_1 .. Y_bar_{q+1}]^T + [B_bar_1 .. B_bar_q, B_bar_0] [Y_1 .. Y_q, Pi]^T
  launch_transpose(B.Wbar, f64, m, B.RtA, f64, d, d, m, s);
  if (q > 0) launch_transpose(F.W, f64, m, B.RtB, f64, d, d, static_cast<int64_t>(q) * k, s);
  launch_transpose(F.Pi, f64, k, static_cast<char*>(B.RtB) + static_cast<size_t>(q) * k * d * es,
                   f64, d, d, k, s);
  nn(F.Q, wt, m, n, m, B.RtA, f64, d, static_cast<int>(d), Abar, f64, ld_bar, 1.0, 0.0);
  nn(B.Bbar, wt, m, n, m, B.RtB, f64, d, static_cast<int>(d), Abar, f64, ld_bar, 1.0, 1.0);
  BK_TRY_LAUNCH();
  BK_TRY(hipStreamSynchronize(s));
  return BK_OK;
}

bool valid_kq(int64_t n, int64_t d, int32_t k, int32_t q) {
  if (n <= 0 || d <= 0 || k < 1 || q < 0) return false;
  if (k > std::min(n, d)) return false;
  if (static_cast<int64_t>(q + 1) * k > std::min(n, d)) return false;
  return true;
}

// Block width of a solve (Section 6 oversampling): p >= k; the Krylov space
// has (q+1) p columns, or p for simultaneous iteration.  0 on invalid input.
int32_t block_width(int64_t n, int64_t d, int32_t k, int32_t q, const Options& o) {
  if (n <= 0 || d <= 0 || k < 1 || q < 0 || o.p < 0) return 0;
  const int32_t p = o.p > 0 ? o.p : k;
  if (p < k || p > std::min(n, d)) return 0;
  if (!o.si && static_cast<int64_t>(q + 1) * p > std::min(n, d)) return 0;
  if (o.save && (p != k || o.si || o.bl)) return 0;
  return p;
}

struct DevBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~DevBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

// The CSR solve's preparation: the structure check (before any kernel
// indexes through it), the CSR of A^T unless given, the work plans of both
// products for block width pw, the row means (centring); then
// run(op, L, extra): extra is `extra_bytes` of the workspace after the
// layout.
template <typename Run>
int csr_prepare_and_run(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                        const int32_t* t_row_ptr, const int32_t* t_col_idx, const float* t_vals,
                        int64_t n, int64_t d, int64_t nnz, int32_t pw, int32_t q,
                        const Options& o, void* workspace, size_t workspace_bytes,
                        size_t extra_bytes, bk_info* info, hipStream_t s, Run run) {
  const bool given_t = t_row_ptr && t_col_idx && t_vals;
  const size_t lay =
      align_up(make_layout(nullptr, n, d, nnz, pw, q, false, o, true, !given_t).bytes, 256);
  const size_t need = lay + extra_bytes;
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  Layout L = make_layout(base, n, d, nnz, pw, q, false, o, true, !given_t);

  Timer prep;
  prep.on = o.timing != 0;
  prep.mask = o.timing_phases;
  prep.s = s;
  prep.begin(BK_PH_PREP);
  // Validate the structure before any kernel indexes through it.
  launch_ctrl_init(L.ctrl, q, s);
  launch_csr_validate(row_ptr, col_idx, n, d, nnz, L.ctrl, s);
  if (given_t) launch_csr_validate(t_row_ptr, t_col_idx, d, n, nnz, L.ctrl, s);
  Ctrl h;
  BK_TRY(hipMemcpyAsync(&h, L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  BK_TRY_LAUNCH();
  if (h.csr_bad) return BK_EINVAL;
  const int32_t* trp = t_row_ptr;
  const int32_t* tci = t_col_idx;
  const float* tv = t_vals;
  if (!given_t) {
    if (launch_csr_transpose(row_ptr, col_idx, vals, n, d, nnz, L.trp, L.tci, L.tv, L.cursor,
                             L.tscratch, L.tscratch_bytes, s) != 0)
      return BK_EHIP;
    trp = L.trp;
    tci = L.tci;
    tv = L.tv;
  }
  launch_csr_plan(row_ptr, n, pw, L.plan_a, L.counters, s);
  launch_csr_plan(trp, d, pw, L.plan_t, L.counters + 4, s);
  if (o.center) launch_csr_row_means(row_ptr, vals, n, d, L.mu, s);
  int32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  BK_TRY(hipMemcpyAsync(cnt, L.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  BK_TRY_LAUNCH();
  L.plan_t.operand = 1;
  CsrPlan* plans[2] = {&L.plan_a, &L.plan_t};
  for (int i = 0; i < 2; ++i) {
    plans[i]->nshort = cnt[4 * i];
    plans[i]->npieces = cnt[4 * i + 1];
    plans[i]->nmulti = cnt[4 * i + 2];
    plans[i]->short_nnz = cnt[4 * i + 3];
  }
  prep.end(0);

  CsrOp op;
  op.n = n;
  op.d = d;
  op.f64 = false;
  op.rp = row_ptr;
  op.ci = col_idx;
  op.v = vals;
  op.trp = trp;
  op.tci = tci;
  op.tv = tv;
  op.pa = &L.plan_a;
  op.pt = &L.plan_t;
  op.mu = o.center ? L.mu : nullptr;
  op.colpart = L.colpart;
  op.colvec = L.colvec;
  op.xs = L.xs;
  op.ys = L.ys;
  const int st = run(op, L, base + lay);
  if (info && o.timing) {
    float ms = 0.0f;
    if (!prep.marks.empty())
      (void)hipEventElapsedTime(&ms, prep.marks[0].second.first, prep.marks[0].second.second);
    info->ms[BK_PH_PREP] += ms;
  }
  return st;
}

size_t csr_workspace_bytes(int64_t n, int64_t d, int64_t nnz, int32_t pw, int32_t q,
                           const Options& o, bool own_transpose, size_t extra_bytes) {
  return align_up(make_layout(nullptr, n, d, nnz, pw, q, false, o, true, own_transpose).bytes,
                  256) +
         extra_bytes;
}

// ------------------------------------------------------ error measures --
struct MetricsWs {
  void* tmp = nullptr;   // n x k working type: R^T's projected operand
  double* C = nullptr;   // k x k FP64: Z^T Y of the projection
  void* W = nullptr;     // d x k working type: Abar^T Z
  double* G = nullptr;   // k x k FP64: W^T W
  double* part = nullptr;
  double* fro2 = nullptr;
  void* zs = nullptr;    // n working type: top left singular vector of R
  double* rs = nullptr;  // its singular value
  size_t bytes = 0;
};

MetricsWs make_metrics_ws(char* base, int64_t n, int64_t d, int k, bool f64) {
  Arena ar;
  ar.base = base;
  MetricsWs w;
  const size_t es = f64 ? 8 : 4;
  const size_t kk = static_cast<size_t>(k) * k;
  w.tmp = ar.take<char>(static_cast<size_t>(n) * k * es);
  w.C = ar.take<double>(kk);
  w.W = ar.take<char>(static_cast<size_t>(d) * k * es);
  w.G = ar.take<double>(kk);
  w.part = ar.take<double>(
      static_cast<size_t>(std::max(fro2_partial_elems(), tn_partial_elems(d, k, k))));
  w.fro2 = ar.take<double>(1);
  w.zs = ar.take<char>(static_cast<size_t>(n) * es);
  w.rs = ar.take<double>(1);
  w.bytes = align_up(ar.off, 256);
  return w;
}

// The error measures of Z (n x k, orthonormal columns) against Abar:
//   ||Abar||_F^2 (the `fro2` launcher), captured_i = ||Abar^T z_i||^2 =
//   z_i^T Abar Abar^T z_i (the diagonal of W^T W, W = Abar^T Z), the
//   Frobenius residual by the Pythagorean identity of Section 3.2, and the
//   spectral residual as the top Ritz value of a depth-q_spec block Krylov
//   solve (block width k) on R = (I - Z Z^T) Abar.  The ratios of eqs.
//   (1)-(3) follow from sigma (host, n_sigma >= k + 1 values) when given.
// L is a solve layout for block width k and depth q_spec over `op`.
template <typename Fro2>
int metrics_run(Op& op, Layout& L, const MetricsWs& w, const void* Z, int64_t ldz, int k,
                int q_spec, uint64_t seed, const double* sigma, int64_t n_sigma,
                double* captured, bk_metrics* out, hipStream_t s, Fro2 fro2) {
  const bool f64 = op.f64;
  Timer off;
  op.tm = &off;
  op.partial = L.partial;
  op.partial_elems = L.partial_elems;
  fro2(w.part, w.fro2);
  op.aty(Z, ldz, k, w.W, k, s);
  TNArgs g;
  g.L = op.d;
  g.p = k;
  g.r = k;
  g.X = w.W;
  g.ldx = k;
  g.x_type = f64 ? BK_F64 : BK_F32;
  g.Y = w.W;
  g.ldy = k;
  g.y_f64 = f64;
  g.C = w.G;
  g.ldc = k;
  g.c_f64 = true;
  g.partial = w.part;
  g.sym = true;
  launch_tn(g, s);
  std::vector<double> G(static_cast<size_t>(k) * k);
  double f2 = 0.0;
  BK_TRY(hipMemcpyAsync(G.data(), w.G, G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  BK_TRY(hipMemcpyAsync(&f2, w.fro2, sizeof(double), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  BK_TRY_LAUNCH();

  ProjOp pop;
  pop.n = op.n;
  pop.d = op.d;
  pop.f64 = f64;
  pop.base = &op;
  pop.Z = Z;
  pop.ldz = ldz;
  pop.kz = k;
  pop.tmp = w.tmp;
  pop.C = w.C;
  Options so;
  so.p = k;
  so.tau = f64 ? 1e-11 : 1e-5;
  const int st = solve(pop, L, so, 1, q_spec, seed, nullptr, w.zs, 1, w.rs, nullptr, s);
  if (st != BK_OK && st != BK_ERANK) return st;
  // BK_ERANK: R Pi is rank deficient (R of rank below k); the spectral
  // residual is then left unestimated (NaN)
  double rs = std::numeric_limits<double>::quiet_NaN();
  if (st == BK_OK) {
    BK_TRY(hipMemcpyAsync(&rs, w.rs, sizeof(double), hipMemcpyDeviceToHost, s));
    BK_TRY(hipStreamSynchronize(s));
  }

  const double nan = std::numeric_limits<double>::quiet_NaN();
  double csum = 0.0;
  for (int i = 0; i < k; ++i) {
    const double c = G[static_cast<size_t>(i) * k + i];
    csum += c;
    if (captured) captured[i] = c;
  }
  bk_metrics m;
  m.fro2 = f2;
  m.captured_fro2 = csum;
  m.resid_fro = std::sqrt(std::max(f2 - csum, 0.0));
  m.resid_spec = rs;
  m.fro_ratio = m.spec_ratio = m.per_vector = nan;
  if (sigma && n_sigma >= k + 1) {
    double head = 0.0, tail = 0.0, pv = 0.0;
    for (int i = 0; i < k; ++i) head += sigma[i] * sigma[i];
    if (n_sigma >= std::min(op.n, op.d))
      for (int64_t i = k; i < n_sigma; ++i) tail += sigma[i] * sigma[i];
    else
      tail = f2 - head;  // ||Abar - Abar_k||_F^2 = ||Abar||_F^2 - sum_{i<=k} sigma_i^2
    const double sk1 = sigma[k];
    for (int i = 0; i < k; ++i)
      pv = std::max(pv, std::fabs(sigma[i] * sigma[i] - G[static_cast<size_t>(i) * k + i]));
    if (tail > 0.0) m.fro_ratio = m.resid_fro / std::sqrt(tail);
    if (sk1 > 0.0) {
      m.spec_ratio = rs / sk1;
      m.per_vector = pv / (sk1 * sk1);
    }
  }
  if (out) *out = m;
  return st;
}

}  // namespace
}  // namespace bk

using namespace bk;

// ------------------------------------------------ allocation-free solve --
// The scratch of bk_svd_dense_noalloc: one static array per GPU the library
// runs on (the code object's global, allocated when the module is loaded on
// that device).  In host code `scratch` names a host-side stand-in, not a
// device address, so it is never passed to a kernel or a copy: the device
// address comes from hipGetSymbolAddress, looked up once per device with
// that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[BK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;

struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxScratchDevices];

// Device address of `scratch` on the device of stream s (nullptr on error).
void* scratch_address(hipStream_t s) {
  int dev = 0;
  if (s) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess) return nullptr;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  ScratchSlot& slot = g_scratch[dev];
  std::call_once(slot.once, [&] {
    int cur = 0;
    slot.err = hipGetDevice(&cur);
    if (slot.err != hipSuccess) return;
    if (cur != dev && (slot.err = hipSetDevice(dev)) != hipSuccess) return;
    void* p = nullptr;
    slot.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (slot.err == hipSuccess) slot.ptr = p;
    if (cur != dev) (void)hipSetDevice(cur);
  });
  return slot.err == hipSuccess ? slot.ptr : nullptr;
}

}  // namespace

extern "C" {

const char* bk_status_string(int status) {
  switch (status) {
    case BK_OK: return "ok";
    case BK_EINVAL: return "invalid argument";
    case BK_ENOMEM: return "workspace too small or allocation failed";
    case BK_EHIP: return "HIP runtime error";
    case BK_ENONFINITE: return "non-finite value in a Gram matrix";
    case BK_ENOCONV: return "Jacobi eigen-solve did not converge";
    case BK_ERANK: return "A Pi is numerically rank deficient";
    default: return "unknown status";
  }
}

const char* bk_version(void) { return "bk 0.1 gfx950"; }

size_t bk_svd_dense_workspace(int64_t n, int64_t d, int32_t k, int32_t q, int32_t a_type,
                              const bk_options* opt) {
  if (a_type < BK_F64 || a_type > BK_FP8_E4M3) return 0;
  const bool f64 = a_type == BK_F64;
  Options o = read_options(opt, f64);
  const int32_t pw = block_width(n, d, k, q, o);
  if (!pw) return 0;
  normalize_refine(o, a_type, true);  // sized for the pass whenever it may run
  return make_layout(nullptr, n, d, 0, pw, q, f64, o, false, false).bytes;
}

int bk_svd_dense(const void* A, int64_t lda, int32_t a_type, const float* a_scales,
                 const float* A_master, int64_t ld_master, int64_t n, int64_t d, int32_t k,
                 int32_t q, uint64_t seed, const bk_options* opt, void* Z, int64_t ldz,
                 double* ritz, bk_info* info, void* workspace, size_t workspace_bytes,
                 void* stream) {
  if (!A || !Z || !ritz || lda < d || ldz < k) return BK_EINVAL;
  if (a_type < BK_F64 || a_type > BK_FP8_E4M3) return BK_EINVAL;
  if (a_type == BK_FP8_E4M3 && !a_scales) return BK_EINVAL;
  const bool f64 = a_type == BK_F64;
  Options o = read_options(opt, f64);
  const int32_t pw = block_width(n, d, k, q, o);
  if (!pw) return BK_EINVAL;
  normalize_refine(o, a_type, A_master != nullptr);
  if (o.refine && (!A_master || ld_master < d)) return BK_EINVAL;
  if (o.center) return BK_EINVAL;  // dense centring is not offered
  if (o.at && (a_type == BK_BF16 || a_type == BK_FP8_E4M3) &&
      (o.ld_at < n || (a_type == BK_FP8_E4M3 && !o.at_scales)))
    return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = make_layout(nullptr, n, d, 0, pw, q, f64, o, false, false).bytes;
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  Layout L = make_layout(base, n, d, 0, pw, q, f64, o, false, false);
  DenseOp op;
  op.n = n;
  op.d = d;
  op.f64 = f64;
  op.A = A;
  op.lda = lda;
  op.a_type = a_type;
  op.ascale = a_type == BK_FP8_E4M3 ? a_scales : nullptr;
  op.fp32_cores = o.fp32_cores;
  if (o.at && (a_type == BK_BF16 || a_type == BK_FP8_E4M3)) {
    op.At = o.at;
    op.ld_at = o.ld_at;
    op.atscale = a_type == BK_FP8_E4M3 ? o.at_scales : nullptr;
  }
  DenseOp master;
  const DenseOp* mp = nullptr;
  if (o.refine) {
    master.n = n;
    master.d = d;
    master.f64 = false;
    master.A = A_master;
    master.lda = ld_master;
    master.a_type = BK_F32;
    master.fp32_cores = o.fp32_cores;
    mp = &master;
  }
  return solve(op, L, o, k, q, seed, mp, Z, ldz, ritz, info, s);
}

int bk_svd_dense_noalloc(const void* A, int64_t lda, int32_t a_type, const float* a_scales,
                         const float* A_master, int64_t ld_master, int64_t n, int64_t d,
                         int32_t k, int32_t q, uint64_t seed, const bk_options* opt, void* Z,
                         int64_t ldz, double* ritz, bk_info* info, void* stream) {
  if (!A || !Z || !ritz || lda < d || ldz < k) return BK_EINVAL;
  // a struct too short to hold the fields read_options takes counts as
  // "all defaults", as in bk_svd_dense
  const bool has_opt =
      opt && opt->struct_size >= static_cast<int32_t>(offsetof(bk_options, timing_phases));
  if (has_opt && opt->save_for_backward)
    return BK_EINVAL;  // the next call would overwrite the saved state
  const size_t need = bk_svd_dense_workspace(n, d, k, q, a_type, opt);
  if (need == 0) return BK_EINVAL;
  if (need > BK_NOALLOC_SCRATCH_BYTES) return BK_ENOMEM;
  bk_options o{};
  if (has_opt)
    std::memcpy(&o, opt, std::min(sizeof(o), static_cast<size_t>(opt->struct_size)));
  o.struct_size = static_cast<int32_t>(sizeof(o));
  o.timing = 0;  // timing would create events; launch counts are kept
  void* ws = scratch_address(static_cast<hipStream_t>(stream));
  if (!ws) return BK_EHIP;
  return bk_svd_dense(A, lda, a_type, a_scales, A_master, ld_master, n, d, k, q, seed, &o, Z,
                      ldz, ritz, info, ws, BK_NOALLOC_SCRATCH_BYTES, stream);
}

size_t bk_svd_csr_workspace(int64_t n, int64_t d, int64_t nnz, int32_t k, int32_t q,
                            const bk_options* opt) {
  if (nnz < 0 || nnz >= (int64_t(1) << 31)) return 0;
  Options o = read_options(opt, false);
  o.refine = 0;
  o.save = 0;
  const int32_t pw = block_width(n, d, k, q, o);
  if (!pw || (o.resid && pw != k)) return 0;
  return csr_workspace_bytes(n, d, nnz, pw, q, o, true, 0);
}

int bk_svd_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
               const int32_t* t_row_ptr, const int32_t* t_col_idx, const float* t_vals,
               int64_t n, int64_t d, int64_t nnz, int32_t k, int32_t q, uint64_t seed,
               const bk_options* opt, float* Z, int64_t ldz, double* ritz, bk_info* info,
               void* workspace, size_t workspace_bytes, void* stream) {
  if (nnz < 0 || nnz >= (int64_t(1) << 31) || !row_ptr || !Z || !ritz || ldz < k)
    return BK_EINVAL;
  if (nnz > 0 && (!col_idx || !vals)) return BK_EINVAL;
  const bool given_t = t_row_ptr && t_col_idx && t_vals;
  if ((t_row_ptr || t_col_idx || t_vals) && !given_t) return BK_EINVAL;
  Options o = read_options(opt, false);
  o.refine = 0;
  o.save = 0;
  const int32_t pw = block_width(n, d, k, q, o);
  if (!pw) return BK_EINVAL;
  if (o.resid && pw != k) return BK_EINVAL;  // the work plans are for width pw
  hipStream_t s = static_cast<hipStream_t>(stream);
  return csr_prepare_and_run(
      row_ptr, col_idx, vals, t_row_ptr, t_col_idx, t_vals, n, d, nnz, pw, q, o, workspace,
      workspace_bytes, 0, info, s, [&](CsrOp& op, Layout& L, char*) {
        return solve(op, L, o, k, q, seed, nullptr, Z, ldz, ritz, info, s);
      });
}

size_t bk_error_metrics_dense_workspace(int64_t n, int64_t d, int32_t k, int32_t q_spec,
                                        int32_t a_type) {
  if (a_type != BK_F64 && a_type != BK_F32) return 0;
  const bool f64 = a_type == BK_F64;
  Options o;
  if (!block_width(n, d, k, q_spec, o)) return 0;
  return align_up(make_layout(nullptr, n, d, 0, k, q_spec, f64, o, false, false).bytes, 256) +
         make_metrics_ws(nullptr, n, d, k, f64).bytes;
}

int bk_error_metrics_dense(const void* A, int64_t lda, int32_t a_type, int64_t n, int64_t d,
                           const void* Z, int64_t ldz, int32_t k, int32_t q_spec,
                           uint64_t seed, const double* sigma_true, int64_t n_sigma,
                           double* captured, bk_metrics* out, void* workspace,
                           size_t workspace_bytes, void* stream) {
  if (!A || !Z || lda < d || ldz < k) return BK_EINVAL;
  if (a_type != BK_F64 && a_type != BK_F32) return BK_EINVAL;
  const bool f64 = a_type == BK_F64;
  Options o;
  o.tau = f64 ? 1e-11 : 1e-5;
  if (!block_width(n, d, k, q_spec, o)) return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t lay =
      align_up(make_layout(nullptr, n, d, 0, k, q_spec, f64, o, false, false).bytes, 256);
  const size_t need = lay + make_metrics_ws(nullptr, n, d, k, f64).bytes;
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  Layout L = make_layout(base, n, d, 0, k, q_spec, f64, o, false, false);
  const MetricsWs w = make_metrics_ws(base + lay, n, d, k, f64);
  DenseOp op;
  op.n = n;
  op.d = d;
  op.f64 = f64;
  op.A = A;
  op.lda = lda;
  op.a_type = a_type;
  op.pack = L.pack;
  op.pack_bytes = L.pack_bytes;
  return metrics_run(op, L, w, Z, ldz, k, q_spec, seed, sigma_true, n_sigma, captured, out, s,
                     [&](double* part, double* res) {
                       launch_dense_fro2(A, f64, n, d, lda, part, res, s);
                     });
}

size_t bk_error_metrics_csr_workspace(int64_t n, int64_t d, int64_t nnz, int32_t k,
                                      int32_t q_spec) {
  if (nnz < 0 || nnz >= (int64_t(1) << 31)) return 0;
  Options o;
  if (!block_width(n, d, k, q_spec, o)) return 0;
  return csr_workspace_bytes(n, d, nnz, k, q_spec, o, true,
                             make_metrics_ws(nullptr, n, d, k, false).bytes);
}

int bk_error_metrics_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                         const int32_t* t_row_ptr, const int32_t* t_col_idx,
                         const float* t_vals, int64_t n, int64_t d, int64_t nnz,
                         int32_t center_rows, const float* Z, int64_t ldz, int32_t k,
                         int32_t q_spec, uint64_t seed, const double* sigma_true,
                         int64_t n_sigma, double* captured, bk_metrics* out, void* workspace,
                         size_t workspace_bytes, void* stream) {
  if (nnz < 0 || nnz >= (int64_t(1) << 31) || !row_ptr || !Z || ldz < k) return BK_EINVAL;
  if (nnz > 0 && (!col_idx || !vals)) return BK_EINVAL;
  const bool given_t = t_row_ptr && t_col_idx && t_vals;
  if ((t_row_ptr || t_col_idx || t_vals) && !given_t) return BK_EINVAL;
  Options o;
  o.tau = 1e-5;
  o.center = center_rows ? 1 : 0;
  if (!block_width(n, d, k, q_spec, o)) return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t wbytes = make_metrics_ws(nullptr, n, d, k, false).bytes;
  return csr_prepare_and_run(
      row_ptr, col_idx, vals, t_row_ptr, t_col_idx, t_vals, n, d, nnz, k, q_spec, o,
      workspace, workspace_bytes, wbytes, nullptr, s, [&](CsrOp& op, Layout& L, char* extra) {
        const MetricsWs w = make_metrics_ws(extra, n, d, k, false);
        return metrics_run(op, L, w, Z, ldz, k, q_spec, seed, sigma_true, n_sigma, captured,
                           out, s, [&](double* part, double* res) {
                             launch_csr_fro2(row_ptr, vals, n, d, o.center != 0, part, res, s);
                           });
      });
}

size_t bk_svd_dense_backward_workspace(int64_t n, int64_t d, int32_t k, int32_t q,
                                       int32_t a_type) {
  if (!valid_kq(n, d, k, q) || (a_type != BK_F64 && a_type != BK_F32)) return 0;
  return make_bwd_layout(nullptr, n, d, k, q, a_type == BK_F64).bytes;
}

int bk_svd_dense_backward(const void* A, int64_t lda, int32_t a_type, int64_t n, int64_t d,
                          int32_t k, int32_t q, const void* Z, int64_t ldz, const double* ritz,
                          const void* Z_bar, const double* ritz_bar, void* A_bar,
                          int64_t ld_bar, const void* fwd_workspace, size_t fwd_bytes,
                          void* workspace, size_t workspace_bytes, void* stream) {
  (void)Z;
  (void)ritz;
  if (!valid_kq(n, d, k, q) || (a_type != BK_F64 && a_type != BK_F32) || !A || !A_bar ||
      !fwd_workspace || lda < d || ld_bar < d || (Z_bar && ldz < k))
    return BK_EINVAL;
  const bool f64 = a_type == BK_F64;
  const Options fo = backward_fwd_options(f64);
  const Layout F = make_layout(static_cast<char*>(const_cast<void*>(fwd_workspace)), n, d, 0, k,
                               q, f64, fo, false, false);
  if (fwd_bytes < F.bytes) return BK_EINVAL;  // not a save_for_backward workspace
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = make_bwd_layout(nullptr, n, d, k, q, f64).bytes;
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  const BwdLayout B = make_bwd_layout(base, n, d, k, q, f64);
  DenseOp op;
  op.n = n;
  op.d = d;
  op.f64 = f64;
  op.A = A;
  op.lda = lda;
  op.a_type = a_type;
  return backward_dense(op, k, q, F, B, Z_bar, ldz, ritz_bar, A_bar, ld_bar, s);
}

int bk_gaussian(uint64_t seed, int64_t rows, int64_t cols, int64_t ld, int32_t dtype, void* out,
                void* stream) {
  if (rows < 0 || cols < 0 || ld < cols || !out || (dtype != BK_F64 && dtype != BK_F32))
    return BK_EINVAL;
  launch_gaussian(seed, rows, cols, ld, dtype == BK_F64, out, static_cast<hipStream_t>(stream));
  BK_TRY_LAUNCH();
  return BK_OK;
}

int bk_philox4x32_10(const uint32_t* in, int64_t count, uint32_t* out, void* stream) {
  if (count < 0 || (count > 0 && (!in || !out))) return BK_EINVAL;
  launch_philox_raw(in, count, out, static_cast<hipStream_t>(stream));
  BK_TRY_LAUNCH();
  return BK_OK;
}

int bk_quantize_dense(const float* A, int64_t n, int64_t d, int64_t lda, int32_t to, void* out,
                      float* tile_scales, void* stream) {
  if (n < 0 || d < 0 || lda < d || !A || !out) return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (to == BK_BF16) {
    launch_quant_bf16(A, n, d, lda, static_cast<bf16_t*>(out), s);
  } else if (to == BK_FP8_E4M3) {
    if (!tile_scales) return BK_EINVAL;
    launch_quant_fp8(A, n, d, lda, static_cast<fp8_t*>(out), tile_scales, s);
  } else {
    return BK_EINVAL;
  }
  BK_TRY_LAUNCH();
  return BK_OK;
}

int bk_quantize_dense_transposed(const float* A, int64_t n, int64_t d, int64_t lda, int32_t to,
                                 void* out_t, float* tile_scales_t, void* stream) {
  if (n < 0 || d < 0 || lda < d || !A || !out_t) return BK_EINVAL;
  if (to != BK_BF16 && to != BK_FP8_E4M3) return BK_EINVAL;
  if (to == BK_FP8_E4M3 && !tile_scales_t) return BK_EINVAL;
  launch_quant_t(A, n, d, lda, to, out_t, tile_scales_t, static_cast<hipStream_t>(stream));
  BK_TRY_LAUNCH();
  return BK_OK;
}

size_t bk_dense_product_workspace(int32_t trans, int64_t n, int64_t d, int32_t k,
                                  int32_t a_type) {
  if (n <= 0 || d <= 0 || k <= 0) return 0;
  // FP64 partials (A^T X) + the matrix-core packing of X (FP32 / BF16 / FP8)
  const size_t part =
      trans ? align_up(static_cast<size_t>(tn_partial_elems(n, d, k)) * sizeof(double), 256)
            : 256;
  // (FP32 A^T X: Y's three BF16 limb planes)
  const size_t pack =
      (a_type == BK_F64)
          ? 0
          : static_cast<size_t>(trans ? (a_type == BK_F32 ? x3_pack_bytes(n, k)
                                                          : mfma_pack_bytes(n, k, a_type))
                                      : mfma_nn_work_bytes(n, d, k, a_type));
  return part + pack;
}

int bk_dense_product(int32_t trans, const void* A, int64_t lda, int32_t a_type,
                     const float* a_scales, int64_t n, int64_t d, const void* X, int64_t ldx,
                     int32_t k, void* Y, int64_t ldy, void* workspace, size_t workspace_bytes,
                     void* stream) {
  if (n <= 0 || d <= 0 || k <= 0 || !A || !X || !Y || lda < d || ldx < k || ldy < k)
    return BK_EINVAL;
  if (a_type < BK_F64 || a_type > BK_FP8_E4M3) return BK_EINVAL;
  if (a_type == BK_FP8_E4M3 && !a_scales) return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = bk_dense_product_workspace(trans, n, d, k, a_type);
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  const size_t part =
      trans ? align_up(static_cast<size_t>(tn_partial_elems(n, d, k)) * sizeof(double), 256)
            : 256;
  Timer tm;
  DenseOp op;
  op.n = n;
  op.d = d;
  op.f64 = a_type == BK_F64;
  op.A = A;
  op.lda = lda;
  op.a_type = a_type;
  op.ascale = a_type == BK_FP8_E4M3 ? a_scales : nullptr;
  op.partial = reinterpret_cast<double*>(base);
  if (a_type != BK_F64) {
    op.pack = base + part;
    op.pack_bytes = need - part;
  }
  op.tm = &tm;
  if (trans) op.aty(X, ldx, k, Y, ldy, s);
  else op.ax(X, ldx, k, Y, ldy, s);
  BK_TRY_LAUNCH();
  return BK_OK;
}

int bk_csr_product(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                   int64_t rows, int64_t cols, int64_t nnz, const float* X, int64_t ldx,
                   int32_t k, float* Y, int64_t ldy, void* stream) {
  if (rows < 0 || cols < 0 || nnz < 0 || k <= 0 || !row_ptr || !X || !Y || ldx < k || ldy < k)
    return BK_EINVAL;
  // every row by the row kernel (no long-row plan for a one-off product)
  launch_csr_spmm(row_ptr, col_idx, vals, rows, k, X, cols, ldx, Y, ldy, nullptr, nullptr,
                  nnz >= 16 * rows, static_cast<hipStream_t>(stream));
  BK_TRY_LAUNCH();
  return BK_OK;
}

size_t bk_csr_transpose_workspace(int64_t rows, int64_t cols, int64_t nnz) {
  (void)rows;
  if (cols < 0 || nnz < 0) return 0;
  return align_up(static_cast<size_t>(cols) * 4, 256) + csr_transpose_scratch_bytes(nnz, cols) +
         align_up(sizeof(Ctrl), 256) + 256;
}

int bk_csr_transpose(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                     int64_t rows, int64_t cols, int64_t nnz, int32_t* t_row_ptr,
                     int32_t* t_col_idx, float* t_vals, void* workspace,
                     size_t workspace_bytes, void* stream) {
  if (rows < 0 || cols <= 0 || nnz < 0 || nnz >= (int64_t(1) << 31) || !row_ptr || !t_row_ptr)
    return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = bk_csr_transpose_workspace(rows, cols, nnz);
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  int32_t* cursor = reinterpret_cast<int32_t*>(base);
  const size_t koff = align_up(static_cast<size_t>(cols) * 4, 256);
  const size_t sb = csr_transpose_scratch_bytes(nnz, cols);
  char* scratch = base + koff;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + koff + sb);
  // the structure is checked before the transpose indexes through it
  launch_ctrl_init(ctrl, 0, s);
  launch_csr_validate(row_ptr, col_idx, rows, cols, nnz, ctrl, s);
  Ctrl h;
  BK_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  BK_TRY(hipStreamSynchronize(s));
  if (h.csr_bad) return BK_EINVAL;
  if (launch_csr_transpose(row_ptr, col_idx, vals, rows, cols, nnz, t_row_ptr, t_col_idx,
                           t_vals, cursor, scratch, sb, s) != 0)
    return BK_EHIP;
  BK_TRY_LAUNCH();
  return BK_OK;
}

size_t bk_eigh_psd_workspace(int64_t m) {
  if (m <= 0) return 0;
  Arena ar;
  ar.take<Ctrl>(1);
  take_jacobi(ar, m, 0, true);
  ar.take<double>(static_cast<size_t>(m));  // sign
  return align_up(ar.off, 256);
}

int bk_eigh_psd(const double* M, int64_t m, int64_t ldm, double* theta, double* V,
                int64_t ldv, int32_t max_sweeps, double tol, int32_t* sweeps, void* workspace,
                size_t workspace_bytes, void* stream) {
  if (m <= 0 || ldm < m || ldv < m || !M || !theta || !V || m > (int64_t(1) << 20))
    return BK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = bk_eigh_psd_workspace(m);
  DevBuf own;
  char* base = static_cast<char*>(workspace);
  if (!base) {
    own.s = s;
    if (hipMallocAsync(&own.p, need, s) != hipSuccess) return BK_ENOMEM;
    base = static_cast<char*>(own.p);
  } else if (workspace_bytes < need) {
    return BK_ENOMEM;
  }
  Arena ar;
  ar.base = base;
  Layout L;
  L.ctrl = ar.take<Ctrl>(1);
  JacobiWs jw = take_jacobi(ar, m, 0, true);
  double* sign = ar.take<double>(static_cast<size_t>(m));
  Solver S;
  S.L = &L;
  S.o.max_sweeps = max_sweeps > 0 ? max_sweeps : 40;
  S.o.jtol = tol;
  Timer tm;
  S.tm = &tm;
  S.s = s;
  launch_ctrl_init(L.ctrl, 0, s);
  // theta / order via the finalize step; V gets every column.
  int st = S.eig(M, m, jw, static_cast<int>(std::min<int64_t>(m, 0x7FFFFFFF)), V, ldv, nullptr);
  if (st != BK_OK) return st;
  launch_copy2d(jw.theta, true, 1, theta, true, 1, m, 1, s);
  launch_sign_normalize(V, true, m, static_cast<int>(m), ldv, nullptr, 0, 0, sign, s);
  BK_TRY(hipStreamSynchronize(s));
  BK_TRY_LAUNCH();
  if (sweeps) *sweeps = S.sweeps;
  return S.noconv ? BK_ENOCONV : BK_OK;
}

}  // extern "C"
