// Host-side launchers of the gfx950 kernels.  Each launcher only enqueues on
// the given stream; the caller checks hipGetLastError().
#pragma once

#include "common.hpp"

namespace bk {

// ------------------------------------------------------------------ rng --
void launch_gaussian(uint64_t seed, int64_t rows, int64_t cols, int64_t ld,
                     bool f64, void* out, hipStream_t s);
void launch_philox_raw(const uint32_t* in, int64_t count, uint32_t* out,
                       hipStream_t s);

// ----------------------------------------------------------------- gemm --
// C (n x N, ldc) = alpha * A (n x K, lda) . X (K x N, ldx) + beta * C.
// a_type: BK_F64 / BK_F32 / BK_BF16 / BK_FP8_E4M3 (FP8 with 128 x 128 tile
// scales, ascale_ld = ceil(K / 128)).  X and C are FP64 or FP32.  The FP64
// path (a_type BK_F64) accumulates in FP64, every other path in FP32.
struct NNArgs {
  int64_t n = 0, K = 0;
  int N = 0;
  const void* A = nullptr;
  int64_t lda = 0;
  int a_type = BK_F32;
  const float* ascale = nullptr;
  int64_t ascale_ld = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  bool x_f64 = false;
  void* C = nullptr;
  int64_t ldc = 0;
  bool c_f64 = false;
  double alpha = 1.0, beta = 0.0;
  // scratch for the matrix-core path (X^T packed in A's type), nullable
  void* work = nullptr;
  size_t work_bytes = 0;
  // N <= 32 only: per-row-block partial Grams of the stored C rows (FP64,
  // nn_gram_partial_elems doubles), added up by launch_gram_reduce; the
  // vector kernel then runs (no matrix-core path)
  double* gram_partial = nullptr;
  // FP64 scratch (nullable) for splitting K when few row tiles leave the
  // chip idle (vector path, no gram_partial): S n N doubles
  double* split_work = nullptr;
  int64_t split_work_elems = 0;
  // FP32 A on the FP32 matrix cores (32 x 32 x 2 steps) instead of as three
  // BF16 limbs on the BF16 matrix cores
  bool fp32_cores = false;
};
// returns the number of kernels launched (0: not launched)
int launch_nn(const NNArgs& a, hipStream_t s);
int64_t nn_gram_partial_elems(int64_t n, int N);  // 0 if N > 32
// G (N x N, ld N) = sum of the partial Grams of an n-row launch_nn
int launch_gram_reduce(int64_t n, int N, const double* gpart, double* G, hipStream_t s);

// C (p x r, ldc) = alpha * X^T . Y + beta * C with X L x p (ldx), Y L x r
// (ldy): the reduction over the long L is split into S chunks whose FP64
// partial sums are added in a fixed order.  x_type as a_type above (FP8
// scales index [l / 128][p / 128]); Y is FP64 or FP32 (FP64 iff X is).
struct TNArgs {
  int64_t L = 0, p = 0;
  int r = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  int x_type = BK_F32;
  const float* xscale = nullptr;
  int64_t xscale_ld = 0;
  const void* Y = nullptr;
  int64_t ldy = 0;
  bool y_f64 = false;
  void* C = nullptr;
  int64_t ldc = 0;
  bool c_f64 = true;
  double alpha = 1.0, beta = 0.0;
  double* partial = nullptr;  // >= tn_partial_elems(L, p, r) doubles
  // scratch for the matrix-core path (Y^T packed in X's type), nullable
  void* work = nullptr;
  size_t work_bytes = 0;
  // X and Y the same matrix (p = r): tiles below the diagonal are skipped and
  // C mirrored from above it
  bool sym = false;
  // FP32 X on the FP32 matrix cores instead of as three BF16 limbs (the
  // limbs need `work` for Y's limb planes; without it the FP32 cores run)
  bool fp32_cores = false;
};
int tn_splits(int64_t L, int64_t p, int r);
int64_t tn_partial_elems(int64_t L, int64_t p, int r);
int launch_tn(const TNArgs& a, hipStream_t s);  // kernels launched

// Matrix-core paths (gemm_mfma.hip): taken for FP32 / BF16 / FP8 operands
// of aligned, large enough products; otherwise the VALU kernels run.
// Bytes of scratch to pack an lred x cols FP32 operand in `type`.
int64_t mfma_pack_bytes(int64_t lred, int64_t cols, int type);
// Bytes of the three BF16 limb planes of an lred x cols FP32 operand (FP32
// products on the BF16 matrix cores).
int64_t x3_pack_bytes(int64_t lred, int64_t cols);
// Splits of K of the matrix-core A X (n x K times K x N) and the scratch it
// needs: the packed X^T plus, with several splits, their FP32 partials.
int nn_mfma_splits(int64_t n, int64_t K, int64_t N, int type);
int64_t mfma_nn_work_bytes(int64_t n, int64_t K, int64_t N, int type);
int tn_mfma_splits(int64_t L, int64_t p, int r);
// *launches: kernels launched on the matrix-core path (pack, product and,
// with split K, the reduction); 0 if the product was not taken
void launch_nn_mfma_if(const NNArgs& a, hipStream_t s, int* launches);
// *splits = number of FP64 partials written (0: not handled)
void launch_tn_mfma_if(const TNArgs& a, hipStream_t s, int* splits);
// M (m x m FP64, ld ldm, both triangles) = W^T W for an FP32 W (L x m, ld
// ldw; m <= kGramSymMaxM, L >= kGramSymMinL: shorter blocks are faster on
// the vector path) on the matrix cores: FP32 sums of 32-row chunks added in
// FP64; part: gram_sym_partial_elems(L, m) doubles.  Returns the kernels
// launched (0: not applicable).
constexpr int kGramSymMaxM = 384;
constexpr int64_t kGramSymMinL = 32768;
int64_t gram_sym_partial_elems(int64_t L, int m);
int launch_gram_sym_mfma(int64_t L, int m, const float* W, int64_t ldw, double* M, int64_t ldm,
                         double* part, hipStream_t s);

// ---------------------------------------------------------------- small --
// Fill / convert helpers.
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// dst (rows x cols, ldd) = src (rows x cols, lds), any of f64/f32 each side
void launch_copy2d(const void* src, bool src_f64, int64_t lds, void* dst,
                   bool dst_f64, int64_t ldd, int64_t rows, int64_t cols,
                   hipStream_t s);
// y += x (FP64, n elements)
void launch_axpy_f64(const double* x, double* y, int64_t n, hipStream_t s);
void launch_ctrl_init(Ctrl* c, int32_t q, hipStream_t s);
void launch_ctrl_reset_off(Ctrl* c, hipStream_t s);

// One-workgroup Cholesky + triangular inverse of a k x k FP64 Gram matrix
// (see chol_kernel for the modes).
// Cholesky of CholeskyQR: registers of one wavefront for k <= 64, blocked
// by 32 over a chain of chip-wide kernels for k <= kCholBlockedMax (work:
// k k + 4096 doubles), else one workgroup step by step.
constexpr int kCholBlockedMax = 512;

// Squared Frobenius norms for the error measures (metrics.hip): *out (FP64,
// device) = ||A||_F^2 of a dense n x d A (ld lda, FP64 or FP32), or of a CSR
// A (- mu 1^T with centre, mu the row means); part: fro2_partial_elems()
// doubles of scratch.
int64_t fro2_partial_elems();
void launch_dense_fro2(const void* A, bool f64, int64_t n, int64_t d, int64_t lda,
                       double* part, double* out, hipStream_t s);
void launch_csr_fro2(const int32_t* rp, const float* v, int64_t n, int64_t d, bool center,
                     double* part, double* out, hipStream_t s);
// Residual norms of the returned Ritz pairs (metrics.hip): out[c] (FP64,
// device) = ||g_c R_c - sigma_c^2 Z_c||_2 with R = A A^T Z' (n x k, ld ldr),
// Z = Z' diag(g) (n x k, ld ldz; g = rsign, or all +1 when null), both FP64
// or both FP32; part: ritz_resid_partial_elems(k) doubles of scratch.
int64_t ritz_resid_partial_elems(int k);
void launch_ritz_resid(const void* R, int64_t ldr, const void* Z, int64_t ldz, bool f64,
                       int64_t n, int k, const double* sigma, const double* rsign, double* part,
                       double* out, hipStream_t s);
inline int64_t chol_work_doubles(int k) { return static_cast<int64_t>(k) * k + 4096; }
enum CholMode { CHOL_FIRST_BLOCK0 = 0, CHOL_FIRST = 1, CHOL_REPEAT = 2 };
void launch_chol(int k, const double* G, const double* Gpre, int mode,
                 int block, double tau, double shift_coef, double* R,
                 double* Rinv, double* work, Ctrl* ctrl, hipStream_t s);
// T = A . B for k x k upper-triangular FP64 matrices (one workgroup).
void launch_trmm_upper(int k, const double* A, const double* B, double* T,
                       hipStream_t s);
// The block-tridiagonal Q^T A A^T Q of block Lanczos into M (m x m, ld
// ldm), m = (q+1) k: diagonal blocks from the two projection passes' FP64
// coefficients (block i's pass-j coefficients at Cband + (2 i + j) cstride,
// ld k) and Tqq (the last block), sub-diagonal blocks R3 R2 R1 from the
// CholeskyQR factors (block i's pass j at Rband + (3 i + j) k^2); P holds
// (q+1) k^2 doubles of scratch.  Returns the kernels launched.
int launch_block_tridiag(int64_t m, int k, int q, const double* Cband, int64_t cstride,
                         const double* Rband, double* P, const double* Tqq, double* M,
                         int64_t ldm, hipStream_t s);
// One CholeskyQR pass for k <= kCqrPassMaxK in one launch: G = the sum of
// the P FP64 Gram partials Gin (k x k each), R = chol(G [+ shift]) under
// the modes of launch_chol (R written, ctrl updated), Y = X R^-1 by
// forward substitution per row (X, Y n x k in the working type, X may be
// Y), and the Gram partials of the stored Y in gout (one per workgroup,
// cqr_pass_grid(n) of them; nullable).  Returns the kernels launched.
constexpr int kCqrPassMaxK = 32;
struct CqrPass {
  int64_t n = 0;
  int k = 0;
  const double* Gin = nullptr;
  int P = 1;
  const double* Gpre = nullptr;
  int mode = 0, block = 0;
  double tau = 0.0, shift_coef = 0.0;
  double* R = nullptr;
  Ctrl* ctrl = nullptr;
  const void* X = nullptr;
  int64_t ldx = 0;
  void* Y = nullptr;
  int64_t ldy = 0;
  bool f64 = false;
  int64_t rows_per_wg = 0;  // set by the launcher
  double* gout = nullptr;
  // > 0: when max |G - I| <= skip_tol the pass leaves X as it is (R = I);
  // then X must be Y (in place)
  double skip_tol = 0.0;
  // nullable: mupart[b k + c] = sum over workgroup b's rows r of
  // mu[r] Y[r][c] (FP64, the stored values): the block partials of mu^T Y
  // that launch_colsum_final adds up (a skipped pass writes none)
  const float* mu = nullptr;
  double* mupart = nullptr;
};
int cqr_pass_grid(int64_t n, int64_t* rows_per_wg);
int64_t cqr_pass_partial_elems(int k);
int launch_cqr_pass(const CqrPass& a, hipStream_t s);

// Helpers of the adjoint.
// dst (cols x rows) = src (rows x cols)^T, FP64/FP32 either side.
void launch_transpose(const void* src, bool src_f64, int64_t lds, void* dst,
                      bool dst_f64, int64_t ldd, int64_t rows, int64_t cols,
                      hipStream_t s);
// out = copyltu(-S) (symmetric, lower triangle of -S mirrored), k x k.
void launch_copyltu_neg(int k, const double* S, double* out, hipStream_t s);
// G (m x k) of the eigen-decomposition adjoint (see small.hip).
void launch_eig_adjoint(int64_t m, int k, const double* theta, const double* H,
                        const double* ritz, const double* ritz_bar, double* G,
                        hipStream_t s);
void launch_symmetrize(int64_t m, double* M, hipStream_t s);
// out = (R^-1)^T of an upper-triangular k x k R; work: k x k scratch.
void launch_trinv_t(int k, const double* R, double* work, double* out, hipStream_t s);
// U (m x m) = eigenvector columns in descending order (order[]), first k
// columns multiplied by sign[].
void launch_gather_vectors(const double* Vc, int64_t ldc, int64_t m,
                           const int32_t* order, const double* sign, int k,
                           double* U, hipStream_t s);

// Column signs of Z (n x k): sign[c] = +1 / -1 so that the largest-|.|
// entry of column c (lowest row on ties) becomes positive; then Z and the
// m x k matrix U (nullable) are multiplied column-wise by sign.
void launch_sign_normalize(void* Z, bool f64, int64_t n, int k, int64_t ldz,
                           double* U, int64_t m, int64_t ldu, double* sign,
                           hipStream_t s);

// --------------------------------------------------------------- jacobi --
// One-sided block Jacobi on the columns of a symmetric PSD M (see
// jacobi.hip).  Xc / Vc are column-major m x nbp (ld ldc).
int jacobi_default_block(int64_t m);
int64_t jacobi_padded_cols(int64_t m, int b);
void launch_jacobi_init(const double* M, int64_t m, int64_t ldm, double* Xc,
                        double* Vc, int64_t ldc, int64_t nbp, hipStream_t s);
void launch_jacobi_round(int b, int64_t m, int nb, int round, double* Xc,
                         double* Vc, int64_t ldc, double tol, int inner_max,
                         Ctrl* ctrl, hipStream_t s);
// theta (descending), order; Uk (m x k, ld ldu) = normalised eigenvectors of
// the top k (from Vc when non-null, else Xc / theta); ritz = sqrt(theta).
void launch_jacobi_finalize(const double* Xc, const double* Vc, int64_t ldc,
                            int64_t m, int k, double* theta_sorted,
                            int32_t* order, double* norms, double* Uk,
                            int64_t ldu, double* ritz, hipStream_t s);

// ------------------------------------------------------------ tridiagonal --
// Top-k eigenpairs of a symmetric m x m FP64 matrix through Householder
// tridiagonalisation, multisection + inverse iteration, back-transformation
// (tridiag.hip).  theta: k values descending; Uk m x k (ld ldu); ritz
// (nullable) = sqrt(max(theta, 0)).  scratch: tridiag_scratch_doubles(m, k).
constexpr int64_t kTridiagMax = 2560;
int64_t tridiag_scratch_doubles(int64_t m, int k);
// ctrl (nullable) gets CTRL_STALL if a grid barrier of the cooperative
// reduction gave up waiting.
void launch_tridiag_topk(const double* M, int64_t m, int64_t ldm, int k,
                         double* scratch, double* theta, double* Uk, int64_t ldu,
                         double* ritz, Ctrl* ctrl, hipStream_t s);

// ------------------------------------------------------------------ csr --
void launch_csr_validate(const int32_t* rp, const int32_t* ci, int64_t rows,
                         int64_t cols, int64_t nnz, Ctrl* ctrl, hipStream_t s);
// Y (rows x k) = A X - rowvec (x) colvec (rowvec nullable = all ones,
// colvec nullable = no correction), every row by one slot of KC lanes
// (no work plan: the one-off product of the public helper).
void launch_csr_spmm(const int32_t* rp, const int32_t* ci, const float* v,
                     int64_t rows, int k, const float* X, int64_t xrows, int64_t ldx,
                     float* Y, int64_t ldy, const float* rowvec,
                     const double* colvec, bool batch, hipStream_t s);

// Work plan of one CSR operand for the Krylov products.  Rows of at most
// kCsrShort nonzeros are listed in row order and taken SLOTS = 64 / KC to a
// wavefront; longer rows are cut into pieces of csr_piece_len(k) nonzeros,
// one wavefront each; a row of several pieces is finished by a combine
// kernel that adds its piece sums in piece order (deterministic).  The plan
// depends only on the sparsity structure and k.
constexpr int kCsrShort = 64;
constexpr int kCsrSlotRows = 8;  // consecutive short rows per KC-lane slot
int csr_piece_len(int k);
// upper bound on the number of pieces of any matrix with nnz nonzeros
int64_t csr_max_pieces(int64_t nnz, int64_t rows);
struct CsrPlan {
  int32_t* short_rows = nullptr;   // rows: short rows, row order
  int32_t* piece_row = nullptr;    // max pieces: row of piece p
  int32_t* piece_first = nullptr;  // max pieces: first piece of that row
  int32_t* multi_row = nullptr;    // max pieces: rows of several pieces
  int32_t* multi_first = nullptr;  // max pieces: their first piece
  int32_t* blk = nullptr;          // 8 * (row chunks + 1): counts and offsets
  float* part = nullptr;           // max pieces * k piece sums
  int64_t rows = 0;
  int nshort = 0, npieces = 0, nmulti = 0;
  int64_t short_nnz = 0;           // nonzeros in the short rows
  int operand = 0;                 // 0: A, 1: A^T (names the kernel instance)
};
// short rows per KC-lane slot of the product kernel (1 .. kCsrSlotRows)
int csr_slot_rows(const CsrPlan& pl, int k);
int64_t csr_plan_chunks(int64_t rows);
// builds the plan on the stream; totals[0..3] = short rows, pieces, rows of
// several pieces, nonzeros in short rows (device, read back by the caller
// before launch_csr_product)
void launch_csr_plan(const int32_t* rp, int64_t rows, int k, CsrPlan& pl,
                     int32_t* totals, hipStream_t s);
// Y = A X - rowvec colvec^T (rowvec nullable = ones, colvec nullable = no
// centring term); Y2 (nullable, ld ldy2) receives a second copy of Y.
void launch_csr_product(const CsrPlan& pl, const int32_t* rp, const int32_t* ci,
                        const float* v, int k, const float* X, int64_t xrows, int64_t ldx,
                        float* Y, int64_t ldy, float* Y2, int64_t ldy2,
                        const float* rowvec, const double* colvec, hipStream_t s);
// finishes the rows of several pieces (after launch_csr_product)
void launch_csr_combine(const CsrPlan& pl, const int32_t* rp, int k, float* Y, int64_t ldy,
                        float* Y2, int64_t ldy2, const float* rowvec, const double* colvec,
                        hipStream_t s);
// Gather copies of the product's right-hand block: row stride
// csr_stage_ld(k) floats (k rounded up to 32: every row on its own 128-byte
// lines), padding zeroed.
int csr_stage_ld(int k);
void launch_csr_stage(const float* X, int64_t ldx, int64_t rows, int k, float* xs,
                      hipStream_t s);
// colvec[c] = sum_r w[r] X[r][c] (FP64) over L rows (w nullable = ones):
// colsum_blocks(L) blocks sum contiguous row ranges into colpart (blocks x k)
// and a one-block kernel adds those in block order (fixed order throughout).
constexpr int kColsumBlocks = 256;
int colsum_blocks(int64_t L);
void launch_colsum(const float* X, int64_t ldx, int64_t L, int k, const float* w,
                   double* colpart, double* colvec, hipStream_t s);
// colvec = the sum of nb block partials (nb x k), in block order
void launch_colsum_final(const double* colpart, int nb, int k, double* colvec, hipStream_t s);
// exclusive scan of n counts into out[0..n] (one workgroup)
void launch_scan_i32(const int32_t* cnt, int64_t n, int32_t* out, hipStream_t s);
void launch_csr_row_means(const int32_t* rp, const float* v, int64_t rows,
                          int64_t cols, float* mu, hipStream_t s);
// CSR transpose: column counts -> scan -> stable radix sort of the column ids
// (positions as payload) -> gather.  cursor: cols ints; scratch:
// csr_transpose_scratch_bytes(nnz, cols).  Returns 0, or -1 when the sort
// could not run (scratch too small / a HIP error).
size_t csr_transpose_scratch_bytes(int64_t nnz, int64_t cols);
int launch_csr_transpose(const int32_t* rp, const int32_t* ci, const float* v, int64_t rows,
                         int64_t cols, int64_t nnz, int32_t* trp, int32_t* tci, float* tv,
                         int32_t* cursor, void* scratch, size_t scratch_bytes, hipStream_t s);

// ---------------------------------------------------------------- quant --
// Transposed copy (d x n, ld n) with the codes of the copies below; FP8
// scales_t [ceil(d/128)][ceil(n/128)] (the transpose of their tile scales).
void launch_quant_t(const float* A, int64_t n, int64_t d, int64_t lda, int to, void* out,
                    float* scales_t, hipStream_t s);
void launch_quant_bf16(const float* A, int64_t n, int64_t d, int64_t lda,
                       bf16_t* out, hipStream_t s);
void launch_quant_fp8(const float* A, int64_t n, int64_t d, int64_t lda,
                      fp8_t* out, float* scales, hipStream_t s);

}  // namespace bk
