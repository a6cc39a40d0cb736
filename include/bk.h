/*
 * bk.h -- C ABI of the MI355X (gfx950) randomized Block Krylov Iteration
 * library (libbk.so).
 *
 * The method is Algorithm 2 of Musco & Musco, "Randomized Block Krylov
 * Methods for Stronger and Faster Approximate Singular Value Decomposition"
 * (NIPS 2015):
 *   Pi ~ N(0,1)^{d x k};  K = [A Pi, (A A^T) A Pi, ..., (A A^T)^q A Pi];
 *   Q = orthonormal basis of span(K);  M = Q^T A A^T Q;
 *   U_k = top-k eigenvectors of M;  Z = Q U_k.
 * The library returns Z (n x k, orthonormal columns) and the Ritz values
 * sigma_i = sqrt(theta_i), theta_1 >= ... >= theta_k the top eigenvalues of M
 * (Lemma 1: M = U S^2 U^T, so sigma_i approximates the i-th singular value).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller, unless the
 *   comment says "host".  Matrices are row-major with the stated leading
 *   dimension (elements between consecutive rows).
 * - All work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *   the default stream).  The solve entry points synchronize `stream` before
 *   returning (they read a device status word); the helpers do not.
 * - Return value: a bk_status.  BK_EINVAL means nothing was launched.  No C++
 *   exception crosses the boundary.  Outputs are fully written only when the
 *   call returns BK_OK.
 * - Calls on distinct streams with distinct workspaces are independent; the
 *   library keeps no state between calls.
 * - Every reduction runs in a fixed order: repeated calls on the same inputs
 *   give bit-identical results.
 */
#ifndef BK_H
#define BK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage / compute types.  BK_F64 and BK_F32 are the plain paths (all
 * Krylov blocks, Z and W in that type).  BK_BF16 and BK_FP8_E4M3 describe a
 * low-precision COPY of A (made by bk_quantize_dense); their solve path keeps
 * Q, W and Z in FP32, accumulates products in FP32, and keeps the Gram,
 * Cholesky and Rayleigh-Ritz eigen-solve in FP64. */
typedef enum {
  BK_F64 = 0,
  BK_F32 = 1,
  BK_BF16 = 2,
  BK_FP8_E4M3 = 3 /* OCP e4m3 (max 448) with one FP32 scale per 128 x 128 tile */
} bk_dtype;

typedef enum {
  BK_OK = 0,
  BK_EINVAL = 1,      /* bad argument; nothing launched                        */
  BK_ENOMEM = 2,      /* workspace too small / allocation failed               */
  BK_EHIP = 3,        /* a HIP runtime call failed                             */
  BK_ENONFINITE = 4,  /* NaN/Inf met in a Gram matrix (non-finite input)       */
  BK_ENOCONV = 5,     /* the Jacobi eigen-solve hit max_jacobi_sweeps          */
  BK_ERANK = 6        /* A Pi is numerically rank deficient (A = 0, rank < k)  */
} bk_status;

/* Options.  Zero-initialise and set struct_size = sizeof(bk_options); a
 * zero field means "default". */
typedef struct bk_options {
  int32_t struct_size;
  int32_t refine;            /* one FP32 correction pass with A_master
                                (Rayleigh-Ritz on span(Z) with the FP32 A):
                                0 = on for BK_BF16 / BK_FP8_E4M3 when
                                A_master is given, > 0 on, < 0 off; never
                                for the plain F32 / F64 paths               */
  int32_t center_rows;       /* 1: work on A - mu 1^T, mu = row means of A,
                                applied as rank-1 corrections (PCA centring,
                                Section 1 footnote).  CSR path only.         */
  int32_t max_jacobi_sweeps; /* default 40                                  */
  double jacobi_tol;         /* relative off-diagonal tolerance of the
                                eigen-solve; default 10 sqrt(m) eps64        */
  double breakdown_tol;      /* tau: block i >= 1 whose projected residual
                                has ||.||_F <= tau * (||.||_F before the
                                projection) ends the iteration (q_eff = i-1);
                                block 0 with a pivot of the Cholesky factor
                                of (A Pi)^T (A Pi) <= max(tau, sqrt(11 (n k +
                                k (k+1)) u)) ||A Pi||_F (u = 2^-53: below
                                that, the Gram's rounding decides) gives
                                BK_ERANK.  Default 1e-11 for F64, 1e-5
                                otherwise.                                   */
  const void* pi;            /* nullable: explicit d x k sketch, row-major,
                                ld = k, FP64 for BK_F64 else FP32; overrides
                                the seed                                     */
  int32_t timing;            /* 1: fill bk_info.ms / launches with per-phase
                                GPU times from HIP events on `stream` (each
                                timed phase costs two event records)        */
  int32_t save_for_backward; /* 1: keep R factors / projection coefficients
                                in the workspace for bk_svd_dense_backward   */
  int32_t jacobi_block;      /* column block of the eigen-solve (default by
                                size); a test knob                           */
  int32_t block_size;        /* p: columns of the sketch and of every Krylov
                                block, p >= k (oversampling, Section 6);
                                0 = k.  Rayleigh-Ritz still returns the top
                                k.  The Krylov space has (q+1) p columns
                                (BK_METHOD_BLOCK_KRYLOV) or p (simultaneous
                                iteration); needs save_for_backward = 0 when
                                p != k                                      */
  int32_t method;            /* BK_METHOD_BLOCK_KRYLOV (0, Algorithm 2),
                                BK_METHOD_SIMULTANEOUS (1, Algorithm 1: the
                                block is replaced by orth(A A^T block) q
                                times, Rayleigh-Ritz on the last one) or
                                BK_METHOD_BLOCK_LANCZOS (2, Section 4.2:
                                the Krylov basis of Algorithm 2, with
                                Q^T A A^T Q taken as the block-tridiagonal
                                matrix of the block Lanczos recurrence --
                                diagonal blocks from the projection
                                coefficients, sub-diagonal blocks from the
                                R factors -- instead of the product W^T W;
                                every block is still reorthogonalized
                                against all earlier ones; not with
                                save_for_backward)                          */
  int32_t timing_phases;     /* with timing = 1: bitmask of the BK_PH_*
                                phases given events (1 << BK_PH_AX | ...);
                                0 = all.  Launch counts are kept for all.   */
  int32_t reserved[2];
  double* residuals;         /* nullable DEVICE array of k FP64: the
                                residual norms r_i = ||A A^T z_i -
                                sigma_i^2 z_i||_2 of the returned Ritz
                                pairs, formed after the solve with two more
                                k-wide block products (A: the FP32 master
                                when the correction pass ran, else the
                                matrix the solve used, centred when
                                center_rows).  For the unit vector z_i and
                                the symmetric A A^T, some eigenvalue of
                                A A^T lies within r_i of sigma_i^2
                                (Bauer-Fike), so some singular value s of
                                A has |sigma_i - s| <= r_i / sigma_i.  CSR
                                path: needs block_size = k.             */
  const void* a_transposed;  /* nullable DEVICE matrix: A^T (d x n, ld
                                ld_at) in a_type, BK_BF16 or BK_FP8_E4M3
                                only (bk_quantize_dense_transposed makes
                                it), with at_scales (FP8: the transpose of
                                a_scales, ceil(d/128) x ceil(n/128)).  When
                                given, the A^T Y products (Algorithm 2,
                                step 3) read it row by row, as the A X
                                products read A, instead of A column-wise:
                                the same products, 2 n d bytes of HBM held
                                instead of n d.  Ignored for BK_F32 /
                                BK_F64 and the CSR path.                  */
  int64_t ld_at;             /* leading dimension of a_transposed (>= n)  */
  const float* at_scales;    /* FP8 tile scales of a_transposed (DEVICE)  */
  int32_t fp32_products;     /* FP32 block products on the matrix cores:
                                0 (default): each FP32 operand as three
                                BF16 limbs (a = a1 + a2 + a3 exactly), the
                                six leading limb products on the BF16
                                matrix cores, FP32 sums (error within
                                2^-23 |a b| per product beyond FP32
                                summation); 1: on the FP32 matrix cores
                                (32 x 32 x 2 steps).                     */
  int32_t csr_gather;        /* CSR path: where the sparse products
                                (Theorem 6's nnz(A) k term) gather the rows
                                of their right-hand block from.
                                BK_CSR_GATHER_INPLACE (1): from the
                                Krylov block itself (rows (q+1) p
                                floats apart); BK_CSR_GATHER_STAGED (2):
                                from a copy whose rows start on their own
                                128-byte lines (p rounded up to 32 floats;
                                + (n + d) that many floats of workspace);
                                0: the library's choice (in place).  Same
                                sums in the same order either way.        */
} bk_options;

enum { BK_METHOD_BLOCK_KRYLOV = 0, BK_METHOD_SIMULTANEOUS = 1, BK_METHOD_BLOCK_LANCZOS = 2 };
enum { BK_CSR_GATHER_DEFAULT = 0, BK_CSR_GATHER_INPLACE = 1, BK_CSR_GATHER_STAGED = 2 };

/* Phases of bk_info.ms[] / launches[]. */
enum {
  BK_PH_PI = 0,      /* sketch                                         */
  BK_PH_AX = 1,      /* A X product kernels                            */
  BK_PH_ATY = 2,     /* A^T Y product kernels                          */
  BK_PH_PROJ = 3,    /* block Gram-Schmidt projection                  */
  BK_PH_CHOLQR = 4,  /* Gram + Cholesky + triangular apply             */
  BK_PH_M = 5,       /* M = W^T W                                      */
  BK_PH_EIG = 6,     /* Jacobi eigen-solve + top-k                     */
  BK_PH_Z = 7,       /* Z = Q U_k, sign normalisation                  */
  BK_PH_REFINE = 8,  /* FP32 correction pass                           */
  BK_PH_PREP = 9,    /* CSR validation / transpose / work plans        */
  BK_PH_CENTER = 10, /* CSR operands: centring vectors 1^T X and mu^T Y,
                        staged gather copies (csr_gather)              */
  BK_PH_LONG = 11,   /* CSR: combine of rows cut into several pieces  */
  BK_NPHASE = 12
};

typedef struct bk_info { /* HOST struct, written by the solve calls */
  int32_t q_eff;             /* (A A^T) applications actually used (<= q)   */
  int32_t jacobi_sweeps;     /* sweeps of the eigen-solve                   */
  double jacobi_offdiag;     /* largest relative off-diagonal of the last
                                sweep                                       */
  float ms[BK_NPHASE];       /* per-phase GPU milliseconds (timing = 1)     */
  int32_t launches[BK_NPHASE];/* kernels launched per phase (timing = 1)    */
  int64_t workspace_bytes;   /* bytes of workspace the call used            */
} bk_info;

/* Bytes of workspace bk_svd_dense needs (0 on invalid arguments). */
size_t bk_svd_dense_workspace(int64_t n, int64_t d, int32_t k, int32_t q,
                              int32_t a_type, const bk_options* opt);

/* Block Krylov Iteration on a dense A (Algorithm 2, steps 1-6).
 *
 * A        n x d row-major, leading dimension lda >= d, element type a_type.
 *          BK_FP8_E4M3 additionally needs a_scales: ceil(n/128) x ceil(d/128)
 *          FP32 tile scales, row-major (A[i][j] ~ scale[i/128][j/128] * q_ij).
 * A_master nullable FP32 n x d copy (ld ld_master) used by the correction
 *          pass (opt->refine) of the BF16 / FP8 paths.
 * k, q     rank and depth: 1 <= k, 0 <= q, (q+1) p <= min(n, d) with p
 *          the block width (opt->block_size, default k; for simultaneous
 *          iteration p <= min(n, d)).
 * seed     Philox4x32-10 key of the sketch (see bk_gaussian).
 * Z        n x k output, ld ldz >= k; FP64 for BK_F64, FP32 otherwise.
 *          Column i is the i-th Ritz vector, signed so that its
 *          largest-magnitude entry (lowest row on ties) is positive.
 * ritz     k FP64 Ritz values, descending.
 * info     nullable host struct.
 * workspace / workspace_bytes: device scratch of at least
 *          bk_svd_dense_workspace(...) bytes, or NULL to let the library
 *          allocate (stream-ordered) and free it inside the call.  The
 *          forward workspace is the saved state of bk_svd_dense_backward.
 * A block i >= 1 that breaks down (its projected residual is negligible:
 * the Krylov space is invariant) ends the iteration: info->q_eff = i - 1 and
 * the result is Rayleigh-Ritz over the blocks built so far (BK_OK). */
int bk_svd_dense(const void* A, int64_t lda, int32_t a_type,
                 const float* a_scales, const float* A_master,
                 int64_t ld_master, int64_t n, int64_t d, int32_t k, int32_t q,
                 uint64_t seed, const bk_options* opt, void* Z, int64_t ldz,
                 double* ritz, bk_info* info, void* workspace,
                 size_t workspace_bytes, void* stream);

/* Allocation-free form of bk_svd_dense, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments and results as bk_svd_dense, with
 * no workspace argument: the solve's scratch is a static device array of
 * BK_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is looked up once per device, on the
 * first call there).  The call itself allocates nothing.
 * - Returns BK_ENOMEM, before touching the device, when
 *   bk_svd_dense_workspace(n, d, k, q, a_type, opt) exceeds
 *   BK_NOALLOC_SCRATCH_BYTES; BK_EINVAL as bk_svd_dense, and also for
 *   opt->save_for_backward != 0 (the next call would overwrite the saved
 *   state).  opt->timing is ignored (no per-phase times; launch counts are
 *   still written to info).
 * - Every call on one GPU uses that GPU's one array, which keeps the last
 *   call's contents (the solve initializes what it reads): calls that
 *   overlap on one GPU (different streams, or host threads) race and must
 *   be serialized by the caller, e.g. by issuing them on one stream. */
#define BK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int bk_svd_dense_noalloc(const void* A, int64_t lda, int32_t a_type,
                         const float* a_scales, const float* A_master,
                         int64_t ld_master, int64_t n, int64_t d, int32_t k,
                         int32_t q, uint64_t seed, const bk_options* opt,
                         void* Z, int64_t ldz, double* ritz, bk_info* info,
                         void* stream);

/* Bytes of workspace bk_svd_csr needs (0 on invalid arguments). */
size_t bk_svd_csr_workspace(int64_t n, int64_t d, int64_t nnz, int32_t k,
                            int32_t q, const bk_options* opt);

/* Block Krylov Iteration on a CSR A (Algorithm 2; the products cost
 * O(nnz(A) k) each, Theorem 6).
 * row_ptr  n+1 int32 (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz);
 * col_idx  nnz int32 in [0, d); vals nnz FP32.
 * t_row_ptr / t_col_idx / t_vals: nullable CSR of A^T (d rows, column ids
 *          ascending within each row); built on the GPU when NULL.
 * opt->center_rows applies implicit row centring.
 * The CSR structure is validated on the GPU before any product
 * (BK_EINVAL when it is malformed).
 * Z is n x k FP32 (ldz >= k); ritz k FP64.  Otherwise as bk_svd_dense. */
int bk_svd_csr(const int32_t* row_ptr, const int32_t* col_idx,
               const float* vals, const int32_t* t_row_ptr,
               const int32_t* t_col_idx, const float* t_vals, int64_t n,
               int64_t d, int64_t nnz, int32_t k, int32_t q, uint64_t seed,
               const bk_options* opt, float* Z, int64_t ldz, double* ritz,
               bk_info* info, void* workspace, size_t workspace_bytes,
               void* stream);

/* Error measures of a rank-k basis Z (Section 3 and Section 7):
 * Abar is A, or A - mu 1^T with mu the row means (center_rows, CSR only).
 * eq. (1) uses ||Abar - Z Z^T Abar||_F, obtained from the matrix Pythagorean
 * theorem of Section 3.2 as sqrt(||Abar||_F^2 - ||Z^T Abar||_F^2); eq. (2)
 * uses ||Abar - Z Z^T Abar||_2, estimated as the top Ritz value of a block
 * Krylov solve (Algorithm 2, block width k, depth q_spec, sketch seed `seed`)
 * on the residual operator (I - Z Z^T) Abar, a lower bound that converges
 * to it as q_spec grows (Theorem 1); eq. (3) compares each
 * z_i^T Abar Abar^T z_i with sigma_i^2.  All products run on the GPU. */
typedef struct bk_metrics { /* HOST struct                                  */
  double fro2;          /* ||Abar||_F^2 (FP64 sums of the FP32/FP64 values) */
  double captured_fro2; /* ||Z^T Abar||_F^2 = sum of captured[i]           */
  double resid_fro;     /* ||Abar - Z Z^T Abar||_F                         */
  double resid_spec;    /* ||Abar - Z Z^T Abar||_2 estimate (NaN: residual
                           of rank below k, status BK_ERANK)               */
  double fro_ratio;     /* eq. (1): resid_fro / ||Abar - Abar_k||_F        */
  double spec_ratio;    /* eq. (2): resid_spec / sigma_{k+1}               */
  double per_vector;    /* eq. (3) as reported in Section 7:
                           max_i |sigma_i^2 - captured[i]| / sigma_{k+1}^2
                           (the three ratios are NaN without sigma_true)   */
} bk_metrics;

/* Bytes of workspace bk_error_metrics_dense needs (0 on invalid arguments:
 * a_type other than BK_F64 / BK_F32, or (q_spec+1) k > min(n, d)). */
size_t bk_error_metrics_dense_workspace(int64_t n, int64_t d, int32_t k,
                                        int32_t q_spec, int32_t a_type);

/* Error measures of Z against a dense A (device, n x d row-major, ld lda,
 * BK_F64 or BK_F32; Z device n x k, ld ldz >= k, the same type, orthonormal
 * columns, e.g. the output of bk_svd_dense).
 * sigma_true  nullable HOST array of n_sigma >= k+1 FP64 singular values of
 *             A, descending; with n_sigma >= min(n, d) the tail
 *             ||A - A_k||_F^2 is summed from them, otherwise taken as
 *             ||A||_F^2 - sum_{i<=k} sigma_i^2.
 * captured    nullable HOST array of k FP64: z_i^T A A^T z_i.
 * out         nullable HOST struct.
 * workspace   device scratch of bk_error_metrics_dense_workspace(...) bytes
 *             or NULL (allocated and freed inside, stream-ordered).
 * Synchronizes `stream`.  Returns BK_ERANK when the residual has rank below
 * k (every other field is still written). */
int bk_error_metrics_dense(const void* A, int64_t lda, int32_t a_type,
                           int64_t n, int64_t d, const void* Z, int64_t ldz,
                           int32_t k, int32_t q_spec, uint64_t seed,
                           const double* sigma_true, int64_t n_sigma,
                           double* captured, bk_metrics* out, void* workspace,
                           size_t workspace_bytes, void* stream);

/* Bytes of workspace bk_error_metrics_csr needs (0 on invalid arguments). */
size_t bk_error_metrics_csr_workspace(int64_t n, int64_t d, int64_t nnz,
                                      int32_t k, int32_t q_spec);

/* As bk_error_metrics_dense for a CSR A (arrays as bk_svd_csr, validated on
 * the GPU first: BK_EINVAL when malformed), Z FP32 n x k; center_rows != 0
 * measures against the row-centred A - mu 1^T (footnote on PCA, Section 1),
 * never formed. */
int bk_error_metrics_csr(const int32_t* row_ptr, const int32_t* col_idx,
                         const float* vals, const int32_t* t_row_ptr,
                         const int32_t* t_col_idx, const float* t_vals,
                         int64_t n, int64_t d, int64_t nnz, int32_t center_rows,
                         const float* Z, int64_t ldz, int32_t k, int32_t q_spec,
                         uint64_t seed, const double* sigma_true,
                         int64_t n_sigma, double* captured, bk_metrics* out,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Reverse-mode adjoint of bk_svd_dense for the FP32 and FP64 plain paths.
 * Inputs: the same A / n / d / k / q / a_type as the forward, the forward's
 * workspace (opt->save_for_backward = 1 in the forward, unmodified since),
 * its outputs Z and ritz, and the cotangents Z_bar (n x k, ld ldz, nullable
 * = 0) and ritz_bar (k FP64, nullable = 0).  Writes A_bar (n x d, ld ld_bar,
 * same type as A) = d(loss)/dA, where loss is any function of (Z, ritz) whose
 * value is unchanged by rotations within span(Z) (e.g. sum of the Ritz
 * values, ||Z Z^T A||_F^2).  Krylov blocks are recomputed from the saved
 * orthonormal blocks, not stored.  Pi gets no gradient. */
size_t bk_svd_dense_backward_workspace(int64_t n, int64_t d, int32_t k,
                                       int32_t q, int32_t a_type);
int bk_svd_dense_backward(const void* A, int64_t lda, int32_t a_type,
                          int64_t n, int64_t d, int32_t k, int32_t q,
                          const void* Z, int64_t ldz, const double* ritz,
                          const void* Z_bar, const double* ritz_bar,
                          void* A_bar, int64_t ld_bar,
                          const void* fwd_workspace, size_t fwd_bytes,
                          void* workspace, size_t workspace_bytes,
                          void* stream);

/* The sketch of Algorithm 2, step 1: out = rows x cols N(0,1), row-major
 * with leading dimension ld >= cols, type BK_F64 or BK_F32 (rounded once from
 * FP64).  Element e = r*cols + c; normals 2j and 2j+1 come from one
 * Philox4x32-10 call (Salmon et al., SC'11) with counter (j mod 2^32,
 * j div 2^32, 0, 0) and key (seed mod 2^32, seed div 2^32), words x0..x3:
 *   u1 = ((x0 >> 5) 2^26 + (x1 >> 6) + 1) 2^-53,
 *   u2 = ((x2 >> 5) 2^26 + (x3 >> 6)) 2^-53,
 *   z_2j = sqrt(-2 ln u1) cos(2 pi u2), z_2j+1 = sqrt(-2 ln u1) sin(2 pi u2). */
int bk_gaussian(uint64_t seed, int64_t rows, int64_t cols, int64_t ld,
                int32_t dtype, void* out, void* stream);

/* Raw Philox4x32-10: in = count x 6 uint32 (ctr0..3, key0, key1),
 * out = count x 4 uint32. */
int bk_philox4x32_10(const uint32_t* in, int64_t count, uint32_t* out,
                     void* stream);

/* Low-precision copy of a FP32 A (n x d, ld lda) into out (n x d, ld = d):
 * to = BK_BF16: round to nearest even; to = BK_FP8_E4M3: per 128 x 128 tile,
 * s = amax(tile) / 448 (s = 1 for an all-zero tile), q = RNE-saturate(a / s)
 * in OCP e4m3, tile_scales[ceil(n/128) x ceil(d/128)] = s. */
int bk_quantize_dense(const float* A, int64_t n, int64_t d, int64_t lda,
                      int32_t to, void* out, float* tile_scales, void* stream);

/* The same copy stored transposed: out_t (d x n, ld = n) holds at (c, r) the
 * code bk_quantize_dense gives A[r][c]; FP8 tile_scales_t[ceil(d/128) x
 * ceil(n/128)] is the transpose of its tile scales.  For
 * bk_options.a_transposed. */
int bk_quantize_dense_transposed(const float* A, int64_t n, int64_t d, int64_t lda,
                                 int32_t to, void* out_t, float* tile_scales_t,
                                 void* stream);

/* The block products on their own (the Krylov loop's A.X and A^T.Y,
 * Algorithm 2, steps 2-3):
 * trans = 0: Y (n x k, ld ldy) = A X, X d x k (ld ldx);
 * trans = 1: Y (d x k, ld ldy) = A^T X, X n x k (ld ldx).
 * X and Y are FP64 for a_type BK_F64, FP32 otherwise.  The A^T X form uses a
 * split reduction with FP64 partial sums.  Workspace:
 * bk_dense_product_workspace(...) bytes (NULL: allocated in the call).
 * Matrix cores: for FP32 / BF16 / FP8 A whose rows are 16-byte aligned and
 * whose reduction length is a multiple of 128 bytes of A's type (A X) or
 * whose column count is a multiple of 16 bytes (A^T X), and for products of
 * at least 1e8 (A X) or 1e9 (A^T X) flops, X is packed in A's type (BF16:
 * round to nearest even; FP8: one scale amax / 448 per 128 rows of X) and
 * the product runs on MFMA with FP32 chunk sums; other shapes run on the
 * vector units with X in FP32. */
size_t bk_dense_product_workspace(int32_t trans, int64_t n, int64_t d,
                                  int32_t k, int32_t a_type);
int bk_dense_product(int32_t trans, const void* A, int64_t lda, int32_t a_type,
                     const float* a_scales, int64_t n, int64_t d,
                     const void* X, int64_t ldx, int32_t k, void* Y,
                     int64_t ldy, void* workspace, size_t workspace_bytes,
                     void* stream);

/* CSR product Y = A X (n x k) for FP32 CSR A and FP32 X (d x k); run on the
 * CSR of A^T it gives A^T X.  No centring. */
int bk_csr_product(const int32_t* row_ptr, const int32_t* col_idx,
                   const float* vals, int64_t rows, int64_t cols, int64_t nnz,
                   const float* X, int64_t ldx, int32_t k, float* Y,
                   int64_t ldy, void* stream);

/* CSR of A^T (cols rows) from the CSR of A, column ids ascending within each
 * output row.  workspace: bk_csr_transpose_workspace(...) bytes or NULL. */
size_t bk_csr_transpose_workspace(int64_t rows, int64_t cols, int64_t nnz);
int bk_csr_transpose(const int32_t* row_ptr, const int32_t* col_idx,
                     const float* vals, int64_t rows, int64_t cols,
                     int64_t nnz, int32_t* t_row_ptr, int32_t* t_col_idx,
                     float* t_vals, void* workspace, size_t workspace_bytes,
                     void* stream);

/* Eigen-decomposition of a symmetric positive semi-definite FP64 matrix
 * (the Rayleigh-Ritz step 5; SVD = eig for PSD M, Lemma 1): M is m x m
 * (ld ldm, read only), theta (m, descending, ties by lower index) and
 * V (m x m, ld ldv, column j the eigenvector of theta_j, largest-|.| entry
 * positive).  Synchronizes `stream`; sweeps (nullable host) receives the
 * sweep count.  workspace: bk_eigh_psd_workspace(m) bytes or NULL. */
size_t bk_eigh_psd_workspace(int64_t m);
int bk_eigh_psd(const double* M, int64_t m, int64_t ldm, double* theta,
                double* V, int64_t ldv, int32_t max_sweeps, double tol,
                int32_t* sweeps, void* workspace, size_t workspace_bytes,
                void* stream);

/* Static text for a bk_status value. */
const char* bk_status_string(int status);

/* Library version string ("bk <major>.<minor> gfx950"). */
const char* bk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BK_H */
