/*
 * rbrp.h -- C ABI of an MI355X (gfx950) library for adaptive robust blockwise
 * random pivoting (RBRP) interpolative decompositions.
 *
 * Method: Dong, Chen, Martinsson, Pearce, "Robust blockwise random pivoting:
 * fast and accurate adaptive interpolative decomposition", arXiv:2309.16002.
 * The library computes a row interpolative decomposition X ~= W X(S,:) (the
 * (r, eps)-ID problem statement, eq. id) with the skeletons S chosen by
 * Algorithm 2 and W = X X_S^+ (eq. stable_id) obtained from Algorithm 3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major with a leading dimension (elements between row
 *   starts) >= the number of columns.  The paper's n x d data matrix is
 *   m x n here: m rows (data points), n columns (features).
 * - Pointers are DEVICE pointers unless the argument name ends in _host.
 *   The caller owns every buffer; the library keeps no pointer after return.
 * - ``stream`` is a hipStream_t passed as void* (NULL = the null stream).
 *   All device work is ordered on that stream.
 * - Arguments are validated before any device work is issued.  On
 *   RBRP_E_INVALID / RBRP_E_WORKSPACE nothing is written anywhere.
 * - No entry point allocates device memory: every scratch buffer lives in the
 *   caller-provided workspace (size from rbrp_workspace_size), except for
 *   rbrp_id_batched_noalloc, whose scratch is a static 256 MiB device array
 *   of the library.  The library holds one small pinned host buffer per
 *   process for the per-block stop test.
 * - Calls that share a workspace must not overlap; distinct workspaces on
 *   distinct streams are independent.
 */
#ifndef RBRP_H_
#define RBRP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBRP_OK = 0,
  RBRP_E_INVALID = 1,     /* an argument is out of range or a pointer is NULL */
  RBRP_E_WORKSPACE = 2,   /* ws_bytes < rbrp_workspace_size(...)               */
  RBRP_E_HIP = 3,         /* a HIP runtime call failed                        */
  RBRP_E_NONFINITE = 4,   /* X holds a NaN or an infinity                     */
  RBRP_E_CAPACITY = 5,    /* the tolerance was not met within k_max skeletons;
                             S, k and W describe the k_max skeletons chosen   */
  RBRP_E_UNSUPPORTED = 6  /* a valid combination the library does not provide */
} rbrp_status;

typedef enum { RBRP_F32 = 0, RBRP_F64 = 1 } rbrp_dtype;

/* Arithmetic of the two deflation GEMMs R Q' and (R Q') Q'^T.
 * NATIVE: the input's type on MFMA (FP64 for F64 input; FP32 for F32 input,
 *         the "plain" single-precision form).
 * BF16:   BF16 MFMA operands with FP32 accumulation; per block one BF16
 *         product on a residual stored in BF16 (half the bytes), one BF16
 *         product or hi+lo split BF16 parts (three products) on an FP32
 *         residual, or the FP32 product, the cheapest that the error budget
 *         of rbrp_options.theta allows.
 * In every mode the residual norms, the projection and reorthogonalisation
 * of the basis, the block CPQR and the solve for W are FP64. */
typedef enum { RBRP_PREC_NATIVE = 0, RBRP_PREC_BF16 = 1 } rbrp_precision;

typedef struct {
  double tau_b;        /* filter tolerance of Alg. 2 (Remark 4.2): < 0 -> 1/b
                          (RBRP, the default); 0 -> plain BRP (no filter:
                          every sampled row is kept while the block's
                          pivoted factor stays positive definite); at most 1 */
  int64_t k_max;       /* capacity of S and W; <= 0 -> min(m, n)                */
  int32_t fixed_rank;  /* 1: ignore eps and stop at |S| = k_max (Alg. 2, "or k") */
  int32_t greedy;      /* 1: take the b largest residual norms instead of
                          sampling (RBGP, Remark 4.3)                           */
  int32_t precision;   /* rbrp_precision                                         */
  int32_t w_refine;    /* iterative-refinement steps of the FP64 W solve
                          (Alg. 3); < 0 -> 1                                  */
  double theta;        /* BF16 mode.  > 0: split products while the tracked
                          relative residual is above theta, one BF16 product
                          below it (FP32 residual).  <= 0 (the default):
                          every block takes the cheapest of one BF16 product
                          with a BF16-stored residual, one BF16 product and
                          the split BF16 products on an FP32 residual, and
                          the FP32 product, whose contribution, if kept for
                          the later blocks, holds the error bound err_bound
                          (rbrp_stats) within eps / 4                    */
  int32_t profile;     /* 1: time the phases with HIP events on ``stream`` and
                          report them in rbrp_stats; 2: time only the
                          deflation launches (ms_deflate, deflate_launches)    */
  int32_t trim;        /* 1: rank trimming.  The stopping rule of Alg. 2 runs
                          between blocks, so the last block can add up to
                          b' - 1 rows more than eps needs; with trim the
                          returned k is the shortest prefix S(1:k) whose
                          tracked error meets eps (the last block's columns
                          taken one at a time: the block's starting residual
                          minus the squared norms of its columns of L, which
                          is the prefix's error by Pythagoras over the
                          orthonormal basis), and W is formed for that
                          prefix.  Ignored with fixed_rank and in the BF16
                          precision form (its tracked residual carries the
                          BF16 rounding, which the whole last block's slack
                          covers).  0: keep every selected row (the paper's
                          rule)                                              */
  const double* replay_d; /* test hook (device, FP64 [replay_blocks x m], row
                          t-1 = the squared residual row norms that block t
                          samples from), used when replay_blocks > 0: block t
                          draws from row t-1 instead of the tracked norms (the
                          weights, the Philox stream and the exclusion of rows
                          already in S are unchanged), and the loop runs
                          exactly replay_blocks blocks (fewer only if k_max is
                          reached or a block lies in span(Q)) instead of
                          applying the stopping rule.  Fed the norms another
                          implementation drew from, the skeletons of every
                          block can be compared with its, whatever the
                          deflation's precision.  NULL / 0: off           */
  int32_t replay_blocks;
  int32_t w_method;    /* 0: W = L_2 L_1^{-1} by blocked substitution with
                          w_refine refinement steps (Alg. 3; the default).
                          1: W = L_2 L_1^+ through the truncated SVD of L_1
                          (Remark 5.2): singular values below
                          w_clip * sigma_max(L_1) and their singular vectors
                          are dropped (one-sided Jacobi SVD in FP64, then
                          W = L L_1^+ as one product; w_refine is ignored).
                          W(S,:) = I in both                              */
  double w_clip;       /* w_method 1: relative clip; <= 0 -> 1e-12        */
} rbrp_options;

/* Per-call statistics (optional, host memory). */
typedef struct {
  int32_t blocks;          /* T, the number of sampled blocks                 */
  int32_t blocks_split;    /* BF16 mode: blocks deflated with hi+lo products  */
  double resid_tracked;    /* sqrt(||d||_1 / ||d^(0)||_1) at exit             */
  double err_bound;        /* E_T: bound on ||R - X (I - Q Q^T)||_F / ||X||_F
                              for the part of the deflation rounding that can
                              lower the tracked residual below the optimal
                              error on S (see rbrp_err_bound_increment); the
                              loop stops when resid_tracked + err_bound <= eps */
  double norm_x_fro;       /* ||X||_F                                         */
  /* filled when rbrp_options.profile = 1 (milliseconds, HIP events; with
     profile = 2 only ms_deflate, deflate_flops and deflate_launches) */
  double ms_init;          /* copy X -> residual, initial norms               */
  double ms_select;        /* weights, CDF and sampling, all blocks           */
  double ms_filter;        /* gather, projection, block CPQR, basis, all blocks */
  double ms_deflate;       /* the fused deflation kernel, all blocks          */
  double ms_interp;        /* W from L (Algorithm 3)                          */
  double deflate_flops;    /* algorithmic flops of the deflations: sum 4 m n b' */
  int32_t deflate_launches;
  int32_t blocks_native;   /* BF16 mode: blocks the controller deflated with
                              the FP32 product                              */
  double deflate_bytes;    /* algorithmic HBM bytes of the deflations: per
                              launch the residual read and written (m n
                              values each, in its storage type), d written;
                              per block the new columns of L              */
  int32_t blocks_bf16_stored; /* BF16 mode: blocks whose output residual was
                              stored in BF16                              */
  int32_t w_rank;          /* singular values of L_1 kept (w_method 1); k
                              with substitution                          */
  int32_t bprime[256];     /* b' of the first 256 blocks                       */
} rbrp_stats;

/* Fill *opt with the defaults (tau_b = 1/b, k_max = min(m, n), sampling,
 * NATIVE precision, one refinement step of the W solve). */
void rbrp_default_options(rbrp_options* opt);

/* Bytes of device workspace rbrp_id needs for these arguments (0 when the
 * arguments are invalid). */
size_t rbrp_workspace_size(rbrp_dtype dtype, int64_t m, int64_t n, int32_t b,
                           const rbrp_options* opt);

/*
 * Row interpolative decomposition by RBRP (Algorithm 2, then Algorithm 3).
 *
 * Computes skeleton rows S and W with X ~= W X(S,:), stopping at the first
 * block boundary where ||X - W X(S,:)||_F <= eps ||X||_F as tracked by the
 * residual squared row norms (Alg. 2 stopping rule with tau = eps^2; the
 * rank-adaptive property of the paper's introduction).  The tracked value
 * carries the rounding of the deflation products, so the rule applied is
 * rho + E <= eps, rho = sqrt(||d||_1 / ||d^(0)||_1) and E the running
 * bound err_bound of rbrp_stats (about 1e-7 for FP32 products; for the BF16
 * form at most eps / 4 under the default controller).
 *
 * X      [m x n], ld ldx, dtype F32 or F64; read only.  m <= 4096 * 2048
 *        (the sampler's integer CDF tiles); larger m -> RBRP_E_UNSUPPORTED.
 * eps    relative Frobenius tolerance, 0 < eps < 1 (ignored if fixed_rank).
 * b      block size, 1 <= b <= 256.  Blocks with b' > 128 kept rows are
 *        deflated in two launches (columns 1..128, then the rest); for
 *        b > 128 the host also reads b' once per block before deflating.
 * seed   key of the Philox4x64-10 stream: candidate j of block t draws word 0
 *        of Philox(counter = (j, t, 0, 0), key = (seed, 0)).
 * opt    NULL for defaults.
 * S      [k_max] int64: skeleton row indices (0-based) in selection order.
 * k_host host int64: k = |S|.
 * W      [m x k_max] FP64, ld ldw >= k_max: W(S(j), :) = e_j^T; columns >= k
 *        are left untouched.  May be NULL to skip the interpolation matrix.
 * stats_host optional (NULL allowed).
 * workspace, ws_bytes  device scratch of at least rbrp_workspace_size bytes.
 *
 * The call blocks the host once per block (to read the stop test) and
 * returns after the stream has finished the call's work.
 */
rbrp_status rbrp_id(const void* X, rbrp_dtype dtype, int64_t m, int64_t n,
                    int64_t ldx, double eps, int32_t b, uint64_t seed,
                    const rbrp_options* opt, int64_t* S, int64_t* k_host,
                    double* W, int64_t ldw, rbrp_stats* stats_host,
                    void* workspace, size_t ws_bytes, void* stream);

/* Static text for a status code. */
const char* rbrp_status_string(rbrp_status s);

/*
 * Increment of the squared error bound after one deflated block (host
 * arithmetic only; no device work).  The block removed P = R Q' from the
 * stored residual R (Alg. 2's L-hat update in explicit form); its products
 * round Q' to the operand precision of ``mode`` and accumulate in FP32 (FP64
 * for mode 0).  Rounding that lands in span(Q') only raises the tracked norm
 * (it is orthogonal to X (I - Q Q^T) for every later basis); the rest -- the
 * operand rounding of Q' in the update P Q'^T (applied to P and to the
 * error of P), the product a split form drops and the accumulator rounding --
 * is bounded under the model of independent, mean-zero relative rounding
 * errors uniform in [-u, u] (variance u^2 / 3):
 *
 *   v = (s_q^2 + s_x^2) p^2 + ((s_q u_op)^2 + s_a^2 (bprime / kstep + 1)) r_prev^2,
 *   p^2 = max(r_prev^2 - r_new^2, 0),
 *
 * with r_prev^2, r_new^2 the tracked squared residual norms before and after
 * the block (relative to ||X||_F^2), s_q the operand-rounding deviation of
 * Q' (u / sqrt 3, u = 2^-53, 2^-24, 2^-16 for split BF16, 2^-8 for BF16), s_x
 * that of the dropped lo*lo product (2^-16 / sqrt 3, split only), u_op the
 * relative error bound of the product R Q' (2u; 3 * 2^-16 split), s_a the
 * accumulator's (2^-24 / sqrt 3; 2^-53 / sqrt 3 for FP64) and kstep the
 * columns one MFMA step adds (4 for FP64/FP32, 32 for BF16).  A residual
 * stored in BF16 after the block adds (2^-8 / sqrt 3)^2 r_new^2: its
 * rounding lies in every direction, and later blocks may move all of it
 * into L.
 * The bound after block t is err_bound = 3 sqrt(sum of v over blocks 1..t).
 * mode: 0 FP64, 1 FP32, 2 split BF16 (hi + lo, three products), 3 BF16,
 * 4 BF16 with the output residual stored in BF16 (5: the same, from a
 * BF16-stored residual).
 * Returns a negative value for an unknown mode or bprime < 0.
 */
double rbrp_err_bound_increment(int32_t mode, int32_t bprime, double r_prev_sq,
                                double r_new_sq);

/* ---- single-step entry points (the steps of Algorithm 2 in isolation) ---- */

/*
 * Squared row norms d_i = ||x_i||^2 of Alg. 2's initialisation, accumulated
 * in FP64 from X of type dtype.  d [m] FP64.  Also returns, on the host,
 * sum_i d_i and max_i d_i (either pointer may be NULL).  Fails with
 * RBRP_E_NONFINITE if X holds a NaN or infinity.  workspace of at least
 * rbrp_row_norms_workspace_size(m) bytes.
 */
size_t rbrp_row_norms_workspace_size(int64_t m);
rbrp_status rbrp_row_norms(const void* X, rbrp_dtype dtype, int64_t m,
                           int64_t n, int64_t ldx, double* d,
                           double* sum_host, double* max_host,
                           void* workspace, size_t ws_bytes, void* stream);

/*
 * Block sampling of Alg. 2: up to b distinct indices drawn without
 * replacement from d / ||d||_1, excluding rows with excluded[i] != 0 (may be
 * NULL).  d [m] FP64 (entries <= 0 have no mass), excluded [m] uint8.
 * Fixed-point weights w_i = floor(max(d_i,0) 2^s), s = 62 - e - ceil(log2 m)
 * where max d = f 2^e, f in [0.5, 1); candidate j maps Philox word x_j to the
 * smallest i with C_i > floor(x_j W / 2^64) (C the inclusive prefix of w);
 * first occurrences are accepted; after 32 b candidates the accepted rows are
 * removed from the CDF and each further candidate is accepted.  If at most b
 * rows have positive weight they are all returned in index order.
 * idx [b] int64 device, n_host: number written.  ``ident`` is counter word 2.
 * workspace of at least rbrp_sample_workspace_size(m) bytes.
 */
size_t rbrp_sample_workspace_size(int64_t m);
rbrp_status rbrp_sample_block(const double* d, const uint8_t* excluded,
                              int64_t m, int32_t b, uint64_t seed, uint64_t t,
                              uint64_t ident, int64_t* idx, int32_t* n_host,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * Robust blockwise filter of Alg. 2 (local CPQR + truncation, Remark 4.2) on
 * one block.  Vt [nb x n] FP64, ld ldv: row j is column j of the paper's V
 * (the residual of the j-th sampled row).  Pivot = largest remaining residual
 * norm, ties to the lowest j; b' = max{i : ||R_V(i:nb,i:nb)||_F^2 >=
 * tau_b ||R_V||_F^2 (1 - 4 nb 2^-53)}.
 * piv [nb] int32 (first b' entries meaningful), R [nb x nb] FP64 row-major:
 * the first b' rows of R_V in pivoted column order (upper triangular part),
 * Qt [nb x n] FP64 ld ldq: first b' rows = orthonormal basis of the kept
 * columns (Q_V(:,1:b')^T, signs with positive diagonal of R_V).
 * bprime_host: b'.  1 <= nb <= 256.
 */
size_t rbrp_block_cpqr_workspace_size(int64_t n, int32_t nb);
rbrp_status rbrp_block_cpqr(const double* Vt, int64_t n, int32_t nb,
                            int64_t ldv, double tau_b, int32_t* piv,
                            double* R, double* Qt, int64_t ldq,
                            int32_t* bprime_host, void* workspace,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Sketchy pivoting with LU and partial pivoting (SkLUPP) and the oversampled
 * sketchy interpolation matrix (OSID, Algorithm 4): the fixed-rank
 * comparison method of section 3 ("sketchy pivoting") and section 5.
 *
 *   Y = X Omega                (m x l, FP64; X in its own type)
 *   S = the first k pivot rows of Gaussian elimination with partial pivoting
 *       on Y(:, 0:k) (the active row with the largest |entry| of the current
 *       column, ties to the lowest row; a column with no nonzero active entry
 *       pivots on its lowest active row and eliminates nothing)
 *   W = Y Y(S,:)^+ by Alg. 4: Y(S,:)^T = Q R (Householder), W = (Y Q) R^{-T},
 *       W(S,:) = I            (only when W is not NULL)
 *
 * X      [m x n] row-major, ld ldx, F32 or F64; read only.  m <= 4096 * 2048.
 * k, l   1 <= k <= min(m, l), l <= 65536 (l = 3k is the paper's choice).
 * Omega  device, FP64 [n x l] row-major, ld ldo >= l: the embedding (the
 *        paper draws it Gaussian; the caller supplies it).
 * S      device int64 [k]: skeleton rows in pivot order.
 * W      device FP64 [m x ldw], ldw >= k, or NULL (skeletons only).
 * Y(S,:) must have full rank k for W (a zero diagonal of R gives
 * non-finite W).  Validation as for rbrp_id; stream-ordered, no host
 * synchronisation.
 * ------------------------------------------------------------------------ */
size_t rbrp_sketchy_workspace_size(rbrp_dtype dtype, int64_t m, int64_t n,
                                   int32_t k, int32_t l);
rbrp_status rbrp_sketchy_id(const void* X, rbrp_dtype dtype, int64_t m,
                            int64_t n, int64_t ldx, int32_t k, int32_t l,
                            const double* Omega, int64_t ldo, int64_t* S,
                            double* W, int64_t ldw, void* workspace,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent IDs (for instance the off-diagonal blocks of
 * a hierarchical-matrix compression, the fast-direct-solver use the paper
 * motivates in section 6) in one persistent launch.  Each ID runs the same
 * Alg. 2 + Alg. 3 as rbrp_id with options tau_b, fixed_rank and w_refine
 * (greedy selection, the BF16 form and the truncated-SVD W are not provided
 * here: RBRP_E_UNSUPPORTED); the Philox
 * counter of ID i is (j, t, i, 0), i = its index in ``descs``.  The deflation
 * products run in the input's precision on the vector ALUs; norms, basis and
 * W are FP64.  No host synchronisation, no allocation and no memset: the call
 * may be captured in a HIP graph and replayed.
 * ------------------------------------------------------------------------ */
typedef struct {
  const void* X;     /* device, m x n row-major (ldx >= n), dtype of the call */
  int64_t m, n, ldx;
  int64_t* S;        /* device [k_cap]: skeleton rows in selection order       */
  double* W;         /* device m x ldw FP64 row-major (ldw >= k_cap), or NULL:
                        columns 0..k-1 written, W(S,:) = I                     */
  int64_t ldw;
  int32_t k_cap;     /* 1 <= k_cap <= min(m, n, shape.k_cap_max)                */
  int32_t b;         /* block size 1..shape.b_max; 0 -> shape.b_max             */
} rbrp_batch_desc;

typedef struct {
  int64_t m_max;      /* largest m, <= 16384                                   */
  int64_t n_max;      /* largest n, <= 256                                     */
  int32_t b_max;      /* largest b, <= 32                                      */
  int32_t k_cap_max;  /* largest k_cap, <= 256                                 */
  int32_t num_wg;     /* persistent workgroups; 0 -> 512 (two per CU)          */
  int32_t row_depth;  /* deflation: 8-value chunks of a row whose loads are
                         issued together (1, 2 or 4) per size class, 4 bits
                         each: bits 0-3 n <= 64, 4-7 n <= 128, 8-11 larger;
                         a field of 0 -> 2 (rbrp_batch_autotune sets it)  */
} rbrp_batch_shape;

/* Workspace bytes of rbrp_id_batched for this shape (per-workgroup scratch
 * sized for the largest ID); 0 if the shape is out of range. */
size_t rbrp_batch_workspace_size(rbrp_dtype dtype, const rbrp_batch_shape* shape);

/*
 * count IDs described by descs [count] (device).  order [count] (device, may
 * be NULL): the queue order, a permutation of 0..count-1 (largest IDs first
 * balances the tail; rbrp_batch_autotune computes one).  Outputs per ID i
 * (device): k_out[i] = |S|, status_out[i] (RBRP_OK, RBRP_E_CAPACITY,
 * RBRP_E_NONFINITE, RBRP_E_INVALID for a descriptor outside the shape,
 * RBRP_E_HIP if a block lost orthogonality), resid_out[i] (may be NULL):
 * tracked relative residual.  Host-side validation covers the scalar
 * arguments and the shape only; descriptors are checked on the device.
 */
rbrp_status rbrp_id_batched(const rbrp_batch_desc* descs, const int32_t* order,
                            int32_t count, rbrp_dtype dtype, double eps,
                            uint64_t seed, const rbrp_options* opt,
                            const rbrp_batch_shape* shape, int32_t* k_out,
                            int32_t* status_out, double* resid_out,
                            void* workspace, size_t ws_bytes, void* stream);

/*
 * rbrp_id_batched without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The per-workgroup scratch comes from a
 * static device array of 256 MiB inside the library (one per GPU, held until
 * the process ends; its address is looked up on the first call on each
 * device).  Same arguments, kernels and results as rbrp_id_batched.  The
 * persistent grid is shape->num_wg workgroups (0 -> 512) or as many as the
 * array holds, whichever is fewer; the queue hands out the IDs, so the
 * count changes no result.  A shape whose single workgroup needs more than
 * the array -> RBRP_E_WORKSPACE (validated before any device work).
 * ``stream`` must belong to the current device (else RBRP_E_INVALID).
 * Allocates nothing: no hipMalloc, hipFree, memset or allocating library
 * call.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (concurrent streams or
 * threads) race and must be serialised by the caller.
 */
rbrp_status rbrp_id_batched_noalloc(const rbrp_batch_desc* descs,
                                    const int32_t* order, int32_t count,
                                    rbrp_dtype dtype, double eps, uint64_t seed,
                                    const rbrp_options* opt,
                                    const rbrp_batch_shape* shape,
                                    int32_t* k_out, int32_t* status_out,
                                    double* resid_out, void* stream);

/*
 * Autotuner of the batched form.  descs_host [count] is the host copy of the
 * descriptors, descs [count] their device copy.  Size classes by n
 * (<= 64, <= 128, > 128); for each class the block sizes 8, 16 and 32
 * (<= shape->b_max) are timed on that class's IDs, then, with that b, the
 * deflation's row-load depths 1, 2 and 4; then the number of persistent
 * workgroups (256, 512, 768, those the workspace fits).  On return the
 * device descriptors carry the chosen b, order [count] (device) holds the
 * largest-first queue order, shape->num_wg and shape->row_depth the chosen
 * count and depths, and b_class_host [3] the block size per class.  Synchronises the stream; runs
 * the batch several times (outputs are overwritten).
 */
rbrp_status rbrp_batch_autotune(const rbrp_batch_desc* descs_host,
                                rbrp_batch_desc* descs, int32_t count,
                                rbrp_dtype dtype, double eps, uint64_t seed,
                                const rbrp_options* opt, rbrp_batch_shape* shape,
                                int32_t* order, int32_t* k_out,
                                int32_t* status_out, double* resid_out,
                                void* workspace, size_t ws_bytes, void* stream,
                                int32_t* b_class_host);

#ifdef __cplusplus
}
#endif

#endif /* RBRP_H_ */
