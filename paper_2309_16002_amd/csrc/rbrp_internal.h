// Internal declarations shared by the HIP translation units of the RBRP
// library: launch wrappers (one per kernel family) and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "rbrp.h"

namespace rbrp {

constexpr int kWave = 64;

// Rows of the residual buffer are padded to a multiple of this.
constexpr int kRowPad = 64;
// Rows per workgroup of the norm / weight kernels.
constexpr int kNormRowsPerWG = 64;
constexpr int kNtMaxSlices = 4;     // K slices of the small NT products (see launch_gemm_nt_small)
constexpr int kScanTile = 2048;   // rows per tile of the fixed-point CDF
constexpr int kMaxB = 256;        // largest block size
constexpr int kDeflateMaxB = 128; // largest b' of one deflation launch
constexpr int kRejectionFactor = 32;
constexpr int kMaxScanTiles = 4096;  // tiles of the integer CDF (k_sample.hip)
constexpr int64_t kMaxRows = (int64_t)kMaxScanTiles * kScanTile;

__host__ __device__ inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
__host__ __device__ inline int64_t ceil_div(int64_t x, int64_t a) { return (x + a - 1) / a; }

// Device-resident scalars of one decomposition, written by the kernels and
// read by the host once per block.
struct DevScalars {
  double sum_d;        // ||d||_1
  double max_d;        // max_i d_i over rows not in S
  double d0;           // ||d^(0)||_1
  double tail1;        // ||V||_F^2 of the last block
  double xs2;          // ||X(S_t,:)||_F^2 of the last block
  int32_t nonfinite;   // X holds NaN/Inf
  int32_t nt;          // rows drawn in the last block
  int32_t bprime;      // b' of the last block
  int32_t stop_rank;   // last block numerically inside span(Q)
  int32_t npos;        // rows with positive weight
  int32_t b2;          // steps completed by the reorthogonalisation Cholesky
  int32_t need_exact;  // reorthogonalisation needs the exact Cholesky
  int32_t bchunk[2];   // b' of the two deflation launches when b > kDeflateMaxB
  int32_t pad[1];
};

// ---- launch wrappers (defined next to their kernels) ----

// R <- X (cast, zero padded to ldr columns and mr rows), d_i = ||x_i||^2,
// per-workgroup partial sums / maxima, non-finite flag.
hipError_t launch_init_norms(const void* X, rbrp_dtype dt, int64_t m, int64_t n,
                             int64_t ldx, void* R, int r_is_f64, int64_t mr,
                             int64_t ldr, double* d, double* part_sum,
                             double* part_max, int32_t* nonfinite,
                             hipStream_t s);
int64_t norms_num_partials(int64_t mr);

// Per-workgroup sum / max of max(d_i, 0) over rows with excluded[i] == 0
// (the sampler's scale when rows are excluded by a mask).
hipError_t launch_masked_partials(const double* d, const uint8_t* excluded,
                                  int64_t m, double* part_sum, double* part_max,
                                  hipStream_t s);
int64_t masked_num_partials(int64_t m);
// Squared norms (FP64) of columns c0 .. c0 + nc - 1 (nc <= 256) of L (m rows,
// ld ldl; FP64 if l_f64, else FP32) into out[nc]; part holds
// col_sumsq_groups(m) * nc doubles of partial sums.
int col_sumsq_groups(int64_t m);
hipError_t launch_col_sumsq(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t c0,
                            int nc, double* part, double* out, hipStream_t s);

// Fixed-order reduction of partial sums / maxima into sc->sum_d, sc->max_d
// (and sc->d0 when set_d0).
hipError_t launch_reduce(const double* part_sum, const double* part_max,
                         int64_t np, DevScalars* sc, int set_d0, hipStream_t s);

// Fixed-point weights and per-tile inclusive prefix (uint64).
hipError_t launch_weights_scan(const double* d, const int32_t* sel_block,
                               const uint8_t* excluded, int64_t m,
                               const DevScalars* sc, uint64_t* cdf_local,
                               uint64_t* tile_sum, int32_t* tile_pos,
                               hipStream_t s);
int64_t scan_num_tiles(int64_t m);

// One workgroup: draws the block (rejection, removal fallback, or all rows
// with positive weight) and writes idx[0..nt), sc->nt, sc->npos.
hipError_t launch_sample(const uint64_t* cdf_local, const uint64_t* tile_sum,
                         const int32_t* tile_pos, int64_t m, int32_t b,
                         uint64_t seed, uint64_t t, uint64_t ident,
                         int64_t* idx, DevScalars* sc, hipStream_t s);

// Greedy top-b selection (Remark 4.3): idx[0..n) the rows outside S with the
// largest positive d (ties to the lower row), n = min(b, such rows), in
// sc->nt and sc->npos.  scratch holds topb_scratch_words(m, b) words (none
// for m <= 2048).
int64_t topb_scratch_words(int64_t m, int32_t b);
hipError_t launch_topb(const double* d, const int32_t* sel_block, int64_t m,
                       int32_t b, int64_t* idx, DevScalars* sc, uint64_t* scratch,
                       int64_t scratch_words, hipStream_t s);

// Vt[j,:] = X[idx[j], :] (FP64, zero beyond sc->nt and beyond n),
// xs2[j] = ||X[idx[j],:]||^2.
hipError_t launch_gather_rows(const void* X, rbrp_dtype dt, int64_t n, int64_t ldx,
                              const int64_t* idx, const DevScalars* sc, int32_t bmax,
                              double* Vt, int64_t ldv, double* xs2, hipStream_t s);

// FP64 MFMA GEMM: C = alpha op(A) op(B) + beta C, all row-major.
// A may be FP32 (a_f32).  Dimensions M, N may be overridden by device ints
// (m_dev / n_dev, used when a size is only known on the device); the launch
// covers the host bounds M, N.
hipError_t launch_gemm_f64(int transA, int transB, int64_t M, int64_t N,
                           int64_t K, double alpha, const void* A, int a_f32,
                           int64_t lda, const double* B, int64_t ldb,
                           double beta, double* C, int64_t ldc,
                           const int32_t* m_dev, const int32_t* n_dev,
                           int b_lower_tri, hipStream_t s);

// W L_1 = L_2 by blocked substitution, in place in W (m x K, ldw): the
// diagonal blocks are read from L (FP32 when l_f32) unless L is null (then W
// holds L_2); Bt holds D_J^{-1} on the 64 x 64 diagonal blocks and
// -L_1(I, J) D_J^{-1} below them (K x K, ld K).
hipError_t launch_trsm_tall(int64_t M, int64_t K, const void* L, int l_f32, int64_t ldl,
                            const double* Bt, double* W, int64_t ldw, hipStream_t s);
// A further refinement step of an existing W (W += F, F L_1 = L_2 - W L_1),
// in one pass per 128-row strip.  Tws: round_up(M, 128) x 64 doubles of
// scratch; L1 the lower-triangular K x K factor (ld K), Bt with D_J^{-1} on
// its diagonal blocks (ld K).
hipError_t launch_trsm_refine_step(int64_t M, int64_t K, const void* L, int l_f32,
                                   int64_t ldl, const double* L1, const double* Bt, double* W,
                                   int64_t ldw, double* Tws, hipStream_t s);
// C = Cin - A B (A: M x K FP64; B: K x N; Cin FP32 or FP64), tall A.
// a_vec: the rows of A extend to whole 8-column K steps (vector loads).
hipError_t launch_gemm_tall(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                            bool a_vec, const double* B, int64_t ldb, const void* Cin,
                            int cin_f32, int64_t ldcin, double* C, int64_t ldc, hipStream_t s);
// Pivoted Cholesky of the filter (one workgroup of 256 threads, nb <= kMaxB):
// pivots, b' by the truncation rule, pivot rows Rraw (unpermuted columns),
// R11 in pivoted order (Rp, zero-padded to nb), tail_1 = ||V||_F^2 and the
// rank-guard flag.  G is overwritten when nb > 128.  For nb <= 128, G may
// come as nsl K slices of partial sums gstride apart (added in slice order).
hipError_t launch_cpqr_piv(double* G, int64_t ldg, int32_t nb, const int32_t* nb_dev,
                           double tau_b, const double* xs2_rows, int32_t* piv, double* Rraw,
                           int64_t ldr, double* Rp, int64_t ldp, int32_t* bprime_out,
                           double* tail1_out, int32_t* stop_out, hipStream_t s, int nsl = 1,
                           int64_t gstride = 0);

// X = R^{-1} (or X^T with trans) of the upper triangular R (*bcount x
// *bcount), zero elsewhere in the nb_host x nb_host output; skipped when
// run_flag is given and *run_flag == 0.
hipError_t launch_tri_inv(const double* R, int64_t ldr, const int32_t* bcount, int32_t nb_host,
                          double* X, int64_t ldx, int trans, const int32_t* run_flag,
                          hipStream_t s);
// Inverses of the nbs x nbs diagonal blocks of the lower-triangular n x n
// matrix L (the last block may be smaller), written to the same positions of
// X (the rest of X untouched).
hipError_t launch_lower_diag_inv(const double* L, int64_t ldl, int64_t n, int32_t nbs, double* X,
                                 int64_t ldx, hipStream_t s);

// Qt = (R11^{-1})^T V(:, piv)^T: the orthonormal basis rows of the kept
// columns, p < b'; rows b'..nb_host-1 zero.  Rinv_ws: nb_host^2 doubles.
hipError_t launch_qsolve(const double* Vt, int64_t ldv, const int32_t* piv, const double* Rp,
                         int64_t ldp, const int32_t* bprime, int32_t nb_host, int64_t ncols,
                         double* Qt, int64_t ldq, double* Rinv_ws, hipStream_t s);

// Exact Cholesky-QR factor of G2 (overwritten when nb_host > 128) when
// *need_exact: R2 by Cholesky in natural order (steps done to *steps_out),
// M2t = R2^{-1}; otherwise only *steps_out = *bprime.
hipError_t launch_ortho_exact(double* G2, int64_t ldg, const int32_t* bprime, int32_t nb_host,
                              int32_t* piv2, double* R2raw, double* R2, double* M2,
                              int64_t ldm, int32_t* steps_out, const int32_t* need_exact,
                              hipStream_t s);

// First-order Cholesky-QR factor of G2 = I + E, stored transposed
// (M2t = R2^{-1}), when max|E| <= 1e-8 (need_exact = 0), else need_exact = 1
// and M2t is left to the exact path.  The new basis rows are then
// Qn = M2t^T Qtmp.
hipError_t launch_ortho_first_order(const double* G2, int64_t ldg, const int32_t* bprime,
                                    int32_t nb_host, double* M2, int64_t ldm,
                                    int32_t* need_exact, hipStream_t s);

// C = alpha A B^T + beta C for small M, N and long K (split over waves).
// C[M x N] = alpha A^T B + beta C with A stored K x M and B K x N (small M).
// B's row k is B[brow[k]] when brow is given; K <= *k_dev when k_dev is given.
hipError_t launch_gemm_tn_small(int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, hipStream_t s,
                                const int32_t* brow = nullptr, const int32_t* k_dev = nullptr,
                                int nsl = 1, int64_t astride = 0);
// Products with few 16 x 16 output tiles may split K into slices
// (nt_slice_count); with nsl > 1 (beta = 0) slice z is written to
// C + z cstride and the consumer (launch_gemm_tn_small with the same nsl)
// adds the slices in order.
int nt_slice_count(int64_t M, int64_t N, int64_t K);
hipError_t launch_gemm_nt_small(int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, const int32_t* m_dev,
                                const int32_t* n_dev, hipStream_t s, int nsl = 1,
                                int64_t cstride = 0);

// Skeleton bookkeeping after the filter: S[kS + p] = idx[piv[p]],
// sel_block[S[kS+p]] = t; bchunk (optional) = b' split into deflation
// launches of at most kDeflateMaxB columns.
hipError_t launch_append(const int64_t* idx, const int32_t* piv,
                         const int32_t* bprime, int64_t kS, int32_t t,
                         int64_t* S, int32_t* sel_block, int32_t* bchunk, hipStream_t s);

// Low-precision MFMA fragment copies of Q' (rows kS.. kS+b' of Qt).
hipError_t launch_make_frags(const double* Qt_new, int64_t ldq,
                             const int32_t* bprime, int64_t n_pad, int bmax,
                             int mode, void* fragB1, void* fragA2,
                             hipStream_t s);

// Fused deflation of one block (the hot kernel):
// P = R Q', L[:, kS:kS+b'] = P (rows of earlier skeletons zeroed),
// R <- R - P Q'^T, d_i = ||R_i||^2 (0 on skeletons), partial sums / maxima.
// R16: the BF16 residual (mr x ldr, permuted 32-column groups) that modes
// kModeBF16W write and kModeBF16R read and write; may be NULL otherwise.
// bprime2 (with fragB1b, fragA2b): the second half of a block wider than
// kDeflateMaxB columns (its count, possibly 0, on the device), deflated in
// the same launch on the residual still in registers; only where
// deflate_fuses_halves says so, otherwise NULL and one launch per half.
hipError_t launch_deflate(int mode, void* R, void* R16, int64_t mr, int64_t ldr,
                          int64_t m, const void* fragB1, const void* fragA2,
                          const int32_t* bprime, int bmax, const void* fragB1b,
                          const void* fragA2b, const int32_t* bprime2, void* L,
                          int64_t ldl, int64_t kS, const int32_t* sel_block,
                          int32_t t, double* d, double* part_sum,
                          double* part_max, hipStream_t s);
int64_t deflate_num_partials(int64_t mr);
// BF16 residual back to the FP32 residual (natural column order).
hipError_t launch_r16_to_r32(const void* R16, void* R, int64_t mr, int64_t ldr,
                             hipStream_t s);
int deflate_supported(int mode, int64_t ldr, int bmax);
// whether one launch deflates both halves of a block wider than
// kDeflateMaxB columns in this mode (the one-BF16-product modes)
bool deflate_fuses_halves(int mode);
int deflate_rows_per_wg(int mode, int64_t ldr);
int64_t deflate_pad_cols(int64_t n);
size_t frag_bytes(int mode, int64_t ldr, int bmax);

// Interpolation matrix (Alg. 3): W(rest,:) = L_2 L_1^{-1}, W(S,:) = I.
hipError_t launch_interp(const void* L, int l_f64, int64_t ldl, int64_t m,
                         int64_t k, const int64_t* S, double* W, int64_t ldw,
                         int refine, double* ws, hipStream_t s);
size_t interp_workspace_doubles(int64_t m, int64_t k, int refine);
// W(S,:) = I (exact identity rows of the skeletons).
hipError_t launch_identity_rows(const int64_t* S, int64_t k, double* W, int64_t ldw,
                                hipStream_t s);
// Interpolation matrix through the truncated-SVD pseudo-inverse of L_1
// (Remark 5.2): singular values below clip * sigma_max dropped; kept_host
// (host, written when the stream reaches it) the number kept.  Synchronises
// the stream once per Jacobi sweep.
hipError_t launch_interp_pinv(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t k,
                              const int64_t* S, double* W, int64_t ldw, double clip,
                              double* ws, int32_t* kept_host, hipStream_t s);
size_t pinv_workspace_doubles(int64_t k);

// Sketchy pivoting (LU with partial pivoting on Y = X Omega) and the
// oversampled sketchy interpolation matrix (k_sketchy.hip).
size_t sketchy_workspace_bytes(int64_t m, int64_t k, int64_t l);
hipError_t launch_sketchy(const void* X, int x_f32, int64_t m, int64_t n, int64_t ldx,
                          int64_t k, int64_t l, const double* Omega, int64_t ldo, int64_t* S,
                          double* W, int64_t ldw, void* ws, hipStream_t s);

// Deflation arithmetic modes.
// Deflation modes: the products' arithmetic and, for BF16 products, the
// residual's storage (W: FP32 in, BF16 out; R: BF16 in and out).
enum DeflateMode {
  kModeF64 = 0, kModeF32 = 1, kModeBF16x3 = 2, kModeBF16 = 3, kModeBF16W = 4, kModeBF16R = 5
};
inline bool is_bf16_mode(int mode) { return mode >= kModeBF16x3 && mode <= kModeBF16R; }
inline bool mode_stores_bf16(int mode) { return mode == kModeBF16W || mode == kModeBF16R; }
inline bool mode_reads_bf16(int mode) { return mode == kModeBF16R; }

// ---- batched form (k_batched.hip) ----
bool batch_shape_ok(const rbrp_batch_shape* sh);
size_t batch_workspace_size(rbrp_dtype dt, const rbrp_batch_shape* sh);
// persistent workgroups when the shape gives num_wg = 0
int32_t batch_default_wg();
// largest number of persistent workgroups whose workspace fits in ``bytes``
// (0 if not even one)
int64_t batch_max_wg(rbrp_dtype dt, const rbrp_batch_shape* sh, size_t bytes);
size_t batch_lds_needed(rbrp_dtype dt, const rbrp_batch_shape* sh);
hipError_t launch_batched(const rbrp_batch_desc* descs, const int32_t* order, int32_t count,
                          rbrp_dtype dt, double eps, uint64_t seed, const rbrp_options& o,
                          const rbrp_batch_shape& sh, int32_t* k_out, int32_t* status_out,
                          double* resid_out, void* workspace, hipStream_t s);

}  // namespace rbrp
