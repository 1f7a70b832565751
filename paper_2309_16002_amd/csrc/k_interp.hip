// Interpolation matrix from the Cholesky-like factor L (Algorithm 3,
// Prop. 5.1): with L_1 = L(S,:) (k x k, lower triangular because the rows of
// earlier skeletons are zero in later blocks of L), W(S,:) = I and
// W(rest,:) = L_2 L_1^{-1}, which equals X X_S^+ (eq. stable_id).
//
// All in FP64:
//   1. L_1 gathered from the rows S of L (strict upper part set to zero);
//   2. L_1^{-1} by blocked forward substitution: the 64 x 64 diagonal blocks
//      are inverted in LDS (one workgroup each), the off-diagonal blocks by
//      two MFMA GEMMs per block row;
//   3. W = L L_1^{-1} (one MFMA GEMM, the triangular factor's zero blocks
//      skipped), then refinement steps W += (L - W L_1) L_1^{-1};
//   4. W(S(j),:) = e_j exactly.
#include "rbrp_internal.h"

namespace rbrp {

constexpr int kDiag = 64;

template <typename TL>
__global__ __launch_bounds__(256) void k_gather_l1(const TL* __restrict__ L, int64_t ldl,
                                                   const int64_t* __restrict__ S,
                                                   int64_t k, double* __restrict__ L1) {
  const int64_t j = blockIdx.x;
  const int64_t row = S[j];
  for (int64_t p = threadIdx.x; p < k; p += 256)
    L1[j * k + p] = (p <= j) ? (double)L[row * ldl + p] : 0.0;
}

// Inverse of each lower-triangular 64x64 diagonal block, column-parallel
// forward substitution in LDS.  Dinv[b] is stored in place of the block
// inside Linv (row-major k x k).
__global__ __launch_bounds__(kDiag) void k_diag_inv(const double* __restrict__ L1,
                                                    int64_t k, double* __restrict__ Linv) {
  __shared__ double A[kDiag][kDiag + 1];
  __shared__ double X[kDiag][kDiag + 1];
  const int64_t b0 = (int64_t)blockIdx.x * kDiag;
  const int nbk = (int)min<int64_t>(kDiag, k - b0);
  const int j = threadIdx.x;
  for (int i = 0; i < kDiag; ++i)
    A[i][j] = (i < nbk && j < nbk) ? L1[(b0 + i) * k + b0 + j] : (i == j ? 1.0 : 0.0);
  __syncthreads();
  // column j of the inverse: x_i = (delta_ij - sum_{p<i} A[i][p] x_p) / A[i][i];
  // four partial sums break the FMA dependency chain
  for (int i = 0; i < kDiag; ++i) {
    double v = 0.0;
    if (i >= j) {
      double s0 = (i == j) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int p = j;
      for (; p + 3 < i; p += 4) {
        s0 -= A[i][p] * X[p][j];
        s1 -= A[i][p + 1] * X[p + 1][j];
        s2 -= A[i][p + 2] * X[p + 2][j];
        s3 -= A[i][p + 3] * X[p + 3][j];
      }
      for (; p < i; ++p) s0 -= A[i][p] * X[p][j];
      v = ((s0 + s1) + (s2 + s3)) / A[i][i];
    }
    X[i][j] = v;
  }
  __syncthreads();
  for (int i = 0; i < nbk; ++i)
    if (j < nbk) Linv[(b0 + i) * k + b0 + j] = X[i][j];
}

__global__ __launch_bounds__(256) void k_identity_rows(const int64_t* __restrict__ S,
                                                       int64_t k, double* __restrict__ W,
                                                       int64_t ldw) {
  const int64_t j = blockIdx.x;
  const int64_t row = S[j];
  for (int64_t p = threadIdx.x; p < k; p += 256) W[row * ldw + p] = (p == j) ? 1.0 : 0.0;
}

__global__ void k_zero(double* __restrict__ x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) x[e] = 0.0;
}

// Leading dimension of the m x k FP64 intermediates: rows 16-byte aligned
// and padded to whole K steps of the tall GEMM.
static int64_t interp_ld(int64_t k) { return round_up(k, 16); }

size_t interp_workspace_doubles(int64_t m, int64_t k) {
  // L1, L1inv, T (kDiag x k), W0 and E (m x interp_ld(k) each)
  return (size_t)(2 * k * k + kDiag * k + 2 * m * interp_ld(k));
}

hipError_t launch_interp(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t k,
                         const int64_t* S, double* W, int64_t ldw, int refine,
                         double* ws, hipStream_t s) {
  if (k <= 0 || m <= 0) return hipSuccess;
  double* L1 = ws;
  double* Linv = L1 + k * k;
  double* T = Linv + k * k;
  const int64_t lde = interp_ld(k);
  double* W0 = T + kDiag * k;
  double* E = W0 + m * lde;
  hipError_t e;
  if (l_f64)
    hipLaunchKernelGGL(k_gather_l1<double>, dim3((unsigned)k), dim3(256), 0, s,
                       (const double*)L, ldl, S, k, L1);
  else
    hipLaunchKernelGGL(k_gather_l1<float>, dim3((unsigned)k), dim3(256), 0, s,
                       (const float*)L, ldl, S, k, L1);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div(k * k, 256)), dim3(256), 0, s, Linv,
                     k * k);
  const int64_t nblk = ceil_div(k, kDiag);
  hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)nblk), dim3(kDiag), 0, s, L1, k, Linv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // block row I: Linv[I, 0:I0] = -Dinv_I (L1[I, 0:I0] Linv[0:I0, 0:I0])
  for (int64_t I = 1; I < nblk; ++I) {
    const int64_t i0 = I * kDiag;
    const int64_t ni = (k - i0 < kDiag) ? (k - i0) : kDiag;
    e = launch_gemm_f64(0, 0, ni, i0, i0, 1.0, L1 + i0 * k, 0, k, Linv, k, 0.0, T, k,
                        nullptr, nullptr, 1, s);
    if (e != hipSuccess) return e;
    e = launch_gemm_f64(0, 0, ni, i0, ni, -1.0, Linv + i0 * k + i0, 0, k, T, k, 0.0,
                        Linv + i0 * k, k, nullptr, nullptr, 0, s);
    if (e != hipSuccess) return e;
  }
  // W = L Linv, refined as W += (L - W L1) Linv.  The iterate lives in W0
  // (padded rows, so it can be the A operand of the next product) and only
  // the last step writes the caller's W.
  const int lf32 = l_f64 ? 0 : 1;
  e = launch_gemm_tall(m, k, k, 1.0, L, lf32, ldl, Linv, k, 0.0, nullptr, 0, 0,
                       refine > 0 ? W0 : W, refine > 0 ? lde : ldw, 1, s);
  if (e != hipSuccess) return e;
  for (int it = 0; it < refine; ++it) {
    // E = L - W0 L1 ;  W0 (or W, last step) = W0 + E Linv
    e = launch_gemm_tall(m, k, k, -1.0, W0, 0, lde, L1, k, 1.0, L, lf32, ldl, E, lde, 1, s);
    if (e != hipSuccess) return e;
    const bool last = it + 1 == refine;
    e = launch_gemm_tall(m, k, k, 1.0, E, 0, lde, Linv, k, 1.0, W0, 0, lde, last ? W : W0,
                         last ? ldw : lde, 1, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_identity_rows, dim3((unsigned)k), dim3(256), 0, s, S, k, W, ldw);
  return hipGetLastError();
}

}  // namespace rbrp
