// Interpolation matrix from the Cholesky-like factor L (Algorithm 3,
// Prop. 5.1): with L_1 = L(S,:) (k x k, lower triangular because the rows of
// earlier skeletons are zero in later blocks of L), W(S,:) = I and
// W(rest,:) = L_2 L_1^{-1}, which equals X X_S^+ (eq. stable_id).
//
// All in FP64, by substitution as in Alg. 3:
//   1. L_1 gathered from the rows S of L (strict upper part set to zero);
//   2. the 64 x 64 diagonal blocks D_J of L_1 inverted (one workgroup each,
//      by 16 x 16 blocks on FP64 MFMA) and the sub-diagonal blocks scaled,
//      Bt(I, J) = -L_1(I, J) D_J^{-1} (one small MFMA GEMM per block column);
//   3. W L_1 = L solved in place in W by blocked substitution over the block
//      columns, from the last to the first (MFMA tile loops per 128-row
//      strip), with the first refinement step (the residual E = L - W L_1,
//      F L_1 = E, W += F) taken block by block in the same pass; further
//      steps are one more pass each;
//   4. W(S(j),:) = e_j exactly.
#include "rbrp_internal.h"

#include <algorithm>

namespace rbrp {

constexpr int kDiag = 64;
constexpr int64_t kSuper = 256;   // columns of a super-block of the W solve

template <typename TL>
__global__ __launch_bounds__(256) void k_gather_l1(const TL* __restrict__ L, int64_t ldl,
                                                   const int64_t* __restrict__ S,
                                                   int64_t k, double* __restrict__ L1) {
  const int64_t j = blockIdx.x;
  const int64_t row = S[j];
  for (int64_t p = threadIdx.x; p < k; p += 256)
    L1[j * k + p] = (p <= j) ? (double)L[row * ldl + p] : 0.0;
}

__global__ __launch_bounds__(256) void k_identity_rows(const int64_t* __restrict__ S,
                                                       int64_t k, double* __restrict__ W,
                                                       int64_t ldw) {
  const int64_t j = blockIdx.x;
  const int64_t row = S[j];
  for (int64_t p = threadIdx.x; p < k; p += 256) W[row * ldw + p] = (p == j) ? 1.0 : 0.0;
}

hipError_t launch_identity_rows(const int64_t* S, int64_t k, double* W, int64_t ldw,
                                hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_rows, dim3((unsigned)k), dim3(256), 0, s, S, k, W, ldw);
  return hipGetLastError();
}

size_t interp_workspace_doubles(int64_t m, int64_t k, int refine) {
  // L1 and Bt (k x k each); with refinement a 64-column scratch per row
  return (size_t)(2 * k * k + (refine > 0 ? round_up(m, 128) * 64 : 0));
}

hipError_t launch_interp(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t k,
                         const int64_t* S, double* W, int64_t ldw, int refine,
                         double* ws, hipStream_t s) {
  if (k <= 0 || m <= 0) return hipSuccess;
  double* L1 = ws;
  double* Bt = L1 + k * k;
  double* Tws = Bt + k * k;
  hipError_t e;
  if (l_f64)
    hipLaunchKernelGGL(k_gather_l1<double>, dim3((unsigned)k), dim3(256), 0, s,
                       (const double*)L, ldl, S, k, L1);
  else
    hipLaunchKernelGGL(k_gather_l1<float>, dim3((unsigned)k), dim3(256), 0, s,
                       (const float*)L, ldl, S, k, L1);
  const int64_t nblk = ceil_div(k, kDiag);
  e = launch_lower_diag_inv(L1, k, k, kDiag, Bt, k, s);
  if (e != hipSuccess) return e;
  const int lf32 = l_f64 ? 0 : 1;
  if (refine <= 0) {
    // Bt(I, J) = -L_1(I, J) D_J^{-1} for the block rows I > J
    for (int64_t J = 0; J + 1 < nblk; ++J) {
      const int64_t j0 = J * kDiag, j1 = j0 + kDiag;
      e = launch_gemm_f64(0, 0, k - j1, kDiag, kDiag, -1.0, L1 + j1 * k + j0, 0, k,
                          Bt + j0 * k + j0, k, 0.0, Bt + j1 * k + j0, k, nullptr, nullptr, 0, s);
      if (e != hipSuccess) return e;
    }
    e = launch_trsm_tall(m, k, L, lf32, ldl, Bt, W, ldw, s);
  } else {
    // Substitution with the first refinement step in the same pass, by
    // super-blocks of kSuper columns from the last to the first: the later
    // super-blocks' contribution to a super-block's right sides is one tall
    // GEMM into W's own columns, R_s = L_2(:, s) - W(:, >s) L_1(>s, s), and
    // the super-block is then solved strip by strip from R_s as before.
    // Each strip re-reads its finished 64-column blocks only within its
    // super-block, instead of across all of W.  Further refinement steps
    // run on the whole result.
    const bool a_vec = ldw >= round_up(k, (int64_t)8);
    for (int64_t a = (ceil_div(k, kSuper) - 1) * kSuper; a >= 0 && e == hipSuccess; a -= kSuper) {
      const int64_t nbk = std::min<int64_t>(kSuper, k - a);
      if (a + nbk < k) {
        e = launch_gemm_tall(m, nbk, k - a - nbk, W + a + nbk, ldw, a_vec, L1 + (a + nbk) * k + a,
                             k, l_f64 ? (const void*)((const double*)L + a)
                                      : (const void*)((const float*)L + a),
                             lf32, ldl, W + a, ldw, s);
        if (e != hipSuccess) return e;
        e = launch_trsm_refine(m, nbk, W + a, 0, ldw, L1 + a * k + a, Bt + a * k + a, k, W + a,
                               ldw, a, Tws, 0, s);
      } else {
        e = launch_trsm_refine(m, nbk, l_f64 ? (const void*)((const double*)L + a)
                                             : (const void*)((const float*)L + a),
                               lf32, ldl, L1 + a * k + a, Bt + a * k + a, k, W + a, ldw, a, Tws,
                               0, s);
      }
    }
    for (int it = 1; it < refine && e == hipSuccess; ++it)
      e = launch_trsm_refine(m, k, L, lf32, ldl, L1, Bt, k, W, ldw, 0, Tws, 1, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_identity_rows, dim3((unsigned)k), dim3(256), 0, s, S, k, W, ldw);
  return hipGetLastError();
}

}  // namespace rbrp
