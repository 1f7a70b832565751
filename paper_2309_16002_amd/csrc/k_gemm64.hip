// FP64 MFMA GEMM for the FP64 parts of the path: the projection of the
// sampled rows against the basis (Alg. 2, V <- X(S_t,:)^T - Q (Q^T X(S_t,:)^T)),
// the Gram matrices of the block filter and of the reorthogonalisation, and
// the products of the interpolation-matrix solve (Alg. 3).
//
// C = alpha op(A) op(B) + beta C, row-major, 64x64 output tile per workgroup,
// K staged through LDS 16 at a time.  Four waves each own a 32x32 quarter as
// 2x2 tiles of v_mfma_f64_16x16x4f64.  Lane layout of that instruction
// (measured on gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives D[l/16 + 4q][l%16] for q = 0..3.
#include "rbrp_internal.h"

namespace rbrp {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

template <typename TA, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_gemm_f64(
    int64_t M, int64_t N, int64_t K, double alpha, const TA* __restrict__ A,
    int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
    double* __restrict__ C, int64_t ldc, const int32_t* m_dev,
    const int32_t* n_dev, int b_lower_tri) {
  __shared__ double As[GB_K][GB_M + 2];
  __shared__ double Bs[GB_K][GB_N + 2];
  if (m_dev) M = min(M, (int64_t)*m_dev);
  if (n_dev) N = min(N, (int64_t)*n_dev);
  const int64_t i0 = (int64_t)blockIdx.y * GB_M;
  const int64_t j0 = (int64_t)blockIdx.x * GB_N;
  if (i0 >= M || j0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wy = w >> 1, wx = w & 1;
  d4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = (d4v){0.0, 0.0, 0.0, 0.0};

  int64_t kbeg = 0;
  if (b_lower_tri) kbeg = (j0 / GB_K) * GB_K;  // B[k][j] = 0 for k < j
  for (int64_t k0 = kbeg; k0 < K; k0 += GB_K) {
    // stage A (GB_M x GB_K) as As[k][i]
    if (!TRA) {
      const int ii = tid >> 2, kk = (tid & 3) * 4;
      const int64_t gi = i0 + ii;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gk = k0 + kk + q;
        As[kk + q][ii] = (gi < M && gk < K) ? (double)A[gi * lda + gk] : 0.0;
      }
    } else {
      const int kk = tid >> 4, ii = (tid & 15) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = i0 + ii + q;
        As[kk][ii + q] = (gi < M && gk < K) ? (double)A[gk * lda + gi] : 0.0;
      }
    }
    // stage B (GB_K x GB_N) as Bs[k][j]
    if (!TRB) {
      const int kk = tid >> 4, jj = (tid & 15) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gj = j0 + jj + q;
        Bs[kk][jj + q] = (gj < N && gk < K) ? B[gk * ldb + gj] : 0.0;
      }
    } else {
      const int jj = tid >> 2, kk = (tid & 3) * 4;
      const int64_t gj = j0 + jj;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gk = k0 + kk + q;
        Bs[kk + q][jj] = (gj < N && gk < K) ? B[gj * ldb + gk] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GB_K / 4; ++ks) {
      const int kr = 4 * ks + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kr][32 * wy + 16 * a + (lane & 15)];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = Bs[kr][32 * wx + 16 * c + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = i0 + 32 * wy + 16 * a + (lane >> 4) + 4 * q;
        const int64_t gj = j0 + 32 * wx + 16 * c + (lane & 15);
        if (gi < M && gj < N) {
          double v = alpha * acc[a][c][q];
          if (beta != 0.0) v += beta * C[gi * ldc + gj];
          C[gi * ldc + gj] = v;
        }
      }
}

template <typename TA>
static void dispatch(int ta, int tb, dim3 g, hipStream_t s, int64_t M, int64_t N,
                     int64_t K, double alpha, const TA* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, double* C,
                     int64_t ldc, const int32_t* m_dev, const int32_t* n_dev,
                     int blt) {
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, false, false>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, m_dev, n_dev, blt);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, false, true>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, m_dev, n_dev, blt);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, true, false>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, m_dev, n_dev, blt);
  else
    hipLaunchKernelGGL((k_gemm_f64<TA, true, true>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, m_dev, n_dev, blt);
}

hipError_t launch_gemm_f64(int transA, int transB, int64_t M, int64_t N,
                           int64_t K, double alpha, const void* A, int a_f32,
                           int64_t lda, const double* B, int64_t ldb,
                           double beta, double* C, int64_t ldc,
                           const int32_t* m_dev, const int32_t* n_dev,
                           int b_lower_tri, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)ceil_div(N, GB_N), (unsigned)ceil_div(M, GB_M));
  if (a_f32)
    dispatch<float>(transA, transB, g, s, M, N, K, alpha, (const float*)A, lda, B,
                    ldb, beta, C, ldc, m_dev, n_dev, b_lower_tri);
  else
    dispatch<double>(transA, transB, g, s, M, N, K, alpha, (const double*)A, lda,
                     B, ldb, beta, C, ldc, m_dev, n_dev, b_lower_tri);
  return hipGetLastError();
}

}  // namespace rbrp
