// FP64 MFMA GEMM for the FP64 parts of the path: the projection of the
// sampled rows against the basis (Alg. 2, V <- X(S_t,:)^T - Q (Q^T X(S_t,:)^T)),
// the Gram matrices of the block filter and of the reorthogonalisation, and
// the products of the interpolation-matrix solve (Alg. 3).
//
// C = alpha op(A) op(B) + beta C, row-major, 64x64 output tile per workgroup,
// K staged through double-buffered LDS 32 at a time.  Four waves each own a 32x32 quarter as
// 2x2 tiles of v_mfma_f64_16x16x4f64.  Lane layout of that instruction
// (measured on gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives D[l/16 + 4q][l%16] for q = 0..3.
#include "rbrp_internal.h"

namespace rbrp {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 32;

// Double-buffered LDS tiles: the next K tile is fetched into registers while
// the MFMAs of the current one run, then written to the other LDS buffer.
template <typename TA, bool TRA, bool TRB, typename TC>
__global__ __launch_bounds__(256) void k_gemm_f64(
    int64_t M, int64_t N, int64_t K, double alpha, const TA* __restrict__ A,
    int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
    double* __restrict__ C, int64_t ldc, const TC* __restrict__ Cin, int64_t ldcin,
    const int32_t* m_dev, const int32_t* n_dev, int b_lower_tri) {
  __shared__ double As[2][GB_K][GB_M + 2];
  __shared__ double Bs[2][GB_K][GB_N + 2];
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

  // register staging: 8 elements of A and 8 of B per thread and K tile
  double ra[8], rb[8];
  auto fetch = [&](int64_t k0) {
    if (!TRA) {  // A[i][k]: thread -> row ii, 8 consecutive k
      const int ii = tid >> 2, kk = (tid & 3) * 8;
      const int64_t gi = i0 + ii;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t gk = k0 + kk + q;
        ra[q] = (gi < M && gk < K) ? (double)A[gi * lda + gk] : 0.0;
      }
    } else {     // A[k][i]: thread -> k row kk, 8 consecutive i
      const int kk = tid >> 3, ii = (tid & 7) * 8;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t gi = i0 + ii + q;
        ra[q] = (gi < M && gk < K) ? (double)A[gk * lda + gi] : 0.0;
      }
    }
    if (!TRB) {  // B[k][j]
      const int kk = tid >> 3, jj = (tid & 7) * 8;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t gj = j0 + jj + q;
        rb[q] = (gj < N && gk < K) ? B[gk * ldb + gj] : 0.0;
      }
    } else {     // B[j][k]
      const int jj = tid >> 2, kk = (tid & 3) * 8;
      const int64_t gj = j0 + jj;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t gk = k0 + kk + q;
        rb[q] = (gj < N && gk < K) ? B[gj * ldb + gk] : 0.0;
      }
    }
  };
  auto stash = [&](int buf) {
    if (!TRA) {
      const int ii = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) As[buf][kk + q][ii] = ra[q];
    } else {
      const int kk = tid >> 3, ii = (tid & 7) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) As[buf][kk][ii + q] = ra[q];
    }
    if (!TRB) {
      const int kk = tid >> 3, jj = (tid & 7) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[buf][kk][jj + q] = rb[q];
    } else {
      const int jj = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[buf][kk + q][jj] = rb[q];
    }
  };

  int64_t kbeg = 0;
  if (b_lower_tri) kbeg = (j0 / GB_K) * GB_K;  // B[k][j] = 0 for k < j
  if (kbeg < K) {
    fetch(kbeg);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < K; k0 += GB_K) {
      const bool more = k0 + GB_K < K;
      if (more) fetch(k0 + GB_K);
#pragma unroll
      for (int ks = 0; ks < GB_K / 4; ++ks) {
        const int kr = 4 * ks + (lane >> 4);
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[buf][kr][32 * wy + 16 * a + (lane & 15)];
#pragma unroll
        for (int c = 0; c < 2; ++c) bv[c] = Bs[buf][kr][32 * wx + 16 * c + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
      }
      if (more) {
        stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }
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
          if (beta != 0.0) {
            if (Cin) v += beta * (double)Cin[gi * ldcin + gj];
            else v += beta * C[gi * ldc + gj];
          }
          C[gi * ldc + gj] = v;
        }
      }
}

template <typename TA, typename TC>
static void dispatch(int ta, int tb, dim3 g, hipStream_t s, int64_t M, int64_t N,
                     int64_t K, double alpha, const TA* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, double* C,
                     int64_t ldc, const TC* Cin, int64_t ldcin, const int32_t* m_dev,
                     const int32_t* n_dev, int blt) {
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, false, false, TC>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, Cin, ldcin, m_dev, n_dev, blt);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, false, true, TC>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, Cin, ldcin, m_dev, n_dev, blt);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<TA, true, false, TC>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, Cin, ldcin, m_dev, n_dev, blt);
  else
    hipLaunchKernelGGL((k_gemm_f64<TA, true, true, TC>), g, dim3(256), 0, s, M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, Cin, ldcin, m_dev, n_dev, blt);
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
    dispatch<float, double>(transA, transB, g, s, M, N, K, alpha, (const float*)A, lda, B,
                            ldb, beta, C, ldc, nullptr, 0, m_dev, n_dev, b_lower_tri);
  else
    dispatch<double, double>(transA, transB, g, s, M, N, K, alpha, (const double*)A, lda,
                             B, ldb, beta, C, ldc, nullptr, 0, m_dev, n_dev, b_lower_tri);
  return hipGetLastError();
}

// C = alpha A B + beta Cin with A FP64 (no transposes) and Cin of FP32 or
// FP64 (its own leading dimension): the residual L - W L_1 of the W
// refinement, read straight from the FP32 factor.
hipError_t launch_gemm_f64_cin(int64_t M, int64_t N, int64_t K, double alpha,
                               const double* A, int64_t lda, const double* B, int64_t ldb,
                               double beta, const void* Cin, int cin_f32, int64_t ldcin,
                               double* C, int64_t ldc, int b_lower_tri, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)ceil_div(N, GB_N), (unsigned)ceil_div(M, GB_M));
  if (cin_f32)
    dispatch<double, float>(0, 0, g, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                            (const float*)Cin, ldcin, nullptr, nullptr, b_lower_tri);
  else
    dispatch<double, double>(0, 0, g, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                             (const double*)Cin, ldcin, nullptr, nullptr, b_lower_tri);
  return hipGetLastError();
}

}  // namespace rbrp

namespace rbrp {

// C[M x N] = alpha A[M x K] B[N x K]^T + beta C for small M, N and long K
// (the projections Q^T V and the Gram matrices of the block filter).  One
// workgroup per 16 x 16 output tile; its four waves take interleaved 16-wide
// K chunks straight from global memory into MFMA operands (no LDS staging,
// no barriers in the K loop), and the four partial tiles are summed in LDS in
// wave order.  Within a chunk, lane l loads the 4 consecutive k of row l%16
// starting at 4(l/16); MFMA s then uses k = 4(l/16) + s as its K index for
// both operands, which is a permutation of the chunk's K range.
__global__ __launch_bounds__(256) void k_gemm_nt16(int64_t M, int64_t N, int64_t K,
                                                   double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ B,
                                                   int64_t ldb, double beta,
                                                   double* __restrict__ C, int64_t ldc,
                                                   const int32_t* m_dev,
                                                   const int32_t* n_dev) {
  __shared__ double part[4][256];
  if (m_dev) M = min(M, (int64_t)*m_dev);
  if (n_dev) N = min(N, (int64_t)*n_dev);
  const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16;
  if (i0 >= M || j0 >= N) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ia = i0 + (lane & 15), jb = j0 + (lane & 15);
  const bool va = ia < M, vb = jb < N;
  const double* ap = A + (va ? ia : 0) * lda;
  const double* bp = B + (vb ? jb : 0) * ldb;
  d4v acc = (d4v){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t k0 = 16 * w; k0 < K; k0 += 64) {
    const int64_t kk = k0 + 4 * (lane >> 4);
    double a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool kin = kk + s < K;
      a[s] = (va && kin) ? ap[kk + s] : 0.0;
      b[s] = (vb && kin) ? bp[kk + s] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[w][lane * 4 + q] = acc[q];
  __syncthreads();
  const int t = threadIdx.x;
  const double s = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
  const int ln = t >> 2, q = t & 3;
  const int64_t row = i0 + (ln >> 4) + 4 * q, col = j0 + (ln & 15);
  if (row < M && col < N) {
    double v = alpha * s;
    if (beta != 0.0) v += beta * C[row * ldc + col];
    C[row * ldc + col] = v;
  }
}

hipError_t launch_gemm_nt_small(int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, const int32_t* m_dev,
                                const int32_t* n_dev, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)ceil_div(N, 16), (unsigned)ceil_div(M, 16));
  hipLaunchKernelGGL(k_gemm_nt16, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta,
                     C, ldc, m_dev, n_dev);
  return hipGetLastError();
}

}  // namespace rbrp
