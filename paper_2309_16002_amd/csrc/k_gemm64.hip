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
#include <algorithm>
#include <type_traits>

#include "rbrp_internal.h"

namespace rbrp {

typedef double d2v __attribute__((ext_vector_type(2)));
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

}  // namespace rbrp

namespace rbrp {

// C[M x N] = alpha A[M x K] B[N x K]^T + beta C for small M, N and long K
// (the projections Q^T V and the Gram matrices of the block filter).  One
// workgroup per 16 x 16 output tile and K slice; its NW waves take
// interleaved 16-wide K chunks straight from global memory into MFMA
// operands (no LDS staging, no barriers in the K loop), and the NW partial
// tiles are summed in LDS in wave order.  With several K slices (blockIdx.z,
// kslice long) slice z writes its partial product to C + z cstride (beta =
// 0) and the consumer adds the slices in order: a few output tiles then
// spread their K over more CUs instead of streaming all of K through one.  Within a chunk, lane l loads the 4 consecutive k of row l%16
// starting at 4(l/16); MFMA s then uses k = 4(l/16) + s as its K index for
// both operands, which is a permutation of the chunk's K range.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_nt16(int64_t M, int64_t N, int64_t K,
                                                      double alpha,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double beta, double* __restrict__ C,
                                                      int64_t ldc, const int32_t* m_dev,
                                                      const int32_t* n_dev, int64_t kslice,
                                                      int64_t cstride) {
  __shared__ double part[NW][256];
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
  // groups of four 16-wide chunks per wave: every load of a group is issued
  // before its MFMAs.  Chunk bases past the K slice are clamped to its last
  // chunk (slice bounds are multiples of 16) and their products masked, so
  // no load is conditional.
  const int64_t kbeg = (int64_t)blockIdx.z * kslice;
  const int64_t kend = min(K, kbeg + kslice);
  C += (int64_t)blockIdx.z * cstride;
  const int64_t kstep = 16 * NW;
  const int64_t klast = kend - 16;
  const int koff = 4 * (lane >> 4);
  for (int64_t k0 = kbeg + 16 * w; k0 < kend; k0 += 4 * kstep) {
    d2v a[4][2], b[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kb = min(k0 + u * kstep, klast) + koff;
      a[u][0] = *reinterpret_cast<const d2v*>(ap + kb);
      a[u][1] = *reinterpret_cast<const d2v*>(ap + kb + 2);
      b[u][0] = *reinterpret_cast<const d2v*>(bp + kb);
      b[u][1] = *reinterpret_cast<const d2v*>(bp + kb + 2);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool live = k0 + u * kstep < kend;
      const bool la = live && va, lb = live && vb;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double x = la ? a[u][s >> 1][s & 1] : 0.0;
        const double y = lb ? b[u][s >> 1][s & 1] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[w][lane * 4 + q] = acc[q];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 256) {
    double s = part[0][t];
#pragma unroll
    for (int v = 1; v < NW; ++v) s += part[v][t];
    const int ln = t >> 2, q = t & 3;
    const int64_t row = i0 + (ln >> 4) + 4 * q, col = j0 + (ln & 15);
    if (row < M && col < N) {
      double v = alpha * s;
      if (beta != 0.0) v += beta * C[row * ldc + col];
      C[row * ldc + col] = v;
    }
  }
}

// The same product with 32 x 32 output blocks (four MFMA tiles) per
// workgroup of NW waves: every A or B fragment a wave loads feeds two MFMA
// tiles instead of one, which halves the operand traffic from L2 per flop.
// Used when there are at least 128 such blocks (the projections against a
// basis of a thousand rows and more, where the 16 x 16 form is bound by
// that traffic; splitting their K into slices summed by the consumer was
// measured slower, since the consumer then reads every slice).
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_nt32(int64_t M, int64_t N, int64_t K,
                                                      double alpha,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double beta, double* __restrict__ C,
                                                      int64_t ldc, const int32_t* m_dev,
                                                      const int32_t* n_dev) {
  __shared__ double part[NW][4][256];
  if (m_dev) M = min(M, (int64_t)*m_dev);
  if (n_dev) N = min(N, (int64_t)*n_dev);
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  if (i0 >= M || j0 >= N) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* ap[2];
  const double* bp[2];
  bool va[2], vb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t ia = i0 + 16 * h + (lane & 15), jb = j0 + 16 * h + (lane & 15);
    va[h] = ia < M;
    vb[h] = jb < N;
    ap[h] = A + (va[h] ? ia : 0) * lda;
    bp[h] = B + (vb[h] ? jb : 0) * ldb;
  }
  d4v acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (d4v){0.0, 0.0, 0.0, 0.0};
  // groups of two 16-wide chunks per wave, every load of a group before its
  // MFMAs; chunk bases past K are clamped to the last chunk and masked
  const int64_t kstep = 16 * NW;
  const int64_t klast = K - 16;
  const int koff = 4 * (lane >> 4);
  for (int64_t k0 = 16 * w; k0 < K; k0 += 2 * kstep) {
    d2v a[2][2][2], b[2][2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t kb = min(k0 + u * kstep, klast) + koff;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[u][h][0] = *reinterpret_cast<const d2v*>(ap[h] + kb);
        a[u][h][1] = *reinterpret_cast<const d2v*>(ap[h] + kb + 2);
        b[u][h][0] = *reinterpret_cast<const d2v*>(bp[h] + kb);
        b[u][h][1] = *reinterpret_cast<const d2v*>(bp[h] + kb + 2);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool live = k0 + u * kstep < K;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        double xa[2], yb[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          xa[h] = (live && va[h]) ? a[u][h][st >> 1][st & 1] : 0.0;
          yb[h] = (live && vb[h]) ? b[u][h][st >> 1][st & 1] : 0.0;
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[x], yb[y], acc[x][y], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) part[w][2 * x + y][lane * 4 + q] = acc[x][y][q];
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += 64 * NW) {
    const int t = e >> 8, idx = e & 255;
    double sm = part[0][t][idx];
#pragma unroll
    for (int v = 1; v < NW; ++v) sm += part[v][t][idx];
    const int ln = idx >> 2, q = idx & 3;
    const int64_t row = i0 + 16 * (t >> 1) + (ln >> 4) + 4 * q;
    const int64_t col = j0 + 16 * (t & 1) + (ln & 15);
    if (row < M && col < N) {
      double v = alpha * sm;
      if (beta != 0.0) v += beta * C[row * ldc + col];
      C[row * ldc + col] = v;
    }
  }
}

// Any K (rows of A and B need no padding): per-element loads with the K
// tail masked, four waves.
__global__ __launch_bounds__(256) void k_gemm_nt16_any(int64_t M, int64_t N, int64_t K,
                                                       double alpha,
                                                       const double* __restrict__ A,
                                                       int64_t lda,
                                                       const double* __restrict__ B,
                                                       int64_t ldb, double beta,
                                                       double* __restrict__ C, int64_t ldc) {
  __shared__ double part[4][256];
  const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ia = i0 + (lane & 15), jb = j0 + (lane & 15);
  const bool va = ia < M, vb = jb < N;
  const double* ap = A + (va ? ia : 0) * lda;
  const double* bp = B + (vb ? jb : 0) * ldb;
  d4v acc = (d4v){0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 16 * w; k0 < K; k0 += 64) {
    const int64_t kk = k0 + 4 * (lane >> 4);
    double a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t kc = min(kk + s, K - 1);
      const bool kin = kk + s < K;
      a[s] = ap[kc];
      b[s] = bp[kc];
      a[s] = (va && kin) ? a[s] : 0.0;
      b[s] = (vb && kin) ? b[s] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[w][lane * 4 + q] = acc[q];
  __syncthreads();
  const int t = threadIdx.x;
  const double sm = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
  const int ln = t >> 2, q = t & 3;
  const int64_t row = i0 + (ln >> 4) + 4 * q, col = j0 + (ln & 15);
  if (row < M && col < N) {
    double v = alpha * sm;
    if (beta != 0.0) v += beta * C[row * ldc + col];
    C[row * ldc + col] = v;
  }
}

// K a multiple of 16 (the padded row length) with 16-byte aligned rows: the
// batched-load kernel, sixteen waves splitting K when K >= 512; otherwise the
// per-element kernel.  Partial tiles are summed in wave order (deterministic).
// the 32 x 32 form: at least 128 output blocks and a long aligned K
static bool nt32_shape(int64_t M, int64_t N, int64_t K) {
  return K >= 512 && K % 16 == 0 && M >= 32 && N >= 32 &&
         ceil_div(M, (int64_t)32) * ceil_div(N, (int64_t)32) >= 128;
}

int nt_slice_count(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(N, (int64_t)16) * ceil_div(M, (int64_t)16);
  if (tiles > 64 || K < 256 || K % 16) return 1;
  const int64_t want = std::min<int64_t>(kNtMaxSlices, 256 / tiles);
  const int64_t kslice = round_up(ceil_div(K, want), (int64_t)64);
  return (int)ceil_div(K, kslice);
}

hipError_t launch_gemm_nt_small(int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, const int32_t* m_dev,
                                const int32_t* n_dev, hipStream_t s, int nsl, int64_t cstride) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)ceil_div(N, 16), (unsigned)ceil_div(M, 16));
  if (K < 16 || K % 16 || lda % 2 || ldb % 2 || ((uintptr_t)A | (uintptr_t)B) % 16) {
    if (m_dev || n_dev || nsl > 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_nt16_any, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  } else if (nsl > 1) {
    // the slice count the consumer expects must be the one this launch uses
    if (beta != 0.0 || nsl != nt_slice_count(M, N, K)) return hipErrorInvalidValue;
    const int64_t kslice = round_up(ceil_div(K, (int64_t)nsl), (int64_t)64);
    g.z = (unsigned)nsl;
    hipLaunchKernelGGL(k_gemm_nt16<4>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, m_dev, n_dev, kslice, cstride);
  } else if (nt32_shape(M, N, K)) {
    const dim3 g32((unsigned)ceil_div(N, 32), (unsigned)ceil_div(M, 32));
    hipLaunchKernelGGL(k_gemm_nt32<8>, g32, dim3(512), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, m_dev, n_dev);
  } else if (K >= 512) {
    hipLaunchKernelGGL(k_gemm_nt16<16>, g, dim3(1024), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, m_dev, n_dev, K, (int64_t)0);
  } else {
    hipLaunchKernelGGL(k_gemm_nt16<4>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, m_dev, n_dev, K, (int64_t)0);
  }
  return hipGetLastError();
}


// C[M x N] = alpha A[K x M]^T B[K x N] + beta C for small M and long N
// (the basis projections V <- V - C^T Q of the sampled rows: M = b, K = |S|,
// N = n; and Q' = R11^{-T}-weighted pivoted rows of V, with B's rows taken
// through brow and K bounded on the device by *k_dev).  One workgroup per 16 x 16 output tile; its four waves take
// interleaved 16-deep K chunks straight from global memory (16 consecutive
// elements of a row of A or B per quarter-wave), and the partial tiles are
// summed in LDS in wave order.  MFMA step s of a chunk uses K index
// 4 s + l / 16 for both operands.
template <bool GATHER>
__global__ __launch_bounds__(256) void k_gemm_tn16(int64_t M, int64_t N, int64_t K,
                                                   double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ B,
                                                   int64_t ldb, const int32_t* __restrict__ brow,
                                                   const int32_t* __restrict__ k_dev,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc, int nsl, int64_t astride) {
  __shared__ double part[4][256];
  if (k_dev) K = min(K, (int64_t)*k_dev);
  const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ia = i0 + (lane & 15), jb = j0 + (lane & 15);
  const bool va = ia < M, vb = jb < N;
  const int kq = lane >> 4;
  const int64_t iac = va ? ia : 0, jbc = vb ? jb : 0;
  d4v acc = (d4v){0.0, 0.0, 0.0, 0.0};
  // groups of two 16-deep chunks per wave, every load of a group issued before
  // its MFMAs; k past K is clamped to K - 1 (always a valid row) and masked
  for (int64_t k0 = 16 * w; k0 < K; k0 += 128) {
    double a[8], b[8];
    int64_t kr[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t k = min(k0 + 64 * (s >> 2) + 4 * (s & 3) + kq, K - 1);
      kr[s] = GATHER ? (int64_t)brow[k] : k;
      a[s] = A[k * lda + iac];
    }
    // A given as K slices of partial sums (from the sliced NT product):
    // every slice's loads issued together, then added in slice order
    if (nsl > 1) {
      double az[kNtMaxSlices - 1][8];
#pragma unroll
      for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int64_t k = min(k0 + 64 * (s >> 2) + 4 * (s & 3) + kq, K - 1);
          az[z - 1][s] = A[min(z, nsl - 1) * astride + k * lda + iac];
        }
#pragma unroll
      for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
        for (int s = 0; s < 8; ++s) a[s] += z < nsl ? az[z - 1][s] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) b[s] = B[kr[s] * ldb + jbc];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const bool kin = k0 + 64 * (s >> 2) + 4 * (s & 3) + kq < K;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((va && kin) ? a[s] : 0.0,
                                                 (vb && kin) ? b[s] : 0.0, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[w][lane * 4 + q] = acc[q];
  __syncthreads();
  const int t = threadIdx.x;
  const double sm = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
  const int ln = t >> 2, q = t & 3;
  const int64_t row = i0 + (ln >> 4) + 4 * q, col = j0 + (ln & 15);
  if (row < M && col < N) {
    double v = alpha * sm;
    if (beta != 0.0) v += beta * C[row * ldc + col];
    C[row * ldc + col] = v;
  }
}

// The same product with 32 x 32 output blocks (four MFMA tiles) per
// workgroup: each loaded element of A or B feeds two MFMA tiles.  Used for
// the basis projections when there are at least 128 such blocks.
__global__ __launch_bounds__(256) void k_gemm_tn32(int64_t M, int64_t N, int64_t K,
                                                   double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ B,
                                                   int64_t ldb, double beta,
                                                   double* __restrict__ C, int64_t ldc, int nsl,
                                                   int64_t astride) {
  __shared__ double part[4][4][256];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = lane >> 4;
  int64_t iac[2], jbc[2];
  bool va[2], vb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t ia = i0 + 16 * h + (lane & 15), jb = j0 + 16 * h + (lane & 15);
    va[h] = ia < M;
    vb[h] = jb < N;
    iac[h] = va[h] ? ia : 0;
    jbc[h] = vb[h] ? jb : 0;
  }
  d4v acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (d4v){0.0, 0.0, 0.0, 0.0};
  // one 16-deep chunk per wave and step (k past K clamped to K - 1 and
  // masked), every load of a step issued before its MFMAs
  for (int64_t k0 = 16 * w; k0 < K; k0 += 64) {
    double a[4][2], b[4][2];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t k = min(k0 + 4 * st + kq, K - 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[st][h] = A[k * lda + iac[h]];
        b[st][h] = B[k * ldb + jbc[h]];
      }
    }
    // A given as K slices of partial sums: added in slice order
    if (nsl > 1) {
      double az[kNtMaxSlices - 1][4][2];
#pragma unroll
      for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int64_t k = min(k0 + 4 * st + kq, K - 1);
#pragma unroll
          for (int h = 0; h < 2; ++h)
            az[z - 1][st][h] = A[min(z, nsl - 1) * astride + k * lda + iac[h]];
        }
#pragma unroll
      for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int h = 0; h < 2; ++h) a[st][h] += z < nsl ? az[z - 1][st][h] : 0.0;
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const bool kin = k0 + 4 * st + kq < K;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64((va[x] && kin) ? a[st][x] : 0.0,
                                                           (vb[y] && kin) ? b[st][y] : 0.0,
                                                           acc[x][y], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) part[w][2 * x + y][lane * 4 + q] = acc[x][y][q];
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int t = e >> 8, idx = e & 255;
    const double sm = ((part[0][t][idx] + part[1][t][idx]) + part[2][t][idx]) + part[3][t][idx];
    const int ln = idx >> 2, q = idx & 3;
    const int64_t row = i0 + 16 * (t >> 1) + (ln >> 4) + 4 * q;
    const int64_t col = j0 + 16 * (t & 1) + (ln & 15);
    if (row < M && col < N) {
      double v = alpha * sm;
      if (beta != 0.0) v += beta * C[row * ldc + col];
      C[row * ldc + col] = v;
    }
  }
}

hipError_t launch_gemm_tn_small(int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, hipStream_t s,
                                const int32_t* brow, const int32_t* k_dev, int nsl,
                                int64_t astride) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (nsl < 1) return hipErrorInvalidValue;
  dim3 g((unsigned)ceil_div(N, 16), (unsigned)ceil_div(M, 16));
  if (!brow && !k_dev && M >= 32 && N >= 32 &&
      ceil_div(M, (int64_t)32) * ceil_div(N, (int64_t)32) >= 128) {
    const dim3 g32((unsigned)ceil_div(N, 32), (unsigned)ceil_div(M, 32));
    hipLaunchKernelGGL(k_gemm_tn32, g32, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta,
                       C, ldc, nsl, astride);
  } else if (brow)
    hipLaunchKernelGGL(k_gemm_tn16<true>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       brow, k_dev, beta, C, ldc, nsl, astride);
  else
    hipLaunchKernelGGL(k_gemm_tn16<false>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                       brow, k_dev, beta, C, ldc, nsl, astride);
  return hipGetLastError();
}

}  // namespace rbrp

namespace rbrp {

// Tiles of C = alpha A B + beta Cin for tall A (M >> N, K): the blocked
// substitution of the interpolation-matrix solve (Alg. 3) and its
// refinement step below.  A is M x K row-major (FP32 factor or FP64), B is
// K x N FP64.
//
// 128 x 64 output tile per workgroup; four waves each own 64 x 32 of it as
// 4 x 2 tiles of v_mfma_f64_16x16x4f64.  K goes through double-buffered LDS
// TB_K at a time with a two-deep register pipeline: while the MFMAs of step
// t run, step t+1 waits in registers and the loads of step t+2 are in
// flight, so short K loops (k of a few hundred) still hide HBM latency.
// The workgroup index is mapped so that all column tiles of one 128-row
// strip run on the same XCD (blocks are dealt to the eight XCDs
// round-robin), which keeps the strip's rows in that XCD's L2.
//
// Vector path (VA): A 16-byte aligned with lda >= round_up(K, TB_K), so every
// step loads whole vectors inside the row; the K positions >= K are zeroed
// when written to LDS.  Otherwise each element is loaded from a clamped
// index.  Rows >= M of A and columns >= N of B only reach outputs that are
// not stored, so they are loaded from clamped addresses and not masked.
constexpr int TB_M = 128;
constexpr int TA_LD = TB_M + 16;  // row stride: 16 doubles = half the banks

template <typename TA, int TB_K, int TB_N, typename TD>
struct TallStage {
  static constexpr int NA = TB_M * TB_K / 256, NB = TB_N * TB_K / 256;
  static constexpr int VW = 16 / sizeof(TA), NAV = NA / VW;
  static constexpr int VWD = 16 / sizeof(TD), NDV = NA / VWD;
  typedef TA av_t __attribute__((ext_vector_type(VW)));
  typedef TD dv_t __attribute__((ext_vector_type(VWD)));
  av_t a[NAV];
  dv_t d[NDV];   // the same A elements when a step reads them from D
  double b[NB];
};

// One TB_M x TB_N tile of C = alpha A B + beta Cin: rows i0.., columns j0..,
// K from kbeg to K.  Shared by the tall GEMM and the blocked triangular solve
// below (which passes the same array as A and C: every load of A that a tile
// uses completes before the tile's first store, and the pointers here are not
// restrict-qualified).  When D is given, the K steps below kd_end take their
// A elements from D (same rows and columns, leading dimension ldd, type TD)
// instead of A; the step bounds are multiples of TB_K, so a step reads one
// source only.  C's column index is shifted by c_off (Cin's is not).  With
// tri_k0 >= 0 the rows tri_k0 .. tri_k0 + TB_N - 1 of B are lower triangular
// against the tile's columns (B[tri_k0 + r][j0 + c] = 0 for r < c): a wave
// skips the products of a step whose rows all lie above its 16 columns
// (they would add exact zeros).
template <typename TA, bool VA, typename TC, int TB_K, int TB_N, typename TD = TA>
__device__ __forceinline__ void tall_tile(
    int64_t i0, int64_t j0, int64_t kbeg, int64_t M, int64_t N, int64_t K, double alpha,
    const TA* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
    int64_t ldc, const TC* Cin, int64_t ldcin, double (*As)[TB_K][TA_LD],
    double (*Bs)[TB_K][TB_N + 16], const TD* D = nullptr, int64_t ldd = 0,
    int64_t kd_end = 0, int64_t c_off = 0, int64_t tri_k0 = -1) {
  typedef TallStage<TA, TB_K, TB_N, TD> St;
  constexpr int NA = St::NA, NB = St::NB, VW = St::VW, NAV = St::NAV;
  constexpr int VWD = St::VWD, NDV = St::NDV;
  typedef typename St::dv_t dv_t;
  constexpr int WN = TB_N / 32;       // 16-column MFMA tiles per wave (2 x 2 waves)
  typedef typename St::av_t av_t;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wy = w >> 1, wx = w & 1;
  // VA staging: A row ai, NA consecutive k from ak.  Element staging: K
  // column ke of rows re + RS q.  B: k row bk, NB columns from bj.
  constexpr int RS = 256 / TB_K;
  const int ai = tid >> 1, ak = (tid & 1) * NA;
  const int ke = tid % TB_K, re = tid / TB_K;
  const int bk = tid / (TB_N / NB), bj = (tid % (TB_N / NB)) * NB;
  d4v acc[4][WN];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
  const int64_t ga = i0 + ai;
  const TA* ap = A + (ga < M ? ga : M - 1) * lda;
  const TD* dp = D ? D + (ga < M ? ga : M - 1) * ldd : nullptr;
  const int64_t gbj = j0 + bj;
  const bool dsrc_any = D != nullptr;

  auto fetch = [&](St& st, int64_t k0) {
    const bool dsrc = dsrc_any && k0 < kd_end;
    if constexpr (VA && std::is_same<TD, TA>::value) {
      // one register set: only the row pointer changes with the source
      const TA* rp = dsrc ? dp : ap;
#pragma unroll
      for (int v = 0; v < NAV; ++v)
        st.a[v] = *reinterpret_cast<const av_t*>(rp + k0 + ak + v * VW);
    } else if constexpr (VA) {
      if (dsrc) {
#pragma unroll
        for (int v = 0; v < NDV; ++v)
          st.d[v] = *reinterpret_cast<const dv_t*>(dp + k0 + ak + v * VWD);
      } else {
#pragma unroll
        for (int v = 0; v < NAV; ++v)
          st.a[v] = *reinterpret_cast<const av_t*>(ap + k0 + ak + v * VW);
      }
    } else {
#pragma unroll
      for (int v = 0; v < NAV; ++v)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int64_t row = i0 + re + RS * (v * VW + e);
          const int64_t kk = k0 + ke;
          const int64_t rc = row < M ? row : M - 1, kc = kk < K ? kk : K - 1;
          st.a[v][e] = dsrc ? (TA)D[rc * ldd + kc] : A[rc * lda + kc];
        }
    }
    const int64_t gk = (k0 + bk < K) ? k0 + bk : K - 1;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int64_t gj = (gbj + q < N) ? gbj + q : N - 1;
      st.b[q] = B[gk * ldb + gj];
    }
  };
  auto stash = [&](const St& st, int buf, int64_t k0) {
    const bool dsrc = VA && !std::is_same<TD, TA>::value && dsrc_any && k0 < kd_end;
#pragma unroll
    for (int v = 0; v < NAV; ++v)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int q = v * VW + e;
        const double xv = dsrc ? (double)st.d[q / VWD][q % VWD] : (double)st.a[v][e];
        if constexpr (VA)
          As[buf][ak + q][ai] = (k0 + ak + q < K) ? xv : 0.0;
        else
          As[buf][ke][re + RS * q] = (k0 + ke < K) ? xv : 0.0;
      }
    const bool krow = k0 + bk < K;
#pragma unroll
    for (int q = 0; q < NB; ++q) Bs[buf][bk][bj + q] = krow ? st.b[q] : 0.0;
  };
  auto mma = [&](int buf, int64_t k0) {
    // column tiles of this wave that the step leaves unchanged (uniform)
    bool zero[WN];
#pragma unroll
    for (int b = 0; b < WN; ++b)
      zero[b] = tri_k0 >= 0 && k0 >= tri_k0 &&
                k0 + TB_K - 1 - tri_k0 < (TB_N / 2) * wx + 16 * b;
#pragma unroll
    for (int ks = 0; ks < TB_K / 4; ++ks) {
      const int kr = 4 * ks + (lane >> 4);
      double av[4], bv[WN];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][kr][64 * wy + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < WN; ++b) bv[b] = Bs[buf][kr][(TB_N / 2) * wx + 16 * b + (lane & 15)];
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        if (zero[b]) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  };

  // K steps kbeg + t TB_K, t < nt.  At the top of step t, LDS buffer t%2
  // holds step t and register set (t+1)%2 holds step t+1.  Loads and
  // stores run unconditionally (steps past the end re-load the last one
  // into a buffer that is not read again), so the loop body has no
  // branches and each wait covers exactly the older register set.
  const int64_t nt = (K > kbeg) ? ceil_div(K - kbeg, TB_K) : 0;
  if (nt > 0) {
    auto kstep = [&](int64_t t) { return kbeg + (t < nt ? t : nt - 1) * TB_K; };
    St s0, s1;
    fetch(s0, kbeg);
    fetch(s1, kstep(1));
    stash(s0, 0, kbeg);
    __syncthreads();
    int64_t t = 0;
    // The scheduling barriers keep every MFMA of a step ahead of the wait
    // for the registers it stashes, so that each fetch has two steps of
    // MFMA work to arrive in.
    for (; t + 2 <= nt; t += 2) {
      // even step t: LDS 0, registers s1 = step t+1; s0 is free
      fetch(s0, kstep(t + 2));
      mma(0, kstep(t));
      __builtin_amdgcn_sched_barrier(0);
      stash(s1, 1, kstep(t + 1));
      __syncthreads();
      // odd step t+1: LDS 1, registers s0 = step t+2; s1 is free
      fetch(s1, kstep(t + 3));
      mma(1, kstep(t + 1));
      __builtin_amdgcn_sched_barrier(0);
      stash(s0, 0, kstep(t + 2));
      __syncthreads();
    }
    if (t < nt) mma(0, kstep(t));  // nt odd: the last step sits in LDS 0
  }

  // epilogue, one 16-row group of MFMA tiles at a time: its C-input loads
  // first (clamped, unconditional), then its stores, so that the loads of a
  // lane overlap instead of each waiting for the previous one
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double cin[4][WN];
    if (beta != 0.0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = min(i0 + 64 * wy + 16 * a + (lane >> 4) + 4 * q, M - 1);
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          const int64_t gj = min(j0 + (TB_N / 2) * wx + 16 * b + (lane & 15), N - 1);
          cin[q][b] = Cin ? (double)Cin[gi * ldcin + gj] : C[gi * ldc + gj];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gi = i0 + 64 * wy + 16 * a + (lane >> 4) + 4 * q;
      if (gi >= M) continue;
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        const int64_t gj = j0 + (TB_N / 2) * wx + 16 * b + (lane & 15);
        if (gj < N) {
          double v = alpha * acc[a][b][q];
          if (beta != 0.0) v += beta * cin[q][b];
          C[gi * ldc + gj - c_off] = v;
        }
      }
    }
  }
}

// Blocked substitution for W L_1 = L_2 (Alg. 3, lower-triangular L_1), one
// TB_M-row strip of W per workgroup, in place: the 64-wide column blocks J
// of W are formed from the last to the first as
//   W(:, J) = L_2(:, J) D_J^{-1} + sum_{I > J} W(:, I) Bt(I, J),
//   Bt(J, J) = D_J^{-1},  Bt(I, J) = -L_1(I, J) D_J^{-1} (I > J),
// with D_J the diagonal block of L_1: one tile whose first 64 K rows read
// L_2(:, J) from L (FP32 entries widened exactly) and the rest the finished
// blocks of W.  Without L, W itself holds L_2 (block J is read before it is
// overwritten).  Rows of one strip never depend on other rows, so no
// workgroup waits for another; the tiles of one workgroup are ordered by the
// barrier after each tile (its stores are then visible to the workgroup).
template <typename TL, bool VA, int TB_K, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_trsm_tall(
    int64_t M, int64_t K, const TL* __restrict__ L, int64_t ldl, const double* __restrict__ Bt,
    int64_t ldb, double* W, int64_t ldw) {
  constexpr int TBJ = 64;
  __shared__ double As[2][TB_K][TA_LD];
  __shared__ double Bs[2][TB_K][TBJ + 16];
  const int64_t i0 = (int64_t)blockIdx.x * TB_M;
  for (int64_t J = ceil_div(K, (int64_t)TBJ) - 1; J >= 0; --J) {
    tall_tile<double, VA, double, TB_K, TBJ, TL>(i0, TBJ * J, TBJ * J, M, K, K, 1.0, W, ldw, Bt,
                                                 ldb, 0.0, W, ldw, (const double*)nullptr, 0, As,
                                                 Bs, L, ldl, TBJ * (J + 1), 0, TBJ * J);
    __syncthreads();
  }
}

// A further refinement step on an existing W (after the first pass), fused
// per 128-row strip: with the residual E = L_2 - W L_1 the
// correction F of F L_1 = E is formed block by block from the last column
// block to the first as F(:, J) = (E(:, J) - sum_{I > J} F(:, I) L_1(I, J))
// D_J^{-1}, and W(:, J) += F(:, J) at once.  Since W(:, I) + F(:, I) is
// then what W(:, I) holds for I > J, both sums fold into one tile over the
// current W:
//   T = L_2(:, J) - sum_{I >= J} W(:, I) L_1(I, J),   W(:, J) += T D_J^{-1},
// with the strip's T in Tws (TB_M x 64 per strip, rows of the strip only).
// Bt holds D_J^{-1} on its diagonal blocks; L_1 is lower triangular.
template <typename TL, bool VA, int TB_K, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_trsm_refine_step(
    int64_t M, int64_t K, const TL* __restrict__ L, int64_t ldl, const double* __restrict__ L1,
    const double* __restrict__ Bt, double* W, int64_t ldw, double* __restrict__ Tws) {
  constexpr int TBJ = 64;
  __shared__ double As[2][TB_K][TA_LD];
  __shared__ double Bs[2][TB_K][TBJ + 16];
  const int64_t i0 = (int64_t)blockIdx.x * TB_M;
  for (int64_t J = ceil_div(K, (int64_t)TBJ) - 1; J >= 0; --J) {
    const int64_t j0 = TBJ * J, nb = min((int64_t)TBJ, K - j0);
    tall_tile<double, VA, TL, TB_K, TBJ>(i0, j0, j0, M, K, K, -1.0, W, ldw, L1, K, 1.0, Tws,
                                         TBJ, L, ldl, As, Bs, (const double*)nullptr, 0, 0, j0,
                                         j0);
    __syncthreads();
    tall_tile<double, true, double, TB_K, TBJ>(i0, 0, 0, M, nb, nb, 1.0, Tws, TBJ,
                                               Bt + j0 * K + j0, K, 1.0, W + j0, ldw, W + j0,
                                               ldw, As, Bs, (const double*)nullptr, 0, 0, 0, 0);
    __syncthreads();
  }
}


// C = Cin - A B for tall A (M x K, FP64, row-major) and B (K x N): the
// contribution of the later column blocks of W to the right sides of a
// block of columns (the super-block update of the W solve).  One 128 x 64
// tile per workgroup; the tiles of one 128-row strip run on the same XCD
// (workgroups are dealt to the eight XCDs in turn), so the strip of A is
// read from HBM once and from that XCD's L2 by its other tiles.
template <typename TC, bool VA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_gemm_tall(
    int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, const TC* __restrict__ Cin, int64_t ldcin, double* C, int64_t ldc,
    int64_t ntn, int64_t nstrips) {
  constexpr int TB_N = 64, TB_K = 8;
  __shared__ double As[2][TB_K][TA_LD];
  __shared__ double Bs[2][TB_K][TB_N + 16];
  const int64_t b = blockIdx.x;
  const int64_t xcd = b % 8, slot = b / 8;
  const int64_t strip = (slot / ntn) * 8 + xcd, tile = slot % ntn;
  if (strip >= nstrips) return;
  tall_tile<double, VA, TC, TB_K, TB_N>(strip * TB_M, tile * TB_N, 0, M, N, K, -1.0, A, lda, B,
                                        ldb, 1.0, C, ldc, Cin, ldcin, As, Bs,
                                        (const double*)nullptr, 0, 0, 0, -1);
}

hipError_t launch_gemm_tall(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                            bool a_vec, const double* B, int64_t ldb, const void* Cin,
                            int cin_f32, int64_t ldcin, double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t ntn = ceil_div(N, (int64_t)64), nstrips = ceil_div(M, (int64_t)TB_M);
  // whole groups of eight strips per XCD round (surplus workgroups exit)
  const int64_t nwg = ceil_div(nstrips, (int64_t)8) * 8 * ntn;
  const bool vec = a_vec && (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
  const dim3 g((unsigned)nwg);
#define RBRP_TALL(TCV, VAV)                                                                   \
  hipLaunchKernelGGL((k_gemm_tall<TCV, VAV>), g, dim3(256), 0, s, M, N, K, A, lda, B, ldb,   \
                     (const TCV*)Cin, ldcin, C, ldc, ntn, nstrips)
  if (cin_f32) {
    if (vec) RBRP_TALL(float, true); else RBRP_TALL(float, false);
  } else {
    if (vec) RBRP_TALL(double, true); else RBRP_TALL(double, false);
  }
#undef RBRP_TALL
  return hipGetLastError();
}

template <typename TL, bool VA>
static void trsm_typed(int64_t M, int64_t K, const TL* L, int64_t ldl, const double* Bt,
                       double* W, int64_t ldw, hipStream_t s) {
  hipLaunchKernelGGL((k_trsm_tall<TL, VA, 8, 3>), dim3((unsigned)ceil_div(M, TB_M)), dim3(256),
                     0, s, M, K, L, ldl, Bt, K, W, ldw);
}

hipError_t launch_trsm_tall(int64_t M, int64_t K, const void* L, int l_f32, int64_t ldl,
                            const double* Bt, double* W, int64_t ldw, hipStream_t s) {
  if (M <= 0 || K <= 0) return hipSuccess;
  // vector loads: 16-byte aligned rows of W (and of L when given) that
  // extend to whole K steps
  const int64_t kr = round_up(K, (int64_t)8);
  bool vec = (reinterpret_cast<uintptr_t>(W) % 16 == 0) && (ldw % 2 == 0) && ldw >= kr;
  if (L) {
    const int64_t vw = l_f32 ? 4 : 2;
    vec = vec && (reinterpret_cast<uintptr_t>(L) % 16 == 0) && (ldl % vw == 0) && ldl >= kr;
  }
  if (l_f32) {
    if (vec) trsm_typed<float, true>(M, K, (const float*)L, ldl, Bt, W, ldw, s);
    else trsm_typed<float, false>(M, K, (const float*)L, ldl, Bt, W, ldw, s);
  } else {
    if (vec) trsm_typed<double, true>(M, K, (const double*)L, ldl, Bt, W, ldw, s);
    else trsm_typed<double, false>(M, K, (const double*)L, ldl, Bt, W, ldw, s);
  }
  return hipGetLastError();
}

template <typename TL, bool VA>
static void refine_step_typed(int64_t M, int64_t K, const TL* L, int64_t ldl, const double* L1,
                              const double* Bt, double* W, int64_t ldw, double* Tws,
                              hipStream_t s) {
  hipLaunchKernelGGL((k_trsm_refine_step<TL, VA, 8, 3>), dim3((unsigned)ceil_div(M, TB_M)),
                     dim3(256), 0, s, M, K, L, ldl, L1, Bt, W, ldw, Tws);
}

hipError_t launch_trsm_refine_step(int64_t M, int64_t K, const void* L, int l_f32,
                                   int64_t ldl, const double* L1, const double* Bt, double* W,
                                   int64_t ldw, double* Tws, hipStream_t s) {
  if (M <= 0 || K <= 0) return hipSuccess;
  // vector loads of W's rows: the rows must extend to whole K steps
  const int64_t kr = round_up(K, (int64_t)8);
  const bool vec = (reinterpret_cast<uintptr_t>(W) % 16 == 0) && (ldw % 2 == 0) && ldw >= kr;
  if (l_f32) {
    if (vec) refine_step_typed<float, true>(M, K, (const float*)L, ldl, L1, Bt, W, ldw, Tws, s);
    else refine_step_typed<float, false>(M, K, (const float*)L, ldl, L1, Bt, W, ldw, Tws, s);
  } else {
    if (vec) refine_step_typed<double, true>(M, K, (const double*)L, ldl, L1, Bt, W, ldw, Tws, s);
    else refine_step_typed<double, false>(M, K, (const double*)L, ldl, L1, Bt, W, ldw, Tws, s);
  }
  return hipGetLastError();
}


}  // namespace rbrp
