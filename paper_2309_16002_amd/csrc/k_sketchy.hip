// Sketchy pivoting with LU and partial pivoting (SkLUPP) and the oversampled
// sketchy interpolation matrix (OSID, Algorithm 4): the comparison method of
// section 3 and Algorithm 4, on the same MFMA GEMM and FP64 machinery as RBRP.
//
//   Y = X Omega                                  (m x l, FP64 MFMA GEMM)
//   S = the first k pivot rows of Gaussian elimination with partial pivoting
//       on Y(:, 0:k)   (blocked right-looking: panels of kPanel columns; per
//       column one partial argmax over the active rows, one single-workgroup
//       pivot choice, one update of the panel's columns that also yields the
//       next column's partial argmax; per panel the block row U12 of the
//       pivot rows and one GEMM update of the columns to its right)
//   Y(S,:)^T = Q R   (Householder QR, l x k: one launch for each reflector and
//                     one to apply it; Q formed by backward accumulation)
//   P = Q R^{-T}     (l x k, back substitution one row per thread)
//   W = Y P,  W(S,:) = I   (FP64 MFMA GEMM)
//
// Only the pivot order is kept from the elimination (the skeletons); its
// multipliers are kept in place because the panel's block row needs them.
#include "rbrp_internal.h"

#include <math.h>

#include <algorithm>

namespace rbrp {

constexpr int kPanel = 32;
constexpr int kArgWG = 1024;   // workgroups of a partial argmax

struct ArgMax { double v; int64_t i; };

__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b) {
  // larger value; on equal values the lower row
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

// |x|, with NaN ordered above every number: a column holding NaN still has
// a pivot (the result is then non-finite, as the input is).
__device__ __forceinline__ double mag(double x) { return x != x ? INFINITY : fabs(x); }

__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) {
  for (int off = 32; off >= 1; off >>= 1) {
    ArgMax o;
    o.v = __shfl_xor(a.v, off, kWave);
    o.i = __shfl_xor(a.i, off, kWave);
    a = better(a, o);
  }
  return a;
}

// Workgroup argmax (256 threads) written to part[blockIdx.x].
__device__ __forceinline__ void block_argmax_store(ArgMax a, double* part_v, int64_t* part_i) {
  __shared__ double sv[4];
  __shared__ int64_t si[4];
  a = wave_argmax(a);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = a.v;
    si[w] = a.i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ArgMax r{sv[0], si[0]};
    for (int q = 1; q < 4; ++q) r = better(r, ArgMax{sv[q], si[q]});
    part_v[blockIdx.x] = r.v;
    part_i[blockIdx.x] = r.i;
  }
}

// Z = Y(:, 0:k), every row active.
__global__ __launch_bounds__(256) void k_sk_init(const double* __restrict__ Y, int64_t ldy,
                                                 int64_t m, int64_t k, double* __restrict__ Z,
                                                 int64_t ldz, int32_t* __restrict__ active) {
  const int64_t i = blockIdx.x;
  if (i >= m) return;
  for (int64_t c = threadIdx.x; c < k; c += 256) Z[i * ldz + c] = Y[i * ldy + c];
  if (threadIdx.x == 0) active[i] = 1;
}

// Partial argmax of |Z(:, j)| over the active rows.
__global__ __launch_bounds__(256) void k_sk_colmax(const double* __restrict__ Z, int64_t ldz,
                                                   int64_t m, int64_t j,
                                                   const int32_t* __restrict__ active,
                                                   double* __restrict__ part_v,
                                                   int64_t* __restrict__ part_i) {
  ArgMax a{-1.0, m};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    if (active[i]) a = better(a, ArgMax{mag(Z[i * ldz + j]), i});
  block_argmax_store(a, part_v, part_i);
}

// Pivot of column j from the partials (fixed order, one workgroup): S[j],
// the row leaves the active set, and its entries j .. c1 - 1 are kept.
__global__ __launch_bounds__(64) void k_sk_pivot(const double* __restrict__ part_v,
                                                 const int64_t* __restrict__ part_i, int ng,
                                                 const double* __restrict__ Z, int64_t ldz,
                                                 int64_t m, int64_t j, int64_t c1,
                                                 int32_t* __restrict__ active,
                                                 int64_t* __restrict__ S,
                                                 double* __restrict__ prow) {
  ArgMax a{-1.0, m};
  for (int g = threadIdx.x; g < ng; g += 64) a = better(a, ArgMax{part_v[g], part_i[g]});
  a = wave_argmax(a);
  const int64_t p = a.i;
  if (threadIdx.x == 0) {
    S[j] = p;
    active[p] = 0;
  }
  for (int64_t c = j + threadIdx.x; c < c1; c += 64) prow[c - j] = Z[p * ldz + c];
}

// Elimination of pivot column j from the active rows, inside the panel
// (columns j + 1 .. c1 - 1); the multiplier replaces Z(i, j).  With
// next_argmax, the partial argmax of the updated column j + 1.
__global__ __launch_bounds__(256) void k_sk_update(double* __restrict__ Z, int64_t ldz, int64_t m,
                                                   int64_t j, int64_t c1,
                                                   const int32_t* __restrict__ active,
                                                   const double* __restrict__ prow,
                                                   int next_argmax, double* __restrict__ part_v,
                                                   int64_t* __restrict__ part_i) {
  const double pv = prow[0];
  ArgMax a{-1.0, m};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    if (!active[i]) continue;
    double* z = Z + i * ldz;
    const double mult = pv != 0.0 ? z[j] / pv : 0.0;
    z[j] = mult;
    for (int64_t c = j + 1; c < c1; ++c) z[c] -= mult * prow[c - j];
    if (next_argmax) a = better(a, ArgMax{mag(z[j + 1]), i});
  }
  if (next_argmax) block_argmax_store(a, part_v, part_i);
}

// Block row of the panel's pivot rows: U12(t, :) = Z(p_t, c1:k) -
// sum_{s<t} L(p_t, c0 + s) U12(s, :), one thread per column.
__global__ __launch_bounds__(256) void k_sk_u12(const double* __restrict__ Z, int64_t ldz,
                                                const int64_t* __restrict__ Sp, int nbp,
                                                int64_t c0, int64_t c1, int64_t k,
                                                double* __restrict__ U12) {
  const int64_t nc = k - c1;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < nc; c += (int64_t)gridDim.x * 256) {
    for (int t = 0; t < nbp; ++t) {
      const double* zr = Z + Sp[t] * ldz;
      double v = zr[c1 + c];
      for (int s = 0; s < t; ++s) v -= zr[c0 + s] * U12[(int64_t)s * nc + c];
      U12[(int64_t)t * nc + c] = v;
    }
  }
}

// A(c, t) = Y(S(t), c): the sketched skeleton rows, transposed (l x k).
__global__ __launch_bounds__(256) void k_sk_gather(const double* __restrict__ Y, int64_t ldy,
                                                   const int64_t* __restrict__ S, int64_t k,
                                                   int64_t l, double* __restrict__ A) {
  const int64_t t = blockIdx.x;
  const double* y = Y + S[t] * ldy;
  for (int64_t c = threadIdx.x; c < l; c += 256) A[c * k + t] = y[c];
}

__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[4];
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Householder reflector of column j of A (rows j .. l-1), one workgroup:
// alpha = -sign(x0) ||x||, v = x - alpha e_1 stored over x, beta = 1/(||x||
// (||x|| + |x0|)) (0 for a zero column); R(j, j) = alpha.
__global__ __launch_bounds__(256) void k_sk_house(double* __restrict__ A, int64_t lda, int64_t l,
                                                  int64_t j, double* __restrict__ beta,
                                                  double* __restrict__ R, int64_t ldr) {
  double s = 0.0;
  for (int64_t r = j + threadIdx.x; r < l; r += 256) {
    const double x = A[r * lda + j];
    s += x * x;
  }
  s = block_sum256(s);
  if (threadIdx.x == 0) {
    const double sig = sqrt(s);
    const double x0 = A[j * lda + j];
    const double al = x0 >= 0.0 ? -sig : sig;
    A[j * lda + j] = x0 - al;
    beta[j] = sig > 0.0 ? 1.0 / (sig * (sig + fabs(x0))) : 0.0;
    R[j * ldr + j] = al;
  }
}

// Apply H_j = I - beta_j v_j v_j^T to columns c >= c_first of B (rows j .. l-1),
// one workgroup per column; with to_r, row j of the result is row j of R.
__global__ __launch_bounds__(256) void k_sk_apply(const double* __restrict__ V, int64_t ldv,
                                                  int64_t l, int64_t j,
                                                  const double* __restrict__ beta,
                                                  double* __restrict__ B, int64_t ldb,
                                                  int64_t c_first, double* __restrict__ R,
                                                  int64_t ldr) {
  const int64_t c = c_first + blockIdx.x;
  const double bj = beta[j];
  double s = 0.0;
  for (int64_t r = j + threadIdx.x; r < l; r += 256) s += V[r * ldv + j] * B[r * ldb + c];
  s = block_sum256(s);
  const double w = bj * s;
  for (int64_t r = j + threadIdx.x; r < l; r += 256) B[r * ldb + c] -= w * V[r * ldv + j];
  // row j is thread 0's own (r = j + 0)
  if (R && threadIdx.x == 0) R[j * ldr + c] = B[j * ldb + c];
}

// Q = [I_k; 0] (l x k).
__global__ __launch_bounds__(256) void k_sk_eye(double* __restrict__ Q, int64_t l, int64_t k) {
  const int64_t r = blockIdx.x;
  for (int64_t c = threadIdx.x; c < k; c += 256) Q[r * k + c] = (r == c) ? 1.0 : 0.0;
}

// P(r, :) = Q(r, :) R^{-T}: R x = Q(r, :)^T by back substitution, one row per
// thread (R upper triangular, k x k).
__global__ __launch_bounds__(64) void k_sk_backsub(const double* __restrict__ Q,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   int64_t l, int64_t k, double* __restrict__ P) {
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (r >= l) return;
  const double* q = Q + r * k;
  double* x = P + r * k;
  for (int64_t i = k - 1; i >= 0; --i) {
    double v = q[i];
    for (int64_t c = i + 1; c < k; ++c) v -= R[i * ldr + c] * x[c];
    x[i] = v / R[i * ldr + i];
  }
}

size_t sketchy_workspace_bytes(int64_t m, int64_t k, int64_t l) {
  const size_t d = sizeof(double);
  size_t b = 0;
  auto take = [&](size_t n) { b += (n + 255) / 256 * 256; };
  take(m * l * d);          // Y
  take(m * k * d);          // Z
  take(m * sizeof(int32_t));
  take(kArgWG * d);
  take(kArgWG * sizeof(int64_t));
  take(kPanel * d);         // pivot row
  take(kPanel * k * d);     // U12
  take(l * k * d);          // A
  take(l * k * d);          // Q
  take(l * k * d);          // P
  take(k * k * d);          // R
  take(k * d);              // beta
  return b + 256;
}

hipError_t launch_sketchy(const void* X, int x_f32, int64_t m, int64_t n, int64_t ldx,
                          int64_t k, int64_t l, const double* Omega, int64_t ldo, int64_t* S,
                          double* W, int64_t ldw, void* ws, hipStream_t s) {
  char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  size_t off = 0;
  auto take = [&](size_t n) {
    char* p = base + off;
    off += (n + 255) / 256 * 256;
    return p;
  };
  const size_t d = sizeof(double);
  double* Y = (double*)take(m * l * d);
  double* Z = (double*)take(m * k * d);
  int32_t* active = (int32_t*)take(m * sizeof(int32_t));
  double* part_v = (double*)take(kArgWG * d);
  int64_t* part_i = (int64_t*)take(kArgWG * sizeof(int64_t));
  double* prow = (double*)take(kPanel * d);
  double* U12 = (double*)take(kPanel * k * d);
  double* A = (double*)take(l * k * d);
  double* Q = (double*)take(l * k * d);
  double* P = (double*)take(l * k * d);
  double* R = (double*)take(k * k * d);
  double* beta = (double*)take(k * d);
  const int64_t ldy = l, ldz = k;
  hipError_t e;
  // the sketch
  e = launch_gemm_f64(0, 0, m, l, n, 1.0, X, x_f32, ldx, Omega, ldo, 0.0, Y, ldy, nullptr,
                      nullptr, 0, s);
  if (e != hipSuccess) return e;
  // partial-pivoting elimination on Y(:, 0:k), panels of kPanel columns
  const int ng = (int)std::min<int64_t>(kArgWG, ceil_div(m, (int64_t)256));
  hipLaunchKernelGGL(k_sk_init, dim3((unsigned)m), dim3(256), 0, s, Y, ldy, m, k, Z, ldz, active);
  hipLaunchKernelGGL(k_sk_colmax, dim3(ng), dim3(256), 0, s, Z, ldz, m, (int64_t)0, active,
                     part_v, part_i);
  for (int64_t c0 = 0; c0 < k; c0 += kPanel) {
    const int64_t c1 = std::min<int64_t>(c0 + kPanel, k);
    for (int64_t j = c0; j < c1; ++j) {
      hipLaunchKernelGGL(k_sk_pivot, dim3(1), dim3(64), 0, s, part_v, part_i, ng, Z, ldz, m, j,
                         c1, active, S, prow);
      hipLaunchKernelGGL(k_sk_update, dim3(ng), dim3(256), 0, s, Z, ldz, m, j, c1, active, prow,
                         (int)(j + 1 < c1), part_v, part_i);
    }
    if (c1 < k) {
      const int64_t nc = k - c1;
      hipLaunchKernelGGL(k_sk_u12, dim3((unsigned)ceil_div(nc, (int64_t)256)), dim3(256), 0, s, Z,
                         ldz, S + c0, (int)(c1 - c0), c0, c1, k, U12);
      e = launch_gemm_f64(0, 0, m, nc, c1 - c0, -1.0, Z + c0, 0, ldz, U12, nc, 1.0, Z + c1, ldz,
                          nullptr, nullptr, 0, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_sk_colmax, dim3(ng), dim3(256), 0, s, Z, ldz, m, c1, active, part_v,
                         part_i);
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess || !W) return e;
  // OSID: Householder QR of A = Y(S,:)^T, Q formed explicitly, P = Q R^{-T}
  hipLaunchKernelGGL(k_sk_gather, dim3((unsigned)k), dim3(256), 0, s, Y, ldy, S, k, l, A);
  for (int64_t j = 0; j < k; ++j) {
    hipLaunchKernelGGL(k_sk_house, dim3(1), dim3(256), 0, s, A, k, l, j, beta, R, k);
    if (j + 1 < k)
      hipLaunchKernelGGL(k_sk_apply, dim3((unsigned)(k - j - 1)), dim3(256), 0, s, A, k, l, j,
                         beta, A, k, j + 1, R, k);
  }
  hipLaunchKernelGGL(k_sk_eye, dim3((unsigned)l), dim3(256), 0, s, Q, l, k);
  for (int64_t j = k - 1; j >= 0; --j)
    hipLaunchKernelGGL(k_sk_apply, dim3((unsigned)(k - j)), dim3(256), 0, s, A, k, l, j, beta, Q,
                       k, j, (double*)nullptr, k);
  hipLaunchKernelGGL(k_sk_backsub, dim3((unsigned)ceil_div(l, (int64_t)64)), dim3(64), 0, s, Q, R,
                     k, l, k, P);
  e = launch_gemm_f64(0, 0, m, k, l, 1.0, Y, 0, ldy, P, k, 0.0, W, ldw, nullptr, nullptr, 0, s);
  if (e != hipSuccess) return e;
  return launch_identity_rows(S, k, W, ldw, s);
}

}  // namespace rbrp
