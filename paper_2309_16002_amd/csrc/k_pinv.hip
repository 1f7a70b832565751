// Interpolation matrix through the truncated-SVD pseudo-inverse of L_1
// (Remark 5.2, the stable alternative to Alg. 3's substitution):
//   W(S,:) = I,  W = L L_1^+,  L_1^+ = V_r diag(1/sigma_r) U_r^T,
// with the singular values below clip * sigma_max of L_1 = L(S,:) (lower
// triangular, k x k) dropped together with their singular vectors.
//
// SVD by one-sided (Hestenes) Jacobi in FP64: the columns of G = L_1 are
// rotated pairwise until they are orthogonal, G V = U Sigma, V accumulated
// from the identity.  The columns of G and of V are stored as rows (Gt, Vt,
// row-major, leading dimension ld) so that a pair's rotation reads and writes
// two contiguous rows.  One sweep is kp - 1 rounds of the circle schedule
// (kp = k rounded up to even; the index k is a dummy when k is odd), each
// round one launch of kp / 2 independent pairs; sweeps repeat until a sweep
// rotates no pair whose columns have a cosine above tol.  After it,
// row i of Gt is sigma_i u_i^T, so
//   L_1^+ = sum_{kept i} v_i u_i^T / sigma_i = Vt^T diag(d) Gt,
//   d_i = 1 / sigma_i^2 (kept) or 0,
// one k x k product, and W = L L_1^+ one tall product.
#include "rbrp_internal.h"

#include <math.h>

namespace rbrp {

// Gt(i, p) = L_1(p, i) = L(S(p), i) for i <= p, else 0; Vt = I.
template <typename TL>
__global__ __launch_bounds__(256) void k_pinv_init(const TL* __restrict__ L, int64_t ldl,
                                                   const int64_t* __restrict__ S, int64_t k,
                                                   double* __restrict__ Gt, double* __restrict__ Vt,
                                                   int64_t ld) {
  const int64_t p = blockIdx.x;
  const int64_t row = S[p];
  for (int64_t i = threadIdx.x; i < k; i += 256) {
    Gt[i * ld + p] = (i <= p) ? (double)L[row * ldl + i] : 0.0;
    Vt[p * ld + i] = (i == p) ? 1.0 : 0.0;
  }
}

// Sum over the 256 threads of a workgroup in a fixed order.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// One round of the circle schedule: pair q of round r.
__global__ __launch_bounds__(256) void k_jacobi_round(double* __restrict__ Gt,
                                                      double* __restrict__ Vt, int64_t k,
                                                      int64_t ld, int64_t kp, int64_t r,
                                                      double tol, int32_t* __restrict__ rotated) {
  __shared__ double red[3][4];
  const int64_t n1 = kp - 1;
  const int64_t q = blockIdx.x;
  int64_t a, b;
  if (q == 0) {
    a = r;
    b = n1;
  } else {
    a = (r + q) % n1;
    b = (r - q + n1) % n1;
  }
  const int64_t i = a < b ? a : b, j = a < b ? b : a;
  if (j >= k) return;   // the dummy index of an odd k
  double* gi = Gt + i * ld;
  double* gj = Gt + j * ld;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int64_t p = threadIdx.x; p < k; p += 256) {
    const double x = gi[p], y = gj[p];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  al = block_sum(al, red[0]);
  be = block_sum(be, red[1]);
  ga = block_sum(ga, red[2]);
  if (!(fabs(ga) > tol * sqrt(al * be))) return;   // orthogonal to tol (or a zero column)
  // rotation that makes the two columns orthogonal (the smaller angle)
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  for (int64_t p = threadIdx.x; p < k; p += 256) {
    const double x = gi[p], y = gj[p];
    gi[p] = c * x - s * y;
    gj[p] = s * x + c * y;
  }
  double* vi = Vt + i * ld;
  double* vj = Vt + j * ld;
  for (int64_t p = threadIdx.x; p < k; p += 256) {
    const double x = vi[p], y = vj[p];
    vi[p] = c * x - s * y;
    vj[p] = s * x + c * y;
  }
  if (threadIdx.x == 0) atomicAdd(rotated, 1);
}

__global__ __launch_bounds__(64) void k_pinv_zero(int32_t* __restrict__ x) {
  if (threadIdx.x == 0) *x = 0;
}

// sq(i) = ||Gt(i,:)||^2 = sigma_i^2, one workgroup per row (fixed order).
__global__ __launch_bounds__(256) void k_pinv_rownorm(const double* __restrict__ Gt, int64_t k,
                                                      int64_t ld, double* __restrict__ sq) {
  __shared__ double red[4];
  const double* g = Gt + (int64_t)blockIdx.x * ld;
  double v = 0.0;
  for (int64_t p = threadIdx.x; p < k; p += 256) v += g[p] * g[p];
  v = block_sum(v, red);
  if (threadIdx.x == 0) sq[blockIdx.x] = v;
}

// d_i = 1 / sigma_i^2 for sigma_i >= clip * sigma_max, else 0 (one
// workgroup); kept = the number of singular values kept.
__global__ __launch_bounds__(256) void k_pinv_weights(const double* __restrict__ sq, int64_t k,
                                                      double clip, double* __restrict__ dw,
                                                      int32_t* __restrict__ kept) {
  __shared__ double mx[4];
  __shared__ int32_t cnt[4];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < k; i += 256) v = fmax(v, sq[i]);
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = v;
  __syncthreads();
  const double smax2 = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
  const double thr2 = clip * clip * smax2;
  int32_t c = 0;
  for (int64_t i = threadIdx.x; i < k; i += 256) {
    const bool keep = sq[i] > 0.0 && sq[i] >= thr2;
    dw[i] = keep ? 1.0 / sq[i] : 0.0;
    c += keep ? 1 : 0;
  }
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, kWave);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *kept = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Gt(i,:) *= d_i
__global__ __launch_bounds__(256) void k_pinv_scale(double* __restrict__ Gt, int64_t k, int64_t ld,
                                                    const double* __restrict__ dw) {
  const double s = dw[blockIdx.x];
  double* g = Gt + (int64_t)blockIdx.x * ld;
  for (int64_t p = threadIdx.x; p < k; p += 256) g[p] *= s;
}

size_t pinv_workspace_doubles(int64_t k) {
  return (size_t)(3 * k * k + 2 * k + 64);
}

hipError_t launch_interp_pinv(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t k,
                              const int64_t* S, double* W, int64_t ldw, double clip,
                              double* ws, int32_t* kept_host, hipStream_t s) {
  if (k <= 0 || m <= 0) return hipSuccess;
  const int64_t ld = k;
  double* Gt = ws;
  double* Vt = Gt + k * k;
  double* P = Vt + k * k;
  double* sq = P + k * k;
  double* dw = sq + k;
  int32_t* rotated = reinterpret_cast<int32_t*>(dw + k);
  int32_t* kept = rotated + 1;
  if (l_f64)
    hipLaunchKernelGGL(k_pinv_init<double>, dim3((unsigned)k), dim3(256), 0, s,
                       (const double*)L, ldl, S, k, Gt, Vt, ld);
  else
    hipLaunchKernelGGL(k_pinv_init<float>, dim3((unsigned)k), dim3(256), 0, s,
                       (const float*)L, ldl, S, k, Gt, Vt, ld);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t kp = k + (k & 1);
  const double tol = (double)(k > 1 ? k : 1) * ldexp(1.0, -53);
  constexpr int kMaxSweeps = 40;
  int sweep = 0;
  bool converged = k < 2;
  int32_t hrot = 0;
  while (!converged && sweep < kMaxSweeps) {
    hipLaunchKernelGGL(k_pinv_zero, dim3(1), dim3(64), 0, s, rotated);
    for (int64_t r = 0; r + 1 < kp; ++r)
      hipLaunchKernelGGL(k_jacobi_round, dim3((unsigned)(kp / 2)), dim3(256), 0, s, Gt, Vt, k,
                         ld, kp, r, tol, rotated);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&hrot, rotated, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    ++sweep;
    converged = hrot == 0;
  }
  if (!converged) return hipErrorNotReady;
  hipLaunchKernelGGL(k_pinv_rownorm, dim3((unsigned)k), dim3(256), 0, s, Gt, k, ld, sq);
  hipLaunchKernelGGL(k_pinv_weights, dim3(1), dim3(256), 0, s, sq, k, clip, dw, kept);
  hipLaunchKernelGGL(k_pinv_scale, dim3((unsigned)k), dim3(256), 0, s, Gt, k, ld, dw);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // P = L_1^+ = Vt^T diag(d) Gt, then W = L P
  e = launch_gemm_f64(1, 0, k, k, k, 1.0, Vt, 0, ld, Gt, ld, 0.0, P, k, nullptr, nullptr, 0, s);
  if (e != hipSuccess) return e;
  e = launch_gemm_f64(0, 0, m, k, k, 1.0, L, l_f64 ? 0 : 1, ldl, P, k, 0.0, W, ldw, nullptr,
                      nullptr, 0, s);
  if (e != hipSuccess) return e;
  e = launch_identity_rows(S, k, W, ldw, s);
  if (e != hipSuccess) return e;
  if (kept_host) {
    e = hipMemcpyAsync(kept_host, kept, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rbrp
