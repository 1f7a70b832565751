// Robust blockwise filtering of Alg. 2 (local CPQR + truncation, Remark 4.2)
// and the formation of the new orthonormal basis rows Q'^T.
//
// The column-pivoted QR of the block V (n x nb) is computed through its Gram
// matrix G = V^T V: greedy pivoting on the columns of V (pick the column with
// the largest residual norm, project it out of the others, eq. qr_update) is
// pivoted Cholesky on G, step for step in exact arithmetic -- the residual
// norm^2 of column j after p steps is the diagonal of the Schur complement,
// and the pivot row is R_V(p, :).  This is the QR / Cholesky correspondence
// the paper uses to relate random pivoting to RPCholesky.  The whole nb x nb
// G (nb <= 128) sits in LDS and one workgroup runs the nb sequential pivot
// steps; the n-long columns of V are never touched here.
//
// Truncation: tail_i = ||R_V(i:nb, i:nb)||_F^2 is the sum of the remaining
// Schur diagonal before pivot i, and b' is the last i with
// tail_i >= tau_b tail_1 (1 - 4 nb 2^-53); tails are non-increasing, so the
// pivoting stops at the first i below the threshold.
//
// Q' is recovered row-wise as Q'^T = R11^{-T} V(:, piv(1:b'))^T (forward
// substitution, one thread per column), and a second pass on the result
// (projection against the basis + unpivoted Cholesky QR) restores
// orthonormality to working precision.
#include "rbrp_internal.h"

#include <math.h>

namespace rbrp {

constexpr int kCpqrThreads = 256;

__global__ __launch_bounds__(kCpqrThreads) void k_cpqr_gram(
    const double* __restrict__ G, int64_t ldg, int32_t nb_host,
    const int32_t* __restrict__ nb_dev, double tau_b, int pivoted,
    const double* __restrict__ xs2_rows, int32_t* __restrict__ piv,
    double* __restrict__ Rraw, int64_t ldr, double* __restrict__ Rperm,
    int32_t* __restrict__ bprime_out, double* __restrict__ tail1_out,
    int32_t* __restrict__ stop_out) {
  extern __shared__ double Gs[];
  __shared__ double rrow[kMaxB];
  __shared__ int32_t chosen[kMaxB];
  __shared__ int32_t pivs[kMaxB];
  __shared__ double wbest[4];
  __shared__ int32_t wbi[4];
  __shared__ double wtail[4];
  __shared__ int32_t s_piv, s_done, s_bp;
  __shared__ double s_thr, s_r;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  int nb = nb_host;
  if (nb_dev) nb = min(nb, *nb_dev);
  const int ld = nb + 1;
  for (int e = tid; e < nb * nb; e += kCpqrThreads) {
    const int i = e / nb, j = e - i * nb;
    Gs[i * ld + j] = G[(int64_t)i * ldg + j];
  }
  for (int j = tid; j < kMaxB; j += kCpqrThreads) chosen[j] = 0;
  if (tid == 0) {
    s_done = 0;
    s_bp = 0;
  }
  __syncthreads();
  int bp = 0;
  for (int p = 0; p <= nb; ++p) {
    // remaining diagonal: argmax (ties to the lowest column) and sum
    double best = -INFINITY;
    int bi = -1;
    double tail = 0.0;
    for (int j = tid; j < nb; j += kCpqrThreads) {
      if (!chosen[j]) {
        const double v = Gs[j * ld + j];
        tail += fmax(v, 0.0);
        if (v > best) { best = v; bi = j; }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, kWave);
      const int oi = __shfl_xor(bi, off, kWave);
      tail += __shfl_xor(tail, off, kWave);
      if (oi >= 0 && (bi < 0 || ob > best || (ob == best && oi < bi))) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      wbest[wv] = best;
      wbi[wv] = bi;
      wtail[wv] = tail;
    }
    __syncthreads();
    if (tid == 0) {
      double b2 = -INFINITY, t2 = 0.0;
      int i2 = -1;
      for (int q = 0; q < 4; ++q) {
        t2 += wtail[q];
        if (wbi[q] >= 0 && (i2 < 0 || wbest[q] > b2 || (wbest[q] == b2 && wbi[q] < i2))) {
          b2 = wbest[q];
          i2 = wbi[q];
        }
      }
      int done = 0;
      if (p == 0) {
        if (tail1_out) *tail1_out = t2;
        s_thr = tau_b * t2 * (1.0 - 4.0 * nb * 1.1102230246251565e-16);
        if (xs2_rows) {
          double xs2 = 0.0;
          for (int q = 0; q < nb; ++q) xs2 += xs2_rows[q];
          if (!(t2 > 1e-26 * xs2)) {
            done = 1;
            if (stop_out) *stop_out = 1;
          }
        }
      }
      if (pivoted) {
        if (p == nb || i2 < 0 || !(b2 > 0.0) || (p > 0 && t2 < s_thr)) done = 1;
      } else {
        if (p == nb) done = 1;
        else {
          i2 = p;
          b2 = Gs[p * ld + p];
          if (!(b2 > 0.0)) done = 1;
        }
      }
      s_done = done;
      if (!done) {
        s_piv = i2;
        s_r = sqrt(b2);
        pivs[p] = i2;
        chosen[i2] = 1;
      } else {
        s_bp = p;
      }
    }
    __syncthreads();
    if (s_done) {
      bp = s_bp;
      break;
    }
    const int jp = s_piv;
    const double r = s_r;
    // pivot row of R (unpermuted columns)
    for (int j = tid; j < nb; j += kCpqrThreads) {
      double v;
      if (j == jp) v = r;
      else if (chosen[j]) v = 0.0;
      else v = Gs[jp * ld + j] / r;
      rrow[j] = v;
      Rraw[(int64_t)p * ldr + j] = v;
    }
    __syncthreads();
    // Schur complement update on the remaining columns
    for (int e = tid; e < nb * nb; e += kCpqrThreads) {
      const int i = e / nb, j = e - i * nb;
      if (!chosen[i] && !chosen[j]) Gs[i * ld + j] -= rrow[i] * rrow[j];
    }
    __syncthreads();
  }
  // pivot order: the kept pivots, then the rest in increasing column order
  if (tid == 0) {
    int q = bp;
    for (int j = 0; j < nb; ++j)
      if (!chosen[j]) pivs[q++] = j;
    *bprime_out = bp;
  }
  __syncthreads();
  for (int j = tid; j < nb; j += kCpqrThreads) piv[j] = pivs[j];
  if (Rperm) {
    for (int e = tid; e < nb * nb; e += kCpqrThreads) {
      const int p = e / nb, q = e - p * nb;
      Rperm[(int64_t)p * nb + q] = (p < bp && q >= p) ? Rraw[(int64_t)p * ldr + pivs[q]] : 0.0;
    }
  }
}

size_t cpqr_lds_bytes(int32_t nb) { return (size_t)nb * (nb + 1) * sizeof(double); }

hipError_t launch_cpqr_gram_ex(const double* G, int64_t ldg, int32_t nb,
                               const int32_t* nb_dev, double tau_b, int pivoted,
                               const double* xs2_rows, int32_t* piv,
                               double* Rraw, int64_t ldr, double* Rperm,
                               int32_t* bprime_out, double* tail1_out,
                               int32_t* stop_out, hipStream_t s) {
  if (nb <= 0 || nb > kMaxB) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cpqr_gram,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)cpqr_lds_bytes(kMaxB));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_cpqr_gram, dim3(1), dim3(kCpqrThreads), cpqr_lds_bytes(nb), s,
                     G, ldg, nb, nb_dev, tau_b, pivoted, xs2_rows, piv, Rraw, ldr,
                     Rperm, bprime_out, tail1_out, stop_out);
  return hipGetLastError();
}

// Row-wise forward substitution Qt[p,:] = (Vt[piv[p],:] - sum_{q<p}
// R[q][piv[p]] Qt[q,:]) / R[p][piv[p]], one thread per column.  Works in
// place (Vt == Qt with piv == NULL).
__global__ __launch_bounds__(256) void k_qform(const double* Vt, int64_t ldv,
                                               const int32_t* __restrict__ piv,
                                               const double* __restrict__ R,
                                               int64_t ldr,
                                               const int32_t* __restrict__ bprime,
                                               int64_t n, double* Qt, int64_t ldq) {
  __shared__ double rc[kMaxB];
  const int bp = *bprime;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int p = 0; p < bp; ++p) {
    const int jp = piv ? piv[p] : p;
    for (int q = threadIdx.x; q <= p; q += 256) rc[q] = R[(int64_t)q * ldr + jp];
    __syncthreads();
    if (c < n) {
      double v = Vt[(int64_t)jp * ldv + c];
      for (int q = 0; q < p; ++q) v -= rc[q] * Qt[(int64_t)q * ldq + c];
      Qt[(int64_t)p * ldq + c] = v / rc[p];
    }
    __syncthreads();
  }
}

hipError_t launch_qform(const double* Vt, int64_t ldv, const int32_t* piv,
                        const double* R, int64_t ldr, const int32_t* bprime,
                        int32_t bmax, int64_t n, double* Qt, int64_t ldq,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qform, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, Vt,
                     ldv, piv, R, ldr, bprime, n, Qt, ldq);
  return hipGetLastError();
}

__global__ void k_append(const int64_t* __restrict__ idx,
                         const int32_t* __restrict__ piv,
                         const int32_t* __restrict__ bprime, int64_t kS,
                         int32_t t, int64_t* __restrict__ S,
                         int32_t* __restrict__ sel_block) {
  const int p = threadIdx.x;
  if (p < *bprime) {
    const int64_t row = idx[piv[p]];
    S[kS + p] = row;
    sel_block[row] = t;
  }
}

hipError_t launch_append(const int64_t* idx, const int32_t* piv,
                         const int32_t* bprime, int64_t kS, int32_t t,
                         int64_t* S, int32_t* sel_block, hipStream_t s) {
  hipLaunchKernelGGL(k_append, dim3(1), dim3(kMaxB), 0, s, idx, piv, bprime, kS, t,
                     S, sel_block);
  return hipGetLastError();
}

// Vt[j,:] = X[idx[j],:] in FP64 (zero rows beyond nt, zero columns beyond n),
// xs2[j] = ||X[idx[j],:]||^2.
template <typename TX>
__global__ __launch_bounds__(256) void k_gather(const TX* __restrict__ X, int64_t n,
                                                int64_t ldx,
                                                const int64_t* __restrict__ idx,
                                                const DevScalars* __restrict__ sc,
                                                double* __restrict__ Vt, int64_t ldv,
                                                double* __restrict__ xs2) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const bool live = j < sc->nt;
  const int64_t row = live ? idx[j] : 0;
  double acc = 0.0;
  for (int64_t c = threadIdx.x; c < ldv; c += 256) {
    const double v = (live && c < n) ? (double)X[row * ldx + c] : 0.0;
    Vt[(int64_t)j * ldv + c] = v;
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) xs2[j] = red[0];
}

hipError_t launch_gather_rows(const void* X, rbrp_dtype dt, int64_t n, int64_t ldx,
                              const int64_t* idx, const DevScalars* sc, int32_t bmax,
                              double* Vt, int64_t ldv, double* xs2, hipStream_t s) {
  if (dt == RBRP_F64)
    hipLaunchKernelGGL((k_gather<double>), dim3(bmax), dim3(256), 0, s,
                       (const double*)X, n, ldx, idx, sc, Vt, ldv, xs2);
  else
    hipLaunchKernelGGL((k_gather<float>), dim3(bmax), dim3(256), 0, s,
                       (const float*)X, n, ldx, idx, sc, Vt, ldv, xs2);
  return hipGetLastError();
}

}  // namespace rbrp
