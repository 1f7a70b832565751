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
#include "rbrp_wg.h"

#include <math.h>

namespace rbrp {

// One thread per column j of the block (nb <= 128, one or two waves).  Thread
// j keeps the Schur-complement diagonal entry of its column in a register and
// updates its own column of G (in LDS) at every pivot step, so the only
// cross-thread traffic per step is the argmax/sum reduction and the pivot row.
//
// After pivoting, the kernel also forms M = R11^{-T} (b' x b', lower
// triangular) by forward substitution over rows, in the same LDS array: the
// strict upper triangle keeps R11, the strict lower triangle receives M and
// the two diagonals live in separate vectors.  M is written scattered back to
// the sampled order, Mout[p][piv[c]] = M[p][c], so that the new basis rows
// are the plain product Q'^T = Mout V^T.
__global__ __launch_bounds__(128) void k_cpqr_gram(
    const double* __restrict__ G, int64_t ldg, int32_t nb_host,
    const int32_t* __restrict__ nb_dev, double tau_b, int pivoted,
    const double* __restrict__ xs2_rows, int32_t* __restrict__ piv,
    double* __restrict__ Rraw, int64_t ldr, double* __restrict__ Rperm,
    double* __restrict__ Mout, int64_t ldm, int32_t* __restrict__ bprime_out,
    double* __restrict__ tail1_out, int32_t* __restrict__ stop_out,
    const int32_t* __restrict__ run_flag) {
  extern __shared__ double Gs[];
  if (run_flag && *run_flag == 0) {
    if (threadIdx.x == 0 && nb_dev) *bprime_out = *nb_dev;
    return;
  }
  __shared__ double rrow[2][kMaxB];
  __shared__ double rdiag[kMaxB];
  __shared__ double mdiag[kMaxB];
  __shared__ int32_t pivs[kMaxB];
  __shared__ int32_t chosen_s[kMaxB];
  __shared__ double wbest[2], wtail[2];
  __shared__ int32_t wbi[2];
  const int j = threadIdx.x;
  const int lane = j & 63, wv = j >> 6;
  const int nwave = blockDim.x >> 6;
  int nb = nb_host;
  if (nb_dev) nb = min(nb, *nb_dev);
  const int ld = nb + 1;
  const bool active = j < nb;
  for (int e = j; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, c = e - r * nb;
    Gs[r * ld + c] = G[(int64_t)r * ldg + c];
  }
  __syncthreads();
  double dj = active ? Gs[j * ld + j] : 0.0;
  bool chosen = !active;
  double thr = 0.0;
  int bp = 0;
  for (int p = 0; p <= nb; ++p) {
    double best = chosen ? -INFINITY : dj;
    int bi = chosen ? -1 : j;
    double tail = chosen ? 0.0 : fmax(dj, 0.0);
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
    if (nwave > 1) {
      if (lane == 0) {
        wbest[wv] = best;
        wbi[wv] = bi;
        wtail[wv] = tail;
      }
      __syncthreads();
      best = wbest[0];
      bi = wbi[0];
      tail = wtail[0] + wtail[1];
      if (wbi[1] >= 0 && (bi < 0 || wbest[1] > best || (wbest[1] == best && wbi[1] < bi))) {
        best = wbest[1];
        bi = wbi[1];
      }
    }
    // every thread now holds the same best / bi / tail
    bool done = false;
    if (p == 0) {
      if (tail1_out && j == 0) *tail1_out = tail;
      thr = tau_b * tail * (1.0 - 4.0 * nb * 1.1102230246251565e-16);
      if (xs2_rows) {
        double xs2 = 0.0;
        for (int q = 0; q < nb; ++q) xs2 += xs2_rows[q];
        if (!(tail > 1e-26 * xs2)) {
          done = true;
          if (stop_out && j == 0) *stop_out = 1;
        }
      }
    }
    int jp = bi;
    double g = best;
    if (!pivoted && p < nb) {
      jp = p;
      g = Gs[p * ld + p];
    }
    if (p == nb || jp < 0 || !(g > 0.0)) done = true;
    if (pivoted && p > 0 && tail < thr) done = true;
    if (done) {
      bp = p;
      break;
    }
    const double r = sqrt(g);
    const int buf = p & 1;
    if (active) {
      double v;
      if (j == jp) v = r;
      else if (chosen) v = 0.0;
      else v = Gs[jp * ld + j] / r;
      rrow[buf][j] = v;
      Rraw[(int64_t)p * ldr + j] = v;
    }
    if (j == jp) chosen = true;
    if (j == 0) pivs[p] = jp;
    __syncthreads();
    if (active) {
      // G[:, j] -= rrow * rrow[j]; the pivot row and chosen columns end at zero
      const double rj = rrow[buf][j];
      if (rj != 0.0)
        for (int i = 0; i < nb; ++i) Gs[i * ld + j] -= rrow[buf][i] * rj;
      dj = Gs[j * ld + j];
    }
    __syncthreads();
  }
  if (active) chosen_s[j] = chosen ? 1 : 0;
  __syncthreads();
  if (j == 0) {
    int q = bp;
    for (int c = 0; c < nb; ++c)
      if (!chosen_s[c]) pivs[q++] = c;
    *bprime_out = bp;
  }
  __syncthreads();
  if (active) piv[j] = pivs[j];
  if (Rperm) {
    for (int e = j; e < nb * nb; e += blockDim.x) {
      const int a = e / nb, c = e - a * nb;
      Rperm[(int64_t)a * nb + c] = (a < bp && c >= a) ? Rraw[(int64_t)a * ldr + pivs[c]] : 0.0;
    }
  }
  if (!Mout) return;
  // R11[a][c] = Rraw[a][piv[c]] for a <= c < bp: strict upper part into Gs,
  // diagonal into rdiag
  __syncthreads();
  for (int e = j; e < bp * bp; e += blockDim.x) {
    const int a = e / bp, c = e - a * bp;
    if (c > a) Gs[a * ld + c] = Rraw[(int64_t)a * ldr + pivs[c]];
    else if (c == a) rdiag[a] = Rraw[(int64_t)a * ldr + pivs[a]];
  }
  __syncthreads();
  // M = R11^{-T}: M[p][c] = (delta_pc - sum_{c <= q < p} R11[q][p] M[q][c]) / R11[p][p]
  for (int p = 0; p < bp; ++p) {
    if (j <= p && j < bp) {
      double v = (j == p) ? 1.0 : 0.0;
      for (int q = j; q < p; ++q) {
        const double mq = (q == j) ? mdiag[j] : Gs[q * ld + j];
        v -= Gs[q * ld + p] * mq;
      }
      v /= rdiag[p];
      if (j == p) mdiag[p] = v;
      else Gs[p * ld + j] = v;
    }
    __syncthreads();
  }
  // scatter to the sampled order: Mout[p][pivs[c]] = M[p][c]; the whole
  // nb_host x nb_host block is cleared first so that rows and columns past b'
  // are exact zeros for the products that follow
  for (int e = j; e < nb_host * nb_host; e += blockDim.x) {
    const int a = e / nb_host, c = e - a * nb_host;
    Mout[(int64_t)a * ldm + c] = 0.0;
  }
  __syncthreads();
  for (int e = j; e < bp * bp; e += blockDim.x) {
    const int a = e / bp, c = e - a * bp;
    if (c <= a) Mout[(int64_t)a * ldm + pivs[c]] = (c == a) ? mdiag[a] : Gs[a * ld + c];
  }
}

// ---------------------------------------------------------------------------
// Pivoted Cholesky of the block's Gram matrix for the filter (256 threads).
// The Schur complement S (nb x nb) lives in LDS; thread j < nb keeps the
// diagonal entry S[j][j] in a register.  Per pivot step: a fixed-order
// argmax / sum over the diagonal (waves 0-1), the pivot row of R written to
// LDS, and the rank-one update of S spread over all 256 threads (each thread
// updates nb*nb/256 independent entries, so LDS latency overlaps).
// Outputs: pivots (kept ones first, the rest in increasing order), b', the
// pivot rows of R with unpermuted columns (Rraw), R11 in pivoted order
// (Rp, nb x nb, zero outside the leading b' x b' upper triangle), ||V||_F^2
// and the rank-guard flag.
__global__ __launch_bounds__(kPivThreads) void k_cpqr_piv(
    const double* __restrict__ G, int64_t ldg, int32_t nb_host,
    const int32_t* __restrict__ nb_dev, double tau_b,
    const double* __restrict__ xs2_rows, int32_t* __restrict__ piv,
    double* __restrict__ Rraw, int64_t ldr, double* __restrict__ Rp, int64_t ldp,
    int32_t* __restrict__ bprime_out, double* __restrict__ tail1_out,
    int32_t* __restrict__ stop_out) {
  extern __shared__ double Ss[];
  __shared__ PivShared sh;
  wg_piv_chol(G, ldg, nb_host, nb_dev, tau_b, xs2_rows, piv, Rraw, ldr, Rp, ldp, bprime_out,
              tail1_out, stop_out, Ss, sh);
}

// Q' = V(:, piv(1:b')) R11^{-1} (the orthonormal basis of the kept columns),
// as rows of Qtmp: first R11^{-1} by back substitution in one workgroup
// (thread j < b' solves column j; R11 and the inverse live in LDS as packed
// upper triangles), then
// Qtmp = (R11^{-1})^T-weighted sums of the pivoted rows of V^T on MFMA
// (k_gemm_tn16: 16 x 16 output tiles over all columns).  Rows b'..nb_host-1
// of Qtmp come out zero (R11^{-1} is zero outside its leading b' x b' block).
// Upper triangles packed row by row: element (i, j), i <= j < nb, at
// i nb - i (i - 1) / 2 + (j - i).
__device__ __forceinline__ int tri_off(int i, int j, int nb) {
  return i * nb - (i * (i - 1)) / 2 + (j - i);
}

__global__ __launch_bounds__(256) void k_tri_inv_upper(const double* __restrict__ Rp,
                                                       int64_t ldp,
                                                       const int32_t* __restrict__ bprime,
                                                       int32_t nb_host,
                                                       double* __restrict__ Rinv,
                                                       int64_t ldi) {
  // R11 and its inverse, upper triangles packed in LDS (2 x nb (nb + 1) / 2)
  extern __shared__ double tri[];
  const int bp = *bprime;
  const int nb = bp;
  double* Rs = tri;
  double* Xs = tri + (nb * (nb + 1)) / 2;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, c = e - i * nb;
    if (c >= i) Rs[tri_off(i, c, nb)] = Rp[(int64_t)i * ldp + c];
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < bp) {
    // column j: X[j][j] = 1 / R[j][j]; X[i][j] = -(sum_{p=i+1..j} R[i][p] X[p][j]) / R[i][i]
    Xs[tri_off(j, j, nb)] = 1.0 / Rs[tri_off(j, j, nb)];
    for (int i = j - 1; i >= 0; --i) {
      const double* ri = Rs + tri_off(i, 0, nb);  // ri[p] = R[i][p] for p >= i
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int p = i + 1;
      for (; p + 3 <= j; p += 4) {
        s0 += ri[p] * Xs[tri_off(p, j, nb)];
        s1 += ri[p + 1] * Xs[tri_off(p + 1, j, nb)];
        s2 += ri[p + 2] * Xs[tri_off(p + 2, j, nb)];
        s3 += ri[p + 3] * Xs[tri_off(p + 3, j, nb)];
      }
      for (; p <= j; ++p) s0 += ri[p] * Xs[tri_off(p, j, nb)];
      Xs[tri_off(i, j, nb)] = -((s0 + s1) + (s2 + s3)) / ri[i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb_host * nb_host; e += blockDim.x) {
    const int i = e / nb_host, c = e - i * nb_host;
    Rinv[(int64_t)i * ldi + c] = (i < bp && c < bp && i <= c) ? Xs[tri_off(i, c, nb)] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_ortho_first_order(const double* __restrict__ G2,
                                                           int64_t ldg,
                                                           const int32_t* __restrict__ bprime,
                                                           int32_t nb_host,
                                                           double* __restrict__ M2,
                                                           int64_t ldm,
                                                           int32_t* __restrict__ need_exact) {
  __shared__ double red[256];
  const int bp = *bprime;
  double mx = 0.0;
  for (int e = threadIdx.x; e < bp * bp; e += 256) {
    const int a = e / bp, c = e - a * bp;
    const double v = G2[(int64_t)a * ldg + c] - (a == c ? 1.0 : 0.0);
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const bool small = red[0] <= 1e-8;
  if (threadIdx.x == 0) *need_exact = small ? 0 : 1;
  if (!small) return;
  for (int e = threadIdx.x; e < nb_host * nb_host; e += 256) {
    const int a = e / nb_host, c = e - a * nb_host;
    double v = 0.0;
    if (a < bp && c < bp) {
      const double E = G2[(int64_t)a * ldg + c] - (a == c ? 1.0 : 0.0);
      if (a == c) v = 1.0 - 0.5 * E;
      else if (c < a) v = -E;
    }
    M2[(int64_t)a * ldm + c] = v;
  }
}

hipError_t launch_cpqr_piv(const double* G, int64_t ldg, int32_t nb, const int32_t* nb_dev,
                           double tau_b, const double* xs2_rows, int32_t* piv, double* Rraw,
                           int64_t ldr, double* Rp, int64_t ldp, int32_t* bprime_out,
                           double* tail1_out, int32_t* stop_out, hipStream_t s) {
  if (nb <= 0 || nb > kMaxB) return hipErrorInvalidValue;
  static bool attr_set = false;
  const size_t lds = (size_t)kMaxB * (kMaxB + 1) * sizeof(double);
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cpqr_piv,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_cpqr_piv, dim3(1), dim3(kPivThreads),
                     (size_t)nb * (nb + 1) * sizeof(double), s, G, ldg, nb, nb_dev, tau_b,
                     xs2_rows, piv, Rraw, ldr, Rp, ldp, bprime_out, tail1_out, stop_out);
  return hipGetLastError();
}

hipError_t launch_qsolve(const double* Vt, int64_t ldv, const int32_t* piv, const double* Rp,
                         int64_t ldp, const int32_t* bprime, int32_t nb_host, int64_t ncols,
                         double* Qt, int64_t ldq, double* Rinv_ws, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  if (nb_host <= 0 || nb_host > kMaxB) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_tri_inv_upper,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kMaxB * (kMaxB + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_tri_inv_upper, dim3(1), dim3(kMaxB < 256 ? 256 : kMaxB),
                     (size_t)nb_host * (nb_host + 1) * sizeof(double), s, Rp, ldp, bprime,
                     nb_host, Rinv_ws, (int64_t)nb_host);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gemm_tn_small(nb_host, ncols, nb_host, 1.0, Rinv_ws, nb_host, Vt, ldv, 0.0, Qt,
                              ldq, s, piv, bprime);
}

hipError_t launch_ortho_first_order(const double* G2, int64_t ldg, const int32_t* bprime,
                                    int32_t nb_host, double* M2, int64_t ldm,
                                    int32_t* need_exact, hipStream_t s) {
  hipLaunchKernelGGL(k_ortho_first_order, dim3(1), dim3(256), 0, s, G2, ldg, bprime, nb_host,
                     M2, ldm, need_exact);
  return hipGetLastError();
}

size_t cpqr_lds_bytes(int32_t nb) { return (size_t)nb * (nb + 1) * sizeof(double); }

hipError_t launch_cpqr_gram_ex(const double* G, int64_t ldg, int32_t nb,
                               const int32_t* nb_dev, double tau_b, int pivoted,
                               const double* xs2_rows, int32_t* piv,
                               double* Rraw, int64_t ldr, double* Rperm, double* Mout,
                               int64_t ldm, int32_t* bprime_out, double* tail1_out,
                               int32_t* stop_out, hipStream_t s, const int32_t* run_flag) {
  if (nb <= 0 || nb > kMaxB) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cpqr_gram,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)cpqr_lds_bytes(kMaxB));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int threads = nb <= 64 ? 64 : 128;
  hipLaunchKernelGGL(k_cpqr_gram, dim3(1), dim3(threads), cpqr_lds_bytes(nb), s, G, ldg, nb,
                     nb_dev, tau_b, pivoted, xs2_rows, piv, Rraw, ldr, Rperm, Mout, ldm,
                     bprime_out, tail1_out, stop_out, run_flag);
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
