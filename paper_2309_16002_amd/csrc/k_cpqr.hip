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

// Robust blockwise filtering of Alg. 2 (local CPQR + truncation, Remark 4.2)
// and the formation of the new orthonormal basis rows Q'^T.
//
// The column-pivoted QR of the block V (n x nb) is computed through its Gram
// matrix G = V^T V: greedy pivoting on the columns of V (pick the column with
// the largest residual norm, project it out of the others, eq. qr_update) is
// pivoted Cholesky on G, step for step in exact arithmetic -- the residual
// norm^2 of column j after p steps is the diagonal of the Schur complement,
// and the pivot row is R_V(p, :).  This is the QR / Cholesky correspondence
// the paper uses to relate random pivoting to RPCholesky.  One workgroup
// runs the nb sequential pivot steps (wg_piv_chol); G sits in LDS up to
// nb = 128 and is updated in place in global memory (L2) beyond that.  The
// n-long columns of V are never touched here.
//
// Truncation: tail_i = ||R_V(i:nb, i:nb)||_F^2 is the sum of the remaining
// Schur diagonal before pivot i, and b' is the last i with
// tail_i >= tau_b tail_1 (1 - 4 nb 2^-53); tails are non-increasing, so the
// pivoting stops at the first i below the threshold.
//
// Q' = V(:, piv(1:b')) R11^{-1}: R11^{-1} by a blocked triangular inverse
// (FP64 MFMA on 16 x 16 blocks) and one MFMA product over all n columns.  A
// second pass on the result (projection against the basis + Cholesky QR,
// first order when the Gram matrix is within 1e-8 of the identity, exact
// otherwise) restores orthonormality to working precision.
#include "rbrp_wg.h"

#include <math.h>

namespace rbrp {

typedef double d4v_t __attribute__((ext_vector_type(4)));

// Filter: pivoted Cholesky of G (nb <= NBMAX), see wg_piv_chol.  GS: G is the
// Schur complement itself (global memory, overwritten); otherwise it is
// copied into dynamic LDS (nb (nb + 1) doubles).
template <int NBMAX, bool GS>
__global__ __launch_bounds__(kPivThreads) void k_cpqr_piv(
    double* __restrict__ G, int64_t ldg, int32_t nb_host,
    const int32_t* __restrict__ nb_dev, double tau_b,
    const double* __restrict__ xs2_rows, int32_t* __restrict__ piv,
    double* __restrict__ Rraw, int64_t ldr, double* __restrict__ Rp, int64_t ldp,
    int32_t* __restrict__ bprime_out, double* __restrict__ tail1_out,
    int32_t* __restrict__ stop_out, int nsl, int64_t gstride) {
  extern __shared__ double Ss[];
  __shared__ PivShared<NBMAX> sh;
  wg_piv_chol<NBMAX, GS, true>(G, ldg, nb_host, nb_dev, tau_b, xs2_rows, piv, Rraw, ldr, Rp,
                               ldp, bprime_out, tail1_out, stop_out, GS ? G : Ss, sh, nsl,
                               gstride);
}

// Exact reorthogonalisation factor: Cholesky in natural order of the Gram
// matrix of the new basis rows (b' = *nb_dev), R2 into Rp.  Runs only when
// *run_flag != 0; otherwise reports b' steps done.
template <int NBMAX, bool GS>
__global__ __launch_bounds__(kPivThreads) void k_chol_reorth(
    double* __restrict__ G, int64_t ldg, int32_t nb_host, const int32_t* __restrict__ nb_dev,
    int32_t* __restrict__ piv2, double* __restrict__ Rraw, int64_t ldr,
    double* __restrict__ Rp, int64_t ldp, int32_t* __restrict__ steps_out,
    const int32_t* __restrict__ run_flag) {
  if (*run_flag == 0) {
    if (threadIdx.x == 0) *steps_out = *nb_dev;
    return;
  }
  extern __shared__ double Ss[];
  __shared__ PivShared<NBMAX> sh;
  wg_piv_chol<NBMAX, GS, false>(G, ldg, nb_host, nb_dev, 0.0, nullptr, piv2, Rraw, ldr, Rp,
                                ldp, steps_out, nullptr, nullptr, GS ? G : Ss, sh);
}

// X = R^{-1} for the upper triangular R (b' x b', b' = *bcount <= 256,
// row-major, stride ldr; entries past b' are read as zero), by 16 x 16
// blocks in one workgroup of 256 threads:
//   1. diagonal blocks: thread (k, j) forms column j of R_kk^{-1} by back
//      substitution;
//   2. off-diagonal blocks by increasing distance d = j - i from the
//      diagonal, X_ij = -X_ii sum_{l=i+1..j} R_il X_lj, one wave per block
//      and the products on FP64 MFMA (16x16x4: the accumulator of one 16 x 16
//      product is already laid out as the B operand of the next).
// Indices >= b' are padded with the identity, so the padded inverse is block
// diagonal and its leading b' x b' part is R^{-1}.  Output (nb_host x
// nb_host, stride ldx): X, or X^T with trans, there and zero elsewhere.
// With run_flag the kernel does nothing unless *run_flag != 0.
// Batched form (bcount null): workgroup g inverts the diagonal block of
// order min(nb_host, ntot - g nb_host) that starts at row and column
// g nb_host; with rtrans the block is read transposed (R(r, c) = R[c][r]: the
// upper triangular transpose of a lower triangular block).
__global__ __launch_bounds__(256) void k_tri_inv_blocked(
    const double* __restrict__ R, int64_t ldr, const int32_t* __restrict__ bcount,
    int32_t nb_host, double* __restrict__ X, int64_t ldx, int trans,
    const int32_t* __restrict__ run_flag, int rtrans, int32_t ntot) {
  if (run_flag && *run_flag == 0) return;
  __shared__ double Bd[16][16][17];  // diagonal blocks of R, then their inverses
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, lhi = lane >> 4;
  const int64_t boff = (int64_t)blockIdx.x * nb_host;
  R += boff * (ldr + 1);
  X += boff * (ldx + 1);
  const int bp = bcount ? min(*bcount, nb_host) : min(nb_host, ntot - (int)boff);
  const int nbh = bcount ? nb_host : bp;   // order of the output block
  const int nbk = (bp + 15) >> 4;
  auto rat = [&](int r, int c) -> double {
    return rtrans ? R[(int64_t)c * ldr + r] : R[(int64_t)r * ldr + c];
  };
  auto xoff = [&](int r, int c) -> int64_t {
    return trans ? (int64_t)c * ldx + r : (int64_t)r * ldx + c;
  };
  for (int e = tid; e < nbh * nbh; e += 256) {
    const int r = e / nbh, c = e - r * nbh;
    if (!((r >> 4) <= (c >> 4) && (c >> 4) < nbk)) X[xoff(r, c)] = 0.0;
  }
  for (int e = tid; e < nbk * 256; e += 256) {
    const int k = e >> 8, r = (e >> 4) & 15, c = e & 15;
    const int gr = 16 * k + r, gc = 16 * k + c;
    double v;
    if (gr < bp && gc < bp) v = c >= r ? rat(gr, gc) : 0.0;
    else v = r == c ? 1.0 : 0.0;
    Bd[k][r][c] = v;
  }
  __syncthreads();
  const int kd = tid >> 4, jd = tid & 15;
  double x[16];
  if (kd < nbk) {
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double sacc = 0.0;
#pragma unroll
      for (int l = i + 1; l < 16; ++l) sacc += Bd[kd][i][l] * x[l];
      const double num = (i == jd) ? 1.0 : -sacc;
      x[i] = (i <= jd) ? num / Bd[kd][i][i] : 0.0;
    }
  }
  __syncthreads();
  if (kd < nbk) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      Bd[kd][i][jd] = x[i];
      const int gr = 16 * kd + i, gc = 16 * kd + jd;
      if (gr < nbh && gc < nbh) X[xoff(gr, gc)] = (gr < bp && gc < bp) ? x[i] : 0.0;
    }
  }
  __syncthreads();
  for (int dd = 1; dd < nbk; ++dd) {
    for (int i = wv; i + dd < nbk; i += 4) {
      const int j = i + dd;
      d4v_t acc = {0.0, 0.0, 0.0, 0.0};
      // the off-diagonal blocks l = i+1 .. j-1 four at a time, every load of a
      // group issued before its MFMAs (indices clamped into range, values
      // masked); then the diagonal block X_jj from LDS
      const int bc = 16 * j + l16;
      for (int l0 = i + 1; l0 < j; l0 += 4) {
        double av[4][4], bv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int l = min(l0 + u, j - 1);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = 4 * s4 + lhi;
            av[u][s4] = rat(16 * i + l16, min(16 * l + kk, bp - 1));
            bv[u][s4] = X[xoff(16 * l + kk, min(bc, nbh - 1))];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool live = l0 + u < j;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = 4 * s4 + lhi;
            const int l = l0 + u;
            const double a = (live && 16 * l + kk < bp) ? av[u][s4] : 0.0;
            const double b = (live && bc < bp) ? bv[u][s4] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kk = 4 * s4 + lhi;
        const double a = (16 * j + kk < bp) ? rat(16 * i + l16, min(16 * j + kk, bp - 1)) : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bd[j][kk][l16], acc, 0, 0, 0);
      }
      d4v_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        out = __builtin_amdgcn_mfma_f64_16x16x4f64(Bd[i][l16][4 * s4 + lhi], acc[s4], out, 0,
                                                   0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = 16 * i + lhi + 4 * q, gc = 16 * j + l16;
        if (gc < nbh) X[xoff(gr, gc)] = gc < bp ? -out[q] : 0.0;
      }
    }
    __syncthreads();
  }
}

// M2^T, the transpose of the first-order inverse Cholesky factor of
// G2 = I + E when max|E| <= 1e-8 (R2^{-T} ~ I - strict_lower(E) - diag(E) / 2,
// so M2^T is upper triangular); otherwise sets *need_exact and leaves M2^T to
// the exact path.
__global__ __launch_bounds__(256) void k_ortho_first_order(const double* __restrict__ G2,
                                                           int64_t ldg,
                                                           const int32_t* __restrict__ bprime,
                                                           int32_t nb_host,
                                                           double* __restrict__ M2,
                                                           int64_t ldm,
                                                           int32_t* __restrict__ need_exact) {
  // thread (column c, part) handles rows part, part + TPC, ... of column c
  // (nb_host <= 256); eight rows' loads are issued before they are used
  __shared__ double red[256];
  const int bp = *bprime;
  const int tid = threadIdx.x;
  const int ncols = nb_host <= 64 ? 64 : (nb_host <= 128 ? 128 : 256);
  const int tpc = 256 / ncols;
  const int c = tid % ncols, part = tid / ncols;
  double mx = 0.0;
  if (c < bp) {
    for (int a0 = part; a0 < bp; a0 += 8 * tpc) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = G2[(int64_t)min(a0 + u * tpc, bp - 1) * ldg + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int a = a0 + u * tpc;
        if (a < bp) mx = fmax(mx, fabs(x[u] - (a == c ? 1.0 : 0.0)));
      }
    }
  }
  red[tid] = mx;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const bool small = red[0] <= 1e-8;
  if (tid == 0) *need_exact = small ? 0 : 1;
  if (!small) return;
  // (M2^T)[a][c] = M2[c][a]: 1 - E[a][a] / 2 on the diagonal, -E[c][a] above
  if (c < nb_host) {
    for (int a0 = part; a0 < nb_host; a0 += 8 * tpc) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int a = a0 + u * tpc;
        // the diagonal reads G2[a][a], the strict upper part G2[c][a]
        // (clamped index: always in range, used only where it applies)
        x[u] = G2[(int64_t)c * ldg + min(a, nb_host - 1)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int a = a0 + u * tpc;
        if (a >= nb_host) continue;
        double v = 0.0;
        if (a < bp && c < bp) {
          if (a == c) v = 1.0 - 0.5 * (x[u] - 1.0);
          else if (c > a) v = -x[u];
        }
        M2[(int64_t)a * ldm + c] = v;
      }
    }
  }
}

static size_t chol_lds_bytes(int32_t nb) { return (size_t)nb * (nb + 1) * sizeof(double); }
constexpr int kLdsCholMax = 128;   // largest nb whose Schur complement sits in LDS

template <typename K>
static hipError_t set_chol_lds(K kernel, bool* done) {
  if (*done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)chol_lds_bytes(kLdsCholMax));
  if (e == hipSuccess) *done = true;
  return e;
}

hipError_t launch_cpqr_piv(double* G, int64_t ldg, int32_t nb, const int32_t* nb_dev,
                           double tau_b, const double* xs2_rows, int32_t* piv, double* Rraw,
                           int64_t ldr, double* Rp, int64_t ldp, int32_t* bprime_out,
                           double* tail1_out, int32_t* stop_out, hipStream_t s, int nsl,
                           int64_t gstride) {
  if (nb <= 0 || nb > kMaxB || nsl < 1 || nsl > kNtMaxSlices) return hipErrorInvalidValue;
  if (nsl > 1 && nb > kLdsCholMax) return hipErrorInvalidValue;  // S would be G itself
  if (nb <= 64) {
    hipLaunchKernelGGL((k_cpqr_piv<64, false>), dim3(1), dim3(kPivThreads),
                       chol_lds_bytes(nb), s, G, ldg, nb, nb_dev, tau_b, xs2_rows, piv, Rraw,
                       ldr, Rp, ldp, bprime_out, tail1_out, stop_out, nsl, gstride);
  } else if (nb <= kLdsCholMax) {
    static bool attr = false;
    hipError_t e = set_chol_lds(k_cpqr_piv<kLdsCholMax, false>, &attr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cpqr_piv<kLdsCholMax, false>), dim3(1), dim3(kPivThreads),
                       chol_lds_bytes(nb), s, G, ldg, nb, nb_dev, tau_b, xs2_rows, piv, Rraw,
                       ldr, Rp, ldp, bprime_out, tail1_out, stop_out, nsl, gstride);
  } else {
    hipLaunchKernelGGL((k_cpqr_piv<kMaxB, true>), dim3(1), dim3(kPivThreads), 0, s, G, ldg,
                       nb, nb_dev, tau_b, xs2_rows, piv, Rraw, ldr, Rp, ldp, bprime_out,
                       tail1_out, stop_out, 1, (int64_t)0);
  }
  return hipGetLastError();
}

hipError_t launch_tri_inv(const double* R, int64_t ldr, const int32_t* bcount, int32_t nb_host,
                          double* X, int64_t ldx, int trans, const int32_t* run_flag,
                          hipStream_t s) {
  if (nb_host <= 0 || nb_host > kMaxB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_inv_blocked, dim3(1), dim3(256), 0, s, R, ldr, bcount, nb_host, X,
                     ldx, trans, run_flag, 0, 0);
  return hipGetLastError();
}

hipError_t launch_lower_diag_inv(const double* L, int64_t ldl, int64_t n, int32_t nbs, double* X,
                                 int64_t ldx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nbs <= 0 || nbs > kMaxB || n > INT32_MAX) return hipErrorInvalidValue;
  // the transpose of each diagonal block is upper triangular; writing the
  // inverse of that transpose transposed gives the block's own inverse
  hipLaunchKernelGGL(k_tri_inv_blocked, dim3((unsigned)ceil_div(n, (int64_t)nbs)), dim3(256), 0,
                     s, L, ldl, (const int32_t*)nullptr, nbs, X, ldx, 1,
                     (const int32_t*)nullptr, 1, (int32_t)n);
  return hipGetLastError();
}

hipError_t launch_qsolve(const double* Vt, int64_t ldv, const int32_t* piv, const double* Rp,
                         int64_t ldp, const int32_t* bprime, int32_t nb_host, int64_t ncols,
                         double* Qt, int64_t ldq, double* Rinv_ws, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipError_t e = launch_tri_inv(Rp, ldp, bprime, nb_host, Rinv_ws, nb_host, 0, nullptr, s);
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

hipError_t launch_ortho_exact(double* G2, int64_t ldg, const int32_t* bprime, int32_t nb_host,
                              int32_t* piv2, double* R2raw, double* R2, double* M2,
                              int64_t ldm, int32_t* steps_out, const int32_t* need_exact,
                              hipStream_t s) {
  if (nb_host <= 0 || nb_host > kMaxB) return hipErrorInvalidValue;
  if (nb_host <= 64) {
    hipLaunchKernelGGL((k_chol_reorth<64, false>), dim3(1), dim3(kPivThreads),
                       chol_lds_bytes(nb_host), s, G2, ldg, nb_host, bprime, piv2, R2raw,
                       (int64_t)nb_host, R2, (int64_t)nb_host, steps_out, need_exact);
  } else if (nb_host <= kLdsCholMax) {
    static bool attr = false;
    hipError_t e = set_chol_lds(k_chol_reorth<kLdsCholMax, false>, &attr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_chol_reorth<kLdsCholMax, false>), dim3(1), dim3(kPivThreads),
                       chol_lds_bytes(nb_host), s, G2, ldg, nb_host, bprime, piv2, R2raw,
                       (int64_t)nb_host, R2, (int64_t)nb_host, steps_out, need_exact);
  } else {
    hipLaunchKernelGGL((k_chol_reorth<kMaxB, true>), dim3(1), dim3(kPivThreads), 0, s, G2, ldg,
                       nb_host, bprime, piv2, R2raw, (int64_t)nb_host, R2, (int64_t)nb_host,
                       steps_out, need_exact);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // M2^T = R2^{-1}
  return launch_tri_inv(R2, nb_host, steps_out, nb_host, M2, ldm, 0, need_exact, s);
}

__global__ void k_append(const int64_t* __restrict__ idx,
                         const int32_t* __restrict__ piv,
                         const int32_t* __restrict__ bprime, int64_t kS,
                         int32_t t, int64_t* __restrict__ S,
                         int32_t* __restrict__ sel_block, int32_t* __restrict__ bchunk) {
  const int p = threadIdx.x;
  if (bchunk && p == 0) {
    const int bp = *bprime;
    bchunk[0] = min(bp, kDeflateMaxB);
    bchunk[1] = max(bp - kDeflateMaxB, 0);
  }
  if (p < *bprime) {
    const int64_t row = idx[piv[p]];
    S[kS + p] = row;
    sel_block[row] = t;
  }
}

hipError_t launch_append(const int64_t* idx, const int32_t* piv,
                         const int32_t* bprime, int64_t kS, int32_t t,
                         int64_t* S, int32_t* sel_block, int32_t* bchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_append, dim3(1), dim3(kMaxB), 0, s, idx, piv, bprime, kS, t,
                     S, sel_block, bchunk);
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
