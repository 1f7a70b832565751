// Interpolation matrix from the Cholesky-like factor L (Algorithm 3,
// Prop. 5.1): with L_1 = L(S,:) (k x k, lower triangular because the rows of
// earlier skeletons are zero in later blocks of L), W(S,:) = I and
// W(rest,:) = L_2 L_1^{-1}, which equals X X_S^+ (eq. stable_id).
//
// All in FP64, by substitution as in Alg. 3:
//   1. L_1 gathered from the rows S of L (strict upper part set to zero);
//   2. the 64 x 64 diagonal blocks D_J of L_1 inverted (one workgroup each,
//      by 16 x 16 blocks on FP64 MFMA); without refinement also the
//      sub-diagonal blocks scaled, Bt(I, J) = -L_1(I, J) D_J^{-1} (one small
//      MFMA GEMM per block column);
//   3. W L_1 = L solved in place in W by blocked substitution over the block
//      columns, from the last to the first (super-blocks of 256 columns: the
//      later super-blocks' part by one tall MFMA GEMM, then each row's
//      substitution with W in registers), with the first refinement step
//      (the residual E = L - W L_1, F L_1 = E, W += F) taken block by block
//      in the same pass; further steps are one more pass each;
//   4. W(S(j),:) = e_j exactly.
#include "rbrp_internal.h"

#include <algorithm>

namespace rbrp {

constexpr int kDiag = 64;
constexpr int kRegsNJ = 4;   // column blocks of 64 per super-block of the W solve
constexpr int kRegsNB = 1;   // 16-row column blocks of W^T per wave
constexpr int64_t kSuper = 64 * kRegsNJ;   // columns of a super-block

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

typedef double d4w __attribute__((ext_vector_type(4)));

// The A operands of the register-resident substitution below, per
// super-block of at most 64 NJ columns, written once in the order the
// lanes read them: fragment f is 64 doubles, lane l's element at f * 64 + l,
// for the FP64 16x16x4 MFMA's A layout (lane l supplies row l%16, K index
// l/16 of a 16 x 4 step).  Block (jb, kb) of a 64 x 64 operand at K step s
// holds element (16 jb + l%16, 16 kb + 4 s + l/16) of the transposed matrix.
// Per super-block:
//   * for each pair of column blocks I > J (pair index I (I-1)/2 + J):
//     -L_1(I, J)^T, 64 fragments (jb, kb, s);
//   * for each column block J: D_J^{-T} then -D_J^T, 40 fragments each
//     (the blocks kb >= jb of these upper triangular operands, in the order
//     (0,0..3), (1,1..3), (2,2..3), (3,3), four steps each).
// Indices past the super-block's K columns are zero, so the solve needs no
// masks and every fragment load is one contiguous, unconditional load.

// (jb, kb >= jb) -> index 0..9 of a block of an upper triangular operand
constexpr int regs_tri(int jb, int kb) { return jb * 4 - jb * (jb - 1) / 2 + (kb - jb); }

template <int NJ>
struct RegsFrags {
  static constexpr int kPairs = NJ * (NJ - 1) / 2;
  static constexpr int kPerSb = 64 * kPairs + 80 * NJ;
  static constexpr int pair(int I, int J) { return 64 * (I * (I - 1) / 2 + J); }
  static constexpr int diag(int J) { return 64 * kPairs + 80 * J; }
};

template <int NJ>
__global__ __launch_bounds__(256) void k_trsm_regs_frags(const double* __restrict__ L1,
                                                         const double* __restrict__ Bt,
                                                         int64_t k, double* __restrict__ F) {
  typedef RegsFrags<NJ> RF;
  const int sb = blockIdx.y;
  const int64_t a = (int64_t)sb * 64 * NJ;
  const int64_t K = min((int64_t)64 * NJ, k - a);
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= RF::kPerSb) return;
  const int lane = threadIdx.x & 63, l16 = lane & 15, lhi = lane >> 4;
  // which matrix block this fragment comes from
  int64_t r0, c0;  // element (row r0 + i, column c0 + j) of X, i = K index, j = row index
  int jb, kb, s, ni, nj;
  bool neg;
  const double* X;
  if (f < 64 * RF::kPairs) {
    const int p = f / 64, g = f % 64;
    int I = 1;
    while ((I + 1) * I / 2 <= p) ++I;
    const int J = p - I * (I - 1) / 2;
    jb = g / 16; kb = (g / 4) % 4; s = g % 4;
    X = L1; r0 = a + 64 * I; c0 = a + 64 * J;
    ni = (int)max((int64_t)0, min((int64_t)64, K - 64 * I)); nj = 64;
    neg = true;
  } else {
    const int h = f - 64 * RF::kPairs, J = h / 80, g = h % 80;
    const int t = (g % 40) / 4;
    s = g % 4;
    jb = t < 4 ? 0 : t < 7 ? 1 : t < 9 ? 2 : 3;
    kb = jb + t - regs_tri(jb, jb);
    X = g < 40 ? Bt : L1;
    neg = g >= 40;
    r0 = a + 64 * J; c0 = r0;
    ni = nj = (int)max((int64_t)0, min((int64_t)64, K - 64 * J));
  }
  const int i = 16 * kb + 4 * s + lhi, j = 16 * jb + l16;
  double v = 0.0;
  if (i < ni && j < nj) v = X[(r0 + i) * k + c0 + j];
  F[((int64_t)sb * RF::kPerSb + f) * 64 + lane] = neg ? -v : v;
}

// Ra -= L_1(I, J)^T W^T(I) for the later block I of the super-block: the K
// steps over the KI live 16-row tiles of block I (past them both operands
// are zero).  Fp: the pair's fragments.
template <int KI, int NB>
__device__ __forceinline__ void regs_pair(d4w (&Ra)[4][NB], const d4w (&Wi)[4][NB],
                                          const double* Fp) {
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int kb = 0; kb < KI; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = Fp[64 * (16 * jb + 4 * kb + s)];
#pragma unroll
        for (int n = 0; n < NB; ++n)
          Ra[jb][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wi[kb][n][s], Ra[jb][n], 0, 0, 0);
      }
}

// The three products against the diagonal block D_J with KJ live 16-column
// tiles (Fdi: the fragments of D_J^{-T}, then those of -D_J^T):
//   W^T(J) = D_J^{-T} R^T,  T^T = R^T - D_J^T W^T(J) (in place of R^T),
//   W^T(J) += D_J^{-T} T^T.
// Both operands are upper triangular by 16 x 16 blocks (block row jb takes
// the blocks kb >= jb) and zero at tiles >= KJ, so those rows of W^T(J) are
// zero and those of T^T are not needed.
template <int KJ, int NB>
__device__ __forceinline__ void regs_diag(d4w (&Ra)[4][NB], d4w (&Wj)[4][NB],
                                          const double* Fdi) {
  const double* Fd = Fdi + 64 * 40;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int n = 0; n < NB; ++n) Wj[jb][n] = (d4w){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int jb = 0; jb < KJ; ++jb)
#pragma unroll
    for (int kb = jb; kb < KJ; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = Fdi[64 * (4 * regs_tri(jb, kb) + s)];
#pragma unroll
        for (int n = 0; n < NB; ++n)
          Wj[jb][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ra[kb][n][s], Wj[jb][n], 0, 0, 0);
      }
#pragma unroll
  for (int jb = 0; jb < KJ; ++jb)
#pragma unroll
    for (int kb = jb; kb < KJ; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = Fd[64 * (4 * regs_tri(jb, kb) + s)];
#pragma unroll
        for (int n = 0; n < NB; ++n)
          Ra[jb][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wj[kb][n][s], Ra[jb][n], 0, 0, 0);
      }
#pragma unroll
  for (int jb = 0; jb < KJ; ++jb)
#pragma unroll
    for (int kb = jb; kb < KJ; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = Fdi[64 * (4 * regs_tri(jb, kb) + s)];
#pragma unroll
        for (int n = 0; n < NB; ++n)
          Wj[jb][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ra[kb][n][s], Wj[jb][n], 0, 0, 0);
      }
}

// Substitution with one refinement step for a super-block of at most 64 NJ
// columns (Alg. 3), every row independent, with W kept in registers in
// transposed form.  For the FP64 16x16x4 MFMA, lane l of an accumulator
// holds rows l/16 + 4q (q = 0..3) of column l%16 of a 16 x 16 block, which
// is exactly the B operand lane l supplies for the four K steps of the next
// product over that block.  So with W^T, R^T and T^T as 64 x (16 NB)
// column blocks (the columns are this wave's 16 NB rows of W), every
// product of the solve takes its B operand from registers and its A operand
// (from L_1 or D_J^{-1}, shared by all rows) from the fragments above:
//   R^T = L_2(:, J)^T - sum_{I > J} L_1(I, J)^T W^T(I)
//   W^T(J) = D_J^{-T} R^T,  T^T = R^T - D_J^T W^T(J),  W^T(J) += D_J^{-T} T^T
// for the column blocks J of the super-block from the last to the first
// (the later super-blocks' contribution is already in the right sides).
// No LDS, no barriers: each wave runs its own chain.  L may alias W (the
// right sides of a super-block are then W's own columns): a wave reads its
// rows of block J before it stores them.  With NJ = 4 the registers are
// capped at two waves per SIMD (256 per lane, no spills): the compiler's
// own choice, one wave per SIMD, ran the solve about 4 % slower on 200000
// rows.
template <typename TL, int NJ, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_trsm_regs(
    int64_t M, int64_t K, const TL* L, int64_t ldl, const double* __restrict__ F, double* W,
    int64_t ldw) {
  typedef RegsFrags<NJ> RF;
  const int lane = threadIdx.x & 63, l16 = lane & 15, lhi = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (16 * NB);
  if (r0 >= M) return;  // uniform per wave; no barrier follows
  int64_t roff[NB];
  bool rok[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    const int64_t r = r0 + 16 * n + l16;
    rok[n] = r < M;
    roff[n] = r < M ? r : M - 1;
  }
  F += lane;
  const int nblk = (int)((K + 63) >> 6);  // <= NJ
  // live 16-column tiles of the last block (every other block has four);
  // the products of that block run in a form specialised to them
  const int klast = (int)((K - 64 * (nblk - 1) + 15) >> 4);
  d4w Wt[NJ][4][NB];
  d4w Ra[4][NB];
#pragma unroll
  for (int JB = NJ - 1; JB >= 0; --JB) {
    if (JB >= nblk) continue;
    const int64_t j0 = 64 * JB;
    const int nbc = (int)min((int64_t)64, K - j0);
    // right sides R^T(j, r) = L(r, j0 + j)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 16 * kb + lhi + 4 * q;
          const double v = (double)L[roff[n] * ldl + j0 + min(j, nbc - 1)];
          Ra[kb][n][q] = j < nbc ? v : 0.0;
        }
    // the later blocks of the super-block
#pragma unroll
    for (int I = JB + 1; I < NJ; ++I) {
      if (I >= nblk) continue;
      const double* Fp = F + 64 * RF::pair(I, JB);
      if (I < nblk - 1) {
        regs_pair<4, NB>(Ra, Wt[I], Fp);
      } else {
        switch (klast) {
          case 1: regs_pair<1, NB>(Ra, Wt[I], Fp); break;
          case 2: regs_pair<2, NB>(Ra, Wt[I], Fp); break;
          case 3: regs_pair<3, NB>(Ra, Wt[I], Fp); break;
          default: regs_pair<4, NB>(Ra, Wt[I], Fp); break;
        }
      }
    }
    const double* Fdi = F + 64 * RF::diag(JB);
    if (JB < nblk - 1) {
      regs_diag<4, NB>(Ra, Wt[JB], Fdi);
    } else {
      switch (klast) {
        case 1: regs_diag<1, NB>(Ra, Wt[JB], Fdi); break;
        case 2: regs_diag<2, NB>(Ra, Wt[JB], Fdi); break;
        case 3: regs_diag<3, NB>(Ra, Wt[JB], Fdi); break;
        default: regs_diag<4, NB>(Ra, Wt[JB], Fdi); break;
      }
    }
    // W(r, j0 + j) = W^T(j, r)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 16 * kb + lhi + 4 * q;
          if (rok[n] && j < nbc) W[roff[n] * ldw + j0 + j] = Wt[JB][kb][n][q];
        }
  }
}

static size_t regs_frag_doubles(int64_t k) {
  return (size_t)ceil_div(k, kSuper) * RegsFrags<kRegsNJ>::kPerSb * 64;
}

static hipError_t launch_trsm_regs_frags(const double* L1, const double* Bt, int64_t k,
                                         double* F, hipStream_t s) {
  const dim3 g((unsigned)ceil_div((int64_t)RegsFrags<kRegsNJ>::kPerSb, (int64_t)4),
               (unsigned)ceil_div(k, kSuper));
  hipLaunchKernelGGL(k_trsm_regs_frags<kRegsNJ>, g, dim3(256), 0, s, L1, Bt, k, F);
  return hipGetLastError();
}

// Super-block a / kSuper of the solve: K <= kSuper columns, fragments from
// launch_trsm_regs_frags.
static hipError_t launch_trsm_regs(int64_t M, int64_t K, const void* L, int l_f32,
                                   int64_t ldl, const double* F, double* W, int64_t ldw,
                                   hipStream_t s) {
  if (M <= 0 || K <= 0) return hipSuccess;
  if (K > kSuper) return hipErrorInvalidValue;
  const dim3 g((unsigned)ceil_div(M, (int64_t)(64 * kRegsNB)));
  if (l_f32)
    hipLaunchKernelGGL((k_trsm_regs<float, kRegsNJ, kRegsNB>), g, dim3(256), 0, s, M, K,
                       (const float*)L, ldl, F, W, ldw);
  else
    hipLaunchKernelGGL((k_trsm_regs<double, kRegsNJ, kRegsNB>), g, dim3(256), 0, s, M, K,
                       (const double*)L, ldl, F, W, ldw);
  return hipGetLastError();
}

hipError_t launch_identity_rows(const int64_t* S, int64_t k, double* W, int64_t ldw,
                                hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_rows, dim3((unsigned)k), dim3(256), 0, s, S, k, W, ldw);
  return hipGetLastError();
}

size_t interp_workspace_doubles(int64_t m, int64_t k, int refine) {
  // L1 and Bt (k x k each); with refinement the solve's A fragments, and a
  // 64-column scratch per row for further refinement steps
  return (size_t)(2 * k * k) + (refine > 0 ? regs_frag_doubles(k) : 0) +
         (size_t)(refine > 1 ? round_up(m, 128) * 64 : 0);
}

hipError_t launch_interp(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t k,
                         const int64_t* S, double* W, int64_t ldw, int refine,
                         double* ws, hipStream_t s) {
  if (k <= 0 || m <= 0) return hipSuccess;
  double* L1 = ws;
  double* Bt = L1 + k * k;
  double* F = Bt + k * k;
  double* Tws = F + (refine > 0 ? regs_frag_doubles(k) : 0);
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
    // the super-block is then solved from R_s with its rows of W held in
    // registers (k_trsm_regs).  Further refinement steps run on the whole
    // result.
    e = launch_trsm_regs_frags(L1, Bt, k, F, s);
    if (e != hipSuccess) return e;
    const bool a_vec = ldw >= round_up(k, (int64_t)8);
    for (int64_t a = (ceil_div(k, kSuper) - 1) * kSuper; a >= 0 && e == hipSuccess; a -= kSuper) {
      const int64_t nbk = std::min<int64_t>(kSuper, k - a);
      const double* Fsb = F + (a / kSuper) * RegsFrags<kRegsNJ>::kPerSb * 64;
      if (a + nbk < k) {
        e = launch_gemm_tall(m, nbk, k - a - nbk, W + a + nbk, ldw, a_vec, L1 + (a + nbk) * k + a,
                             k, l_f64 ? (const void*)((const double*)L + a)
                                      : (const void*)((const float*)L + a),
                             lf32, ldl, W + a, ldw, s);
        if (e != hipSuccess) return e;
        e = launch_trsm_regs(m, nbk, W + a, 0, ldw, Fsb, W + a, ldw, s);
      } else {
        e = launch_trsm_regs(m, nbk, l_f64 ? (const void*)((const double*)L + a)
                                           : (const void*)((const float*)L + a),
                             lf32, ldl, Fsb, W + a, ldw, s);
      }
    }
    for (int it = 1; it < refine && e == hipSuccess; ++it)
      e = launch_trsm_refine_step(m, k, L, lf32, ldl, L1, Bt, W, ldw, Tws, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_identity_rows, dim3((unsigned)k), dim3(256), 0, s, S, k, W, ldw);
  return hipGetLastError();
}

}  // namespace rbrp
