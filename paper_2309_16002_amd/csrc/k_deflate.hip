// Fused deflation of one RBRP block (the O(m n b') part of Alg. 2):
//
//   P = R Q'                       (the new block of L, "L-hat = X Q'")
//   L[:, kS:kS+b'] = P             (rows of earlier skeletons set to zero)
//   R <- R - P Q'^T                (residual deflation)
//   d_i = ||R_i||^2                (FP64; zero on skeletons)
//
// R (m x n_pad, row-major) is the explicit residual X (I - Q Q^T); since Q'
// is orthogonal to the earlier basis, R Q' = X Q' and the recomputed norms
// equal the paper's downdated d in exact arithmetic, without its
// cancellation.
//
// Design (gfx950): one workgroup owns a panel of MP = 16 RT rows.  Its NW
// waves split the n_pad columns, CT column tiles of 16 each, and hold their
// slice of the panel in registers for the whole kernel, so R is read from
// HBM once and written once.  Phase 1 multiplies the register-resident slice
// by Q' with MFMA (partial P per wave), the partials are summed across waves
// in LDS in a fixed order, and phase 2 applies -P Q'^T with the same registers
// as the MFMA accumulator: the accumulator lane layout of a 16x16 output
// tile, read with the tile transposed (rows = R columns, columns = R rows),
// is exactly the A-operand layout phase 1 used, so no register shuffling is
// needed between the two products.  Q' comes pre-arranged in the per-lane
// fragment order of each product (built by k_make_frags).
//
// Modes: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32), and
// BF16 with FP32 accumulation (v_mfma_f32_16x16x32_bf16), either split into
// hi + lo parts (three products: hi*hi + hi*lo + lo*hi) or one product.
//
// Lane layouts (measured on gfx950): for all three instructions lane l
// supplies A[l%16][k(l)] and B[k(l)][l%16]; the 16x16 result is D[row][l%16]
// with row = 4(l/16) + q for the FP32-accumulating instructions and
// row = l/16 + 4q for the FP64 one (q = 0..3).
#include "rbrp_internal.h"

#include <math.h>

namespace rbrp {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <int MODE> struct DT;
template <> struct DT<kModeF64> { typedef double T; typedef d4v V; };
template <> struct DT<kModeF32> { typedef float T; typedef f4v V; };
template <> struct DT<kModeBF16x3> { typedef float T; typedef f4v V; };
template <> struct DT<kModeBF16> { typedef float T; typedef f4v V; };

// Output row (within a 16x16 tile) of accumulator slot q in lane l.
template <int MODE>
__device__ __forceinline__ int drow(int l, int q) {
  if constexpr (MODE == kModeF64) return (l >> 4) + 4 * q;
  else return 4 * (l >> 4) + q;
}

template <int MODE>
__device__ __forceinline__ typename DT<MODE>::V mfma4(typename DT<MODE>::T a,
                                                      typename DT<MODE>::T b,
                                                      typename DT<MODE>::V c) {
  if constexpr (MODE == kModeF64) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even BF16 split of 8 floats into hi and lo = x - hi.
__device__ __forceinline__ void split8(const float* x, bf8v& hi, bf8v& lo, bool need_lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)x[j];
    hi[j] = h;
    if (need_lo) lo[j] = (__bf16)(x[j] - (float)h);
  }
}

// Element offset of fragment buffers.
//   FP32/FP64: fragB1[g][bt][lane][4], fragA2[g][kb][lane][4]   (BT tiles of 16)
//   BF16:      fragB1[g/2][bt][lane][8] (hi, then lo buffer of the same size),
//              fragA2[g][ks][lane][8]   (ks: chunks of 32 b'-columns)

template <int MODE, int RT, int CT, int BT>
__global__ __launch_bounds__(512) void k_deflate(
    typename DT<MODE>::T* __restrict__ R, int64_t ldr, int64_t m, int nw,
    const void* __restrict__ fragB1, const void* __restrict__ fragA2,
    int64_t frag_stride, const int32_t* __restrict__ bprime_p,
    typename DT<MODE>::T* __restrict__ L, int64_t ldl, int64_t kS,
    const int32_t* __restrict__ sel_block, int32_t t, double* __restrict__ d,
    double* __restrict__ part_sum, double* __restrict__ part_max) {
  typedef typename DT<MODE>::T T;
  typedef typename DT<MODE>::V V;
  constexpr int MP = 16 * RT;
  constexpr bool BF = (MODE == kModeBF16x3 || MODE == kModeBF16);
  constexpr bool SPLIT = (MODE == kModeBF16x3);
  constexpr int SLOT = RT * BT * 64 * 4;  // accumulator elements per wave
  extern __shared__ __align__(16) unsigned char smem[];
  T* Ps = reinterpret_cast<T*>(smem);                          // nw * SLOT
  double* Ns = reinterpret_cast<double*>(smem + (size_t)nw * SLOT * sizeof(T));  // nw * MP

  const int bp = *bprime_p;
  if (bp <= 0) return;
  const int nbt = (bp + 15) >> 4;          // active 16-wide tiles of b'
  const int nks = (bp + 31) >> 5;          // active 32-wide chunks (BF16 phase 2)
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int l16 = lane & 15, lhi = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * MP;
  const int g0 = w * CT;                   // first global column tile of the wave

  // ---- load the panel slice ----
  V Rreg[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const T* rp = R + (r0 + 16 * rt + l16) * ldr;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int64_t c0 = 16 * (int64_t)(g0 + ct);
      if constexpr (MODE == kModeF64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Rreg[rt][ct][q] = rp[c0 + lhi + 4 * q];
      } else {
        Rreg[rt][ct] = *reinterpret_cast<const f4v*>(rp + c0 + 4 * lhi);
      }
    }
  }

  // ---- phase 1: partial P = R_slice Q'_slice ----
  V Pacc[RT][BT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
      for (int q = 0; q < 4; ++q) Pacc[rt][bt][q] = (T)0;

  if constexpr (!BF) {
    const V* fb = reinterpret_cast<const V*>(fragB1);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int bt = 0; bt < BT; ++bt) {
        if (bt < nbt) {
          const V bfr = fb[((int64_t)(g0 + ct) * BT + bt) * 64 + lane];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              Pacc[rt][bt] = mfma4<MODE>(Rreg[rt][ct][i], bfr[i], Pacc[rt][bt]);
        }
      }
    }
  } else {
    const bf8v* fbh = reinterpret_cast<const bf8v*>(fragB1);
    const bf8v* fbl = fbh + frag_stride;
#pragma unroll
    for (int c2 = 0; c2 < CT / 2; ++c2) {
      bf8v ah[RT], al[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        float x[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          x[j] = Rreg[rt][2 * c2][j];
          x[4 + j] = Rreg[rt][2 * c2 + 1][j];
        }
        split8(x, ah[rt], al[rt], SPLIT);
      }
      const int64_t gp = (g0 >> 1) + c2;
#pragma unroll
      for (int bt = 0; bt < BT; ++bt) {
        if (bt < nbt) {
          const int64_t o = (gp * BT + bt) * 64 + lane;
          const bf8v bh = fbh[o];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) Pacc[rt][bt] = mfma_bf16(ah[rt], bh, Pacc[rt][bt]);
          if constexpr (SPLIT) {
            const bf8v bl = fbl[o];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              Pacc[rt][bt] = mfma_bf16(ah[rt], bl, Pacc[rt][bt]);
              Pacc[rt][bt] = mfma_bf16(al[rt], bh, Pacc[rt][bt]);
            }
          }
        }
      }
    }
  }

  // ---- cross-wave reduction of P in LDS (fixed wave order) ----
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
      if (bt < nbt) {
        T* dst = Ps + (size_t)w * SLOT + ((rt * BT + bt) * 64 + lane) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = Pacc[rt][bt][q];
      }
  __syncthreads();
  {
    const int nel = RT * BT * 64 * 4;
    for (int e = threadIdx.x; e < nel; e += nw * 64) {
      const int q = e & 3;
      const int ln = (e >> 2) & 63;
      const int tb = e >> 8;               // rt * BT + bt
      const int bt = tb % BT, rt = tb / BT;
      if (bt >= nbt) continue;
      T s = Ps[e];
      for (int ww = 1; ww < nw; ++ww) s += Ps[(size_t)ww * SLOT + e];
      Ps[e] = s;
      const int row = 16 * rt + drow<MODE>(ln, q);
      const int bcol = 16 * bt + (ln & 15);
      const int64_t grow = r0 + row;
      if (grow < m && bcol < bp) {
        const int32_t sb = sel_block[grow];
        L[grow * ldl + kS + bcol] = (sb >= 0 && sb < t) ? (T)0 : s;
      }
    }
  }
  __syncthreads();

  // ---- phase 2: R <- R - P Q'^T on the register-resident slice ----
  // P fragment for phase 2: B[k][col] = -P[16 rt + col][k]; the reduced P sits
  // in slot 0 in phase-1 accumulator order.
  auto p_at = [&](int row, int bcol) -> T {
    const int rt = row >> 4, rr = row & 15;
    const int bt = bcol >> 4, bc = bcol & 15;
    int ln, q;
    if constexpr (MODE == kModeF64) { ln = 16 * (rr & 3) + bc; q = rr >> 2; }
    else { ln = 16 * (rr >> 2) + bc; q = rr & 3; }
    return Ps[((rt * BT + bt) * 64 + ln) * 4 + q];
  };

  if constexpr (!BF) {
    T Pf[RT][4 * BT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ks = 0; ks < 4 * BT; ++ks)
        Pf[rt][ks] = (ks < 4 * nbt) ? -p_at(16 * rt + l16, 4 * ks + lhi) : (T)0;
    const V* fa = reinterpret_cast<const V*>(fragA2);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int kb = 0; kb < BT; ++kb) {
        if (kb < nbt) {
          const V afr = fa[((int64_t)(g0 + ct) * BT + kb) * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              Rreg[rt][ct] = mfma4<MODE>(afr[j], Pf[rt][4 * kb + j], Rreg[rt][ct]);
        }
      }
    }
  } else {
    constexpr int KS = BT / 2;
    bf8v Ph[RT][KS], Pl[RT][KS];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int bcol = 32 * ks + 8 * lhi + j;
          x[j] = (ks < nks) ? -p_at(16 * rt + l16, bcol) : 0.0f;
        }
        split8(x, Ph[rt][ks], Pl[rt][ks], SPLIT);
      }
    const bf8v* fah = reinterpret_cast<const bf8v*>(fragA2);
    const bf8v* fal = fah + frag_stride;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks < nks) {
          const int64_t o = ((int64_t)(g0 + ct) * KS + ks) * 64 + lane;
          const bf8v ah = fah[o];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) Rreg[rt][ct] = mfma_bf16(ah, Ph[rt][ks], Rreg[rt][ct]);
          if constexpr (SPLIT) {
            const bf8v al = fal[o];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              Rreg[rt][ct] = mfma_bf16(ah, Pl[rt][ks], Rreg[rt][ct]);
              Rreg[rt][ct] = mfma_bf16(al, Ph[rt][ks], Rreg[rt][ct]);
            }
          }
        }
      }
    }
  }

  // ---- squared row norms (FP64) and store ----
  double nrm[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    double s = 0.0;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v = (double)Rreg[rt][ct][q];
        s += v * v;
      }
    s += __shfl_xor(s, 16, kWave);
    s += __shfl_xor(s, 32, kWave);
    nrm[rt] = s;
  }
  if (lane < 16) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) Ns[w * MP + 16 * rt + lane] = nrm[rt];
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    T* rp = R + (r0 + 16 * rt + l16) * ldr;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int64_t c0 = 16 * (int64_t)(g0 + ct);
      if constexpr (MODE == kModeF64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rp[c0 + lhi + 4 * q] = Rreg[rt][ct][q];
      } else {
        *reinterpret_cast<f4v*>(rp + c0 + 4 * lhi) = Rreg[rt][ct];
      }
    }
  }
  __syncthreads();
  if (w == 0) {
    double dv = 0.0;
    if (lane < MP) {
      double s = 0.0;
      for (int ww = 0; ww < nw; ++ww) s += Ns[ww * MP + lane];
      const int64_t row = r0 + lane;
      const bool skel = row >= m || sel_block[row] >= 0;
      dv = skel ? 0.0 : s;
      d[row] = dv;
    }
    double s = dv, mx = dv;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      s += __shfl_xor(s, off, kWave);
      mx = fmax(mx, __shfl_xor(mx, off, kWave));
    }
    if (lane == 0) {
      part_sum[blockIdx.x] = s;
      part_max[blockIdx.x] = mx;
    }
  }
}

// ---------------------------------------------------------------------------
// Fragment builder: Q' = Qt_new^T (FP64, b' rows of n_pad) into the per-lane
// operand order of both products.
template <int MODE>
__global__ __launch_bounds__(256) void k_make_frags(const double* __restrict__ Qt,
                                                    int64_t ldq,
                                                    const int32_t* __restrict__ bprime,
                                                    int64_t G, int BT, void* fragB1,
                                                    void* fragA2, int64_t frag_stride) {
  const int bp = *bprime;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  auto q_at = [&](int64_t c, int bcol) -> double {
    return bcol < bp ? Qt[(int64_t)bcol * ldq + c] : 0.0;
  };
  if constexpr (MODE == kModeF64 || MODE == kModeF32) {
    typedef typename DT<MODE>::T T;
    // e indexes (g, bt, lane, i) for both buffers
    const int64_t total = G * BT * 64 * 4;
    if (e >= total) return;
    const int i = e & 3;
    const int lane = (e >> 2) & 63;
    const int64_t gb = e >> 8;
    const int bt = (int)(gb % BT);
    const int64_t g = gb / BT;
    const int l16 = lane & 15, lhi = lane >> 4;
    const int dr = (MODE == kModeF64) ? (lhi + 4 * i) : (4 * lhi + i);
    reinterpret_cast<T*>(fragB1)[e] = (T)q_at(16 * g + dr, 16 * bt + l16);
    reinterpret_cast<T*>(fragA2)[e] = (T)q_at(16 * g + l16, 16 * bt + 4 * i + lhi);
  } else {
    // fragB1: (g2, bt, lane, j) with G/2 column-tile pairs; fragA2: (g, ks, lane, j)
    const int j = e & 7;
    const int lane = (e >> 3) & 63;
    const int l16 = lane & 15, lhi = lane >> 4;
    const int64_t totB = (G / 2) * BT * 64 * 8;
    if (e < totB) {
      const int64_t gb = e >> 9;
      const int bt = (int)(gb % BT);
      const int64_t g2 = gb / BT;
      const int64_t c = 32 * g2 + (j < 4 ? 4 * lhi + j : 16 + 4 * lhi + (j - 4));
      const float x = (float)q_at(c, 16 * bt + l16);
      const __bf16 h = (__bf16)x;
      reinterpret_cast<__bf16*>(fragB1)[e] = h;
      reinterpret_cast<__bf16*>(fragB1)[frag_stride * 8 + e] = (__bf16)(x - (float)h);
    }
    const int KS = BT / 2;
    const int64_t totA = G * KS * 64 * 8;
    if (e < totA) {
      const int64_t gk = e >> 9;
      const int ks = (int)(gk % KS);
      const int64_t g = gk / KS;
      const float x = (float)q_at(16 * g + l16, 32 * ks + 8 * lhi + j);
      const __bf16 h = (__bf16)x;
      reinterpret_cast<__bf16*>(fragA2)[e] = h;
      reinterpret_cast<__bf16*>(fragA2)[frag_stride * 8 + e] = (__bf16)(x - (float)h);
    }
  }
}

// ---------------------------------------------------------------------------
// Configuration: n_pad = 16 * CT * nw with CT in {2,4,8,16,32}, nw in [1,8].

struct DeflateCfg {
  int ct, rt, nw;
};

static bool pick_cfg(int mode, int64_t ldr, DeflateCfg* c) {
  const int cts[5] = {2, 4, 8, 16, 32};
  for (int i = 0; i < 5; ++i) {
    const int ct = cts[i];
    if (ldr % (16 * ct)) continue;
    const int64_t nw = ldr / (16 * ct);
    if (nw < 1 || nw > 8) continue;
    if (mode == kModeF64 && ct > 16) return false;
    c->ct = ct;
    c->nw = (int)nw;
    c->rt = (ct >= 32 || (mode == kModeF64 && ct >= 16)) ? 1 : 2;
    return true;
  }
  return false;
}

int64_t deflate_pad_cols(int64_t n) {
  // smallest 16*CT*nw >= n over the supported shapes (ties: fewer waves)
  int64_t best = -1;
  const int cts[5] = {2, 4, 8, 16, 32};
  for (int i = 0; i < 5; ++i)
    for (int nw = 1; nw <= 8; ++nw) {
      const int64_t v = 16LL * cts[i] * nw;
      if (v >= n && (best < 0 || v < best)) best = v;
    }
  return best;
}

static int bt_for(int mode, int bmax) {
  int bt = 1;
  while (16 * bt < bmax) bt <<= 1;
  if ((mode == kModeBF16x3 || mode == kModeBF16) && bt < 2) bt = 2;
  return bt;
}

int deflate_supported(int mode, int64_t ldr, int bmax) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return 0;
  return bmax >= 1 && bmax <= kMaxB;
}

int deflate_rows_per_wg(int mode, int64_t ldr) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return 0;
  return 16 * c.rt;
}

int64_t deflate_num_partials(int64_t mr) { return ceil_div(mr, 16); }

int64_t frag_elems(int mode, int64_t ldr, int bmax) {
  // elements (T for FP32/FP64; bf16 for BF16, per hi/lo half) of one buffer
  const int bt = bt_for(mode, bmax);
  const int64_t G = ldr / 16;
  return G * bt * 64 * 4 * ((mode == kModeBF16x3 || mode == kModeBF16) ? 1 : 1);
}

template <int MODE, int RT, int CT, int BT>
static hipError_t run_deflate(const DeflateCfg& c, int64_t grid, hipStream_t s,
                              void* R, int64_t ldr, int64_t m, const void* fB,
                              const void* fA, int64_t fstride, const int32_t* bp,
                              void* L, int64_t ldl, int64_t kS, const int32_t* sel,
                              int32_t t, double* d, double* ps, double* pm) {
  typedef typename DT<MODE>::T T;
  const size_t slot = (size_t)RT * BT * 64 * 4 * sizeof(T);
  const size_t lds = c.nw * slot + (size_t)c.nw * 16 * RT * sizeof(double);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_deflate<MODE, RT, CT, BT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_deflate<MODE, RT, CT, BT>), dim3((unsigned)grid),
                     dim3(64 * c.nw), lds, s, (T*)R, ldr, m, c.nw, fB, fA, fstride,
                     bp, (T*)L, ldl, kS, sel, t, d, ps, pm);
  return hipGetLastError();
}

template <int MODE, int BT>
static hipError_t dispatch_ct(const DeflateCfg& c, int64_t mr, hipStream_t s, void* R,
                              int64_t ldr, int64_t m, const void* fB, const void* fA,
                              int64_t fstride, const int32_t* bp, void* L, int64_t ldl,
                              int64_t kS, const int32_t* sel, int32_t t, double* d,
                              double* ps, double* pm) {
#define RBRP_DEF_CASE(CTV, RTV)                                                        \
  if (c.ct == CTV && c.rt == RTV)                                                      \
    return run_deflate<MODE, RTV, CTV, BT>(c, mr / (16 * RTV), s, R, ldr, m, fB, fA,   \
                                           fstride, bp, L, ldl, kS, sel, t, d, ps, pm);
  if constexpr (MODE == kModeF64) {
    RBRP_DEF_CASE(2, 2)
    RBRP_DEF_CASE(4, 2)
    RBRP_DEF_CASE(8, 2)
    RBRP_DEF_CASE(16, 1)
  } else {
    RBRP_DEF_CASE(2, 2)
    RBRP_DEF_CASE(4, 2)
    RBRP_DEF_CASE(8, 2)
    RBRP_DEF_CASE(16, 2)
    RBRP_DEF_CASE(32, 1)
  }
#undef RBRP_DEF_CASE
  return hipErrorInvalidConfiguration;
}

template <int MODE>
static hipError_t dispatch_bt(int bt, const DeflateCfg& c, int64_t mr, hipStream_t s,
                              void* R, int64_t ldr, int64_t m, const void* fB,
                              const void* fA, int64_t fstride, const int32_t* bp,
                              void* L, int64_t ldl, int64_t kS, const int32_t* sel,
                              int32_t t, double* d, double* ps, double* pm) {
  switch (bt) {
    case 1:
      if constexpr (MODE == kModeF64 || MODE == kModeF32)
        return dispatch_ct<MODE, 1>(c, mr, s, R, ldr, m, fB, fA, fstride, bp, L, ldl, kS,
                                    sel, t, d, ps, pm);
      break;
    case 2:
      return dispatch_ct<MODE, 2>(c, mr, s, R, ldr, m, fB, fA, fstride, bp, L, ldl, kS, sel,
                                  t, d, ps, pm);
    case 4:
      return dispatch_ct<MODE, 4>(c, mr, s, R, ldr, m, fB, fA, fstride, bp, L, ldl, kS, sel,
                                  t, d, ps, pm);
    case 8:
      return dispatch_ct<MODE, 8>(c, mr, s, R, ldr, m, fB, fA, fstride, bp, L, ldl, kS, sel,
                                  t, d, ps, pm);
  }
  return hipErrorInvalidConfiguration;
}

hipError_t launch_deflate(int mode, void* R, int64_t mr, int64_t ldr, int64_t m,
                          const void* fragB1, const void* fragA2,
                          const int32_t* bprime, int bmax, void* L, int64_t ldl,
                          int64_t kS, const int32_t* sel_block, int32_t t, double* d,
                          double* part_sum, double* part_max, hipStream_t s) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return hipErrorInvalidConfiguration;
  if (mr % (16 * c.rt)) return hipErrorInvalidValue;
  const int bt = bt_for(mode, bmax);
  const int64_t fstride = frag_elems(mode, ldr, bmax) / ((mode == kModeBF16x3 || mode == kModeBF16) ? 8 : 4);
  switch (mode) {
    case kModeF64:
      return dispatch_bt<kModeF64>(bt, c, mr, s, R, ldr, m, fragB1, fragA2, fstride, bprime,
                                   L, ldl, kS, sel_block, t, d, part_sum, part_max);
    case kModeF32:
      return dispatch_bt<kModeF32>(bt, c, mr, s, R, ldr, m, fragB1, fragA2, fstride, bprime,
                                   L, ldl, kS, sel_block, t, d, part_sum, part_max);
    case kModeBF16x3:
      return dispatch_bt<kModeBF16x3>(bt, c, mr, s, R, ldr, m, fragB1, fragA2, fstride,
                                      bprime, L, ldl, kS, sel_block, t, d, part_sum, part_max);
    case kModeBF16:
      return dispatch_bt<kModeBF16>(bt, c, mr, s, R, ldr, m, fragB1, fragA2, fstride, bprime,
                                    L, ldl, kS, sel_block, t, d, part_sum, part_max);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_make_frags(const double* Qt_new, int64_t ldq, const int32_t* bprime,
                             int64_t n_pad, int bmax, int mode, void* fragB1,
                             void* fragA2, hipStream_t s) {
  const int bt = bt_for(mode, bmax);
  const int64_t G = n_pad / 16;
  const bool bf = (mode == kModeBF16x3 || mode == kModeBF16);
  const int64_t total = bf ? G * bt * 64 * 4 : G * bt * 64 * 4;
  // BF16: (G/2)*bt*64*8 = G*bt*256 elements (B) and G*(bt/2)*64*8 (A): same count
  const int64_t fstride = bf ? total / 8 : total / 4;
  const unsigned grid = (unsigned)ceil_div(total, 256);
  switch (mode) {
    case kModeF64:
      hipLaunchKernelGGL(k_make_frags<kModeF64>, dim3(grid), dim3(256), 0, s, Qt_new, ldq,
                         bprime, G, bt, fragB1, fragA2, fstride);
      break;
    case kModeF32:
      hipLaunchKernelGGL(k_make_frags<kModeF32>, dim3(grid), dim3(256), 0, s, Qt_new, ldq,
                         bprime, G, bt, fragB1, fragA2, fstride);
      break;
    case kModeBF16x3:
    case kModeBF16:
      hipLaunchKernelGGL(k_make_frags<kModeBF16x3>, dim3(grid), dim3(256), 0, s, Qt_new,
                         ldq, bprime, G, bt, fragB1, fragA2, fstride);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Bytes of one fragment buffer (fragB1 or fragA2), hi+lo halves included.
size_t frag_bytes(int mode, int64_t ldr, int bmax) {
  const int bt = bt_for(mode, bmax);
  const int64_t G = ldr / 16;
  const int64_t elems = G * bt * 64 * 4;  // T elements, or bf16 elements per half
  switch (mode) {
    case kModeF64: return (size_t)elems * 8;
    case kModeF32: return (size_t)elems * 4;
    default: return (size_t)elems * 2 * 2;
  }
}

}  // namespace rbrp
