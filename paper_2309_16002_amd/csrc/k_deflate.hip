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
// row = l/16 + 4q for the FP64 one (q = 0..3).  In phase 2 the result rows
// are columns of R; they are assigned so that lane l's slot q always holds
// column 4(l/16) + q of the 16-column tile (for FP64, tile row r holds column
// pi(r) = 4 (r % 4) + r / 4), which makes every lane's four values contiguous
// in memory.
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
//
// Per-wave partial P tiles in LDS: tile t (= rt * BT + bt) of 16 x 16, stored
// in accumulator order (lane, slot) with 4 floats of padding after each group
// of 16 lanes, so that the transposed gathers of phase 2 hit distinct banks.
constexpr int kLaneGroup = 68;            // 16 lanes x 4 slots + 4 padding
constexpr int kTileElems = 4 * kLaneGroup;

__device__ __forceinline__ int slot_off(int tile, int ln, int q) {
  return tile * kTileElems + (ln >> 4) * kLaneGroup + (ln & 15) * 4 + q;
}

// Loads are issued in the order they are consumed (R chunk ct, then its Q'
// fragments), kDepth chunks ahead, so that phase-1 MFMAs start as soon as the
// first chunk arrives while the rest of the panel streams in; phase 2 streams
// the updated R back out chunk by chunk.  NB, the number of active 16-wide
// b' tiles, is a compile-time constant of each instantiated body.
constexpr int kDepth = 3;   // default prefetch depth (chunks of 16 columns)

// Scheduling fence: keeps the loads issued for later chunks ahead of the
// MFMAs that follow (the compiler's scheduler would otherwise sink them next
// to their first use, leaving about one chunk in flight instead of DEPTH).
// Holding DEPTH chunks really in flight costs registers, so a body is fenced
// only when its estimated footprint (the R slice, the prefetch ring and the
// P accumulators, in VGPRs) fits the 256 of two waves per SIMD and at most
// four b' tiles are active (wider bodies need the registers for phase 2);
// the others keep the compiler's schedule rather than spill.
template <int MODE, int RT, int CT, int NB, int DEPTH, int REGS = 256>
constexpr bool fence_fits() {
  constexpr bool bf = (MODE == kModeBF16x3 || MODE == kModeBF16);
  constexpr int s = (MODE == kModeF64) ? 2 : 1;
  constexpr int r = RT * CT * 4 * s;
  constexpr int ring = bf ? DEPTH * (2 * RT * 4 + NB * 4 * (MODE == kModeBF16x3 ? 2 : 1))
                          : DEPTH * (RT * 4 * s + NB * 4 * s);
  constexpr int pacc = RT * NB * 4 * s;
  return (NB <= 4 || REGS > 256) && r + ring + pacc <= REGS - 40 * (REGS > 256);
}

template <bool ON>
__device__ __forceinline__ void sched_fence() {
  if constexpr (ON) __builtin_amdgcn_sched_barrier(0);
}

// Storage of the residual in a BF16-product launch (RIO): 0 R in its own
// type in and out; 1 FP32 in, BF16 out (the block that switches the storage);
// 2 BF16 in and out.  BF16 R is kept in a column order permuted inside each
// group of 32 columns: storage position 8 h + 4 p + j holds column
// 16 p + 4 h + j (h = 0..3, p = 0..1, j = 0..3), so that the 16 bytes at
// position 8 h of a row are the 8 values lane (16 h + row) feeds the BF16
// MFMA in phase 1 and holds in its two accumulators in phase 2.
// A BF16-stored residual (RIO 2) is read residual first: the packed slice is
// requested whole before any fragment beyond the first few steps (the loads
// land in the registers that hold it anyway, so only the fragments need a
// ring, kRFDepth steps deep; vector-memory counters retire in issue order,
// so without this each step's wait would also cover the residual loads
// issued beside its fragments, and the compiler's own schedule of the
// eight-tile body kept about one load in flight).  The packed values are
// phase 1's A operand as they are; phase 2 widens them to FP32 pair by
// pair.  Phase 1 runs over the b' tiles in passes of at most four, so that
// a pass's P accumulators and fragment ring stay small.  Measured on
// 200000 x 2048 with b' = 128: 0.727 -> 0.677 ms per launch, with results
// identical bit for bit (the products accumulate in the same order).
// (The same order for an FP32 residual, read into its FP32 registers,
// spilled the eight-tile bodies and was slower.)
constexpr int kRFDepth = 4;

// LOADR: phase 1 reads the panel's residual from memory (otherwise it is
// already in Rreg: the second half of a block wider than 128 columns);
// STORER: phase 2 writes it back and forms the row norms (otherwise it stays
// in Rreg for the second half).
template <int MODE, int RT, int CT, int BT, int NB, int DEPTH0, int RIO = 0, int REGS = 256,
          bool LOADR = true, bool STORER = true>
__device__ __forceinline__ void deflate_body(
    typename DT<MODE>::V (&Rreg)[RT][CT],
    typename DT<MODE>::T* __restrict__ Rw, uint16_t* __restrict__ R16w, uint32_t ldr32,
    int64_t m, int nw, int w, int lane,
    const void* __restrict__ fragB1, const void* __restrict__ fragA2, int64_t frag_stride,
    int g0, int bp, typename DT<MODE>::T* __restrict__ Lp, uint32_t ldl32, int32_t t,
    const int32_t* __restrict__ sb_s, typename DT<MODE>::T* __restrict__ Ps,
    double* __restrict__ Ns, int64_t r0, double* __restrict__ d,
    double* __restrict__ part_sum, double* __restrict__ part_max) {
  typedef typename DT<MODE>::T T;
  typedef typename DT<MODE>::V V;
  constexpr int MP = 16 * RT;
  constexpr bool BF = (MODE == kModeBF16x3 || MODE == kModeBF16);
  constexpr bool SPLIT = (MODE == kModeBF16x3);
  constexpr int SLOT = RT * BT * kTileElems;
  // Wide bodies (more than four b' tiles) of single-row-tile panels hold two
  // chunks really in flight (measured 12-16% faster for FP32 and split BF16
  // than DEPTH0 chunks under the compiler's own schedule on 200000 x 2048,
  // despite a few spilled registers); with two row tiles the spills cost
  // more than the prefetch gains (measured), and FP64 keeps its schedule.
  constexpr bool WIDE = NB > 4 && RT == 1 && MODE != kModeF64;
  constexpr int DEPTH = WIDE ? 2 : DEPTH0;
  constexpr bool FENCE = WIDE || fence_fits<MODE, RT, CT, NB, DEPTH0, REGS>();
  const int l16 = lane & 15, lhi = lane >> 4;
  constexpr bool RF = BF && RIO == 2 && LOADR;

  // packed BF16 residual of the residual-first BF16-stored body
  uint4 raw[RT][RF ? CT / 2 : 1];
  V Pacc[RT][NB];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int bt = 0; bt < NB; ++bt)
#pragma unroll
      for (int q = 0; q < 4; ++q) Pacc[rt][bt][q] = (T)0;

  auto load_r = [&](int ct) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      Rreg[rt][ct] = *reinterpret_cast<const V*>(Rw + (uint32_t)(16 * rt + l16) * ldr32 +
                                                 16 * ct + 4 * lhi);
  };
  // chunks 2 c2 and 2 c2 + 1 (one 32-column group)
  auto load_pair = [&](int c2) {
    load_r(2 * c2);
    load_r(2 * c2 + 1);
  };

  // ---- phase 1: partial P = R_slice Q'_slice, R streamed in ----
  if constexpr (!BF) {
    const V* fb = reinterpret_cast<const V*>(fragB1) + (int64_t)g0 * BT * 64;
    V fr[DEPTH][NB];
#pragma unroll
    for (int k = 0; k < DEPTH; ++k) {
      if (k < CT) {
        if constexpr (LOADR) load_r(k);
#pragma unroll
        for (int bt = 0; bt < NB; ++bt) fr[k][bt] = fb[(uint32_t)((k * BT + bt) * 64) + lane];
      }
    }
    sched_fence<FENCE>();
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int sl = ct % DEPTH;
#pragma unroll
      for (int bt = 0; bt < NB; ++bt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            Pacc[rt][bt] = mfma4<MODE>(Rreg[rt][ct][i], fr[sl][bt][i], Pacc[rt][bt]);
      if (ct + DEPTH < CT) {
        if constexpr (LOADR) load_r(ct + DEPTH);
#pragma unroll
        for (int bt = 0; bt < NB; ++bt)
          fr[sl][bt] = fb[(uint32_t)(((ct + DEPTH) * BT + bt) * 64) + lane];
      }
      sched_fence<FENCE>();
    }
  } else if constexpr (RF) {
    constexpr int C2 = CT / 2;
    constexpr int G = NB <= 4 ? NB : 4;                  // b' tiles per pass
    constexpr int NP = NB / G;
    constexpr int NS = NP * C2;                          // steps of all passes
    constexpr int DF = kRFDepth;
    static_assert(!SPLIT, "a BF16-stored residual is deflated with one BF16 product");
    const bf8v* fbh = reinterpret_cast<const bf8v*>(fragB1) + (int64_t)(g0 >> 1) * BT * 64;
    bf8v frh[DF][G];
    auto load_frags = [&](int slot, int st) {
      const int c2 = st % C2, p = st / C2;
#pragma unroll
      for (int g = 0; g < G; ++g)
        frh[slot][g] = fbh[(uint32_t)((c2 * BT + p * G + g) * 64) + lane];
    };
#pragma unroll
    for (int k = 0; k < DF; ++k)
      if (k < NS) load_frags(k, k);
#pragma unroll
    for (int c2 = 0; c2 < C2; ++c2)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        raw[rt][c2] = *reinterpret_cast<const uint4*>(R16w + (uint32_t)(16 * rt + l16) * ldr32 +
                                                      32 * c2 + 8 * lhi);
    sched_fence<true>();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      V Pg[RT][G];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int q = 0; q < 4; ++q) Pg[rt][g][q] = 0.0f;
#pragma unroll
      for (int c2 = 0; c2 < C2; ++c2) {
        const int st = p * C2 + c2;
        const int sl = st % DF;
        bf8v ah[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) ah[rt] = __builtin_bit_cast(bf8v, raw[rt][c2]);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) Pg[rt][g] = mfma_bf16(ah[rt], frh[sl][g], Pg[rt][g]);
        if (st + DF < NS) load_frags(sl, st + DF);
        sched_fence<true>();
      }
      // this pass's partial tiles to the wave's LDS slot
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int g = 0; g < G; ++g) {
          T* dst = Ps + (size_t)w * SLOT + slot_off(rt * BT + p * G + g, lane, 0);
#pragma unroll
          for (int q = 0; q < 4; ++q) dst[q] = Pg[rt][g][q];
        }
    }
  } else {
    constexpr int C2 = CT / 2;
    const bf8v* fbh = reinterpret_cast<const bf8v*>(fragB1) + (int64_t)(g0 >> 1) * BT * 64;
    const bf8v* fbl = fbh + frag_stride;
    bf8v frh[DEPTH][NB], frl[DEPTH][NB];
#pragma unroll
    for (int k = 0; k < DEPTH; ++k) {
      if (k < C2) {
        if constexpr (LOADR) load_pair(k);
#pragma unroll
        for (int bt = 0; bt < NB; ++bt) {
          const uint32_t o = (uint32_t)((k * BT + bt) * 64) + lane;
          frh[k][bt] = fbh[o];
          if constexpr (SPLIT) frl[k][bt] = fbl[o];
        }
      }
    }
    sched_fence<FENCE>();
#pragma unroll
    for (int c2 = 0; c2 < C2; ++c2) {
      const int sl = c2 % DEPTH;
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
#pragma unroll
      for (int bt = 0; bt < NB; ++bt) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) Pacc[rt][bt] = mfma_bf16(ah[rt], frh[sl][bt], Pacc[rt][bt]);
        if constexpr (SPLIT) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            Pacc[rt][bt] = mfma_bf16(ah[rt], frl[sl][bt], Pacc[rt][bt]);
            Pacc[rt][bt] = mfma_bf16(al[rt], frh[sl][bt], Pacc[rt][bt]);
          }
        }
      }
      if (c2 + DEPTH < C2) {
        if constexpr (LOADR) load_pair(c2 + DEPTH);
#pragma unroll
        for (int bt = 0; bt < NB; ++bt) {
          const uint32_t o = (uint32_t)(((c2 + DEPTH) * BT + bt) * 64) + lane;
          frh[sl][bt] = fbh[o];
          if constexpr (SPLIT) frl[sl][bt] = fbl[o];
        }
      }
      sched_fence<FENCE>();
    }
  }

  // ---- cross-wave reduction of P in LDS (fixed wave order), L written ----
  if constexpr (!RF) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int bt = 0; bt < NB; ++bt) {
        T* dst = Ps + (size_t)w * SLOT + slot_off(rt * BT + bt, lane, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = Pacc[rt][bt][q];
      }
  }
  __syncthreads();
  {
    const int nel = RT * NB * 256;
    for (int e = threadIdx.x; e < nel; e += nw * 64) {
      const int q = e & 3;
      const int ln = (e >> 2) & 63;
      const int tb = e >> 8;                   // rt * NB + bt
      const int bt = tb % NB, rt = tb / NB;
      const int off = slot_off(rt * BT + bt, ln, q);
      T s = Ps[off];
      for (int ww = 1; ww < nw; ++ww) s += Ps[(size_t)ww * SLOT + off];
      Ps[off] = s;
      const int row = 16 * rt + drow<MODE>(ln, q);
      const int bcol = 16 * bt + (ln & 15);
      if (r0 + row < m && bcol < bp) {
        const int32_t sb = sb_s[row];
        Lp[(uint32_t)row * ldl32 + (uint32_t)bcol] = (sb >= 0 && sb < t) ? (T)0 : s;
      }
    }
  }
  __syncthreads();

  // reduced P in slot 0, accumulator order of phase 1
  auto p_at = [&](int row, int bcol) -> T {
    const int rt = row >> 4, rr = row & 15;
    const int bt = bcol >> 4, bc = bcol & 15;
    int ln, q;
    if constexpr (MODE == kModeF64) { ln = 16 * (rr & 3) + bc; q = rr >> 2; }
    else { ln = 16 * (rr >> 2) + bc; q = rr & 3; }
    return Ps[slot_off(rt * BT + bt, ln, q)];
  };

  // ---- phase 2: R <- R - P Q'^T, stored chunk by chunk; row norms in FP64 ----
  double nrm[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) nrm[rt] = 0.0;
  auto finish_chunk = [&](int ct) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v = (double)Rreg[rt][ct][q];
        nrm[rt] += v * v;
      }
      *reinterpret_cast<V*>(Rw + (uint32_t)(16 * rt + l16) * ldr32 + 16 * ct + 4 * lhi) =
          Rreg[rt][ct];
    }
  };
  // BF16 storage: chunks 2 c2 and 2 c2 + 1 rounded to nearest even and
  // stored as one 16-byte group; the norms are those of the stored values
  auto finish_pair16 = [&](int c2) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      uint32_t wv[4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const __bf16 a = (__bf16)Rreg[rt][2 * c2 + h][2 * jj];
          const __bf16 b = (__bf16)Rreg[rt][2 * c2 + h][2 * jj + 1];
          const double va = (double)(float)a, vb = (double)(float)b;
          nrm[rt] += va * va + vb * vb;
          wv[2 * h + jj] = (uint32_t)__builtin_bit_cast(uint16_t, a) |
                           ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
        }
      *reinterpret_cast<uint4*>(R16w + (uint32_t)(16 * rt + l16) * ldr32 + 32 * c2 + 8 * lhi) =
          make_uint4(wv[0], wv[1], wv[2], wv[3]);
    }
  };
  if constexpr (!BF) {
    T Pf[RT][4 * NB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ks = 0; ks < 4 * NB; ++ks) Pf[rt][ks] = -p_at(16 * rt + l16, 4 * ks + lhi);
    const V* fa = reinterpret_cast<const V*>(fragA2) + (int64_t)g0 * BT * 64;
    // Chunks are updated in pairs so that 2 RT independent accumulator chains
    // interleave (one chunk alone gives RT chains of 4 NB dependent MFMAs);
    // the fragments of the next pair are in flight during the current pair.
    constexpr int PW = (CT % 2 == 0) ? 2 : 1;
    V fr[2 * PW][NB];
#pragma unroll
    for (int k = 0; k < 2 * PW; ++k)
      if (k < CT) {
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) fr[k][kb] = fa[(uint32_t)((k * BT + kb) * 64) + lane];
      }
#pragma unroll
    for (int c0 = 0; c0 < CT; c0 += PW) {
      const int sl = (c0 / PW) & 1;
#pragma unroll
      for (int kb = 0; kb < NB; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int p = 0; p < PW; ++p)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              Rreg[rt][c0 + p] = mfma4<MODE>(fr[sl * PW + p][kb][j], Pf[rt][4 * kb + j],
                                             Rreg[rt][c0 + p]);
#pragma unroll
      for (int p = 0; p < PW; ++p)
        if (c0 + p + 2 * PW < CT) {
#pragma unroll
          for (int kb = 0; kb < NB; ++kb)
            fr[sl * PW + p][kb] = fa[(uint32_t)(((c0 + p + 2 * PW) * BT + kb) * 64) + lane];
        }
      sched_fence<FENCE>();
#pragma unroll
      for (int p = 0; p < PW; ++p)
        if constexpr (STORER) finish_chunk(c0 + p);
    }
  } else {
    constexpr int KS = BT / 2;               // fragment chunks of 32 in the buffer
    constexpr int NK = (NB + 1) / 2;         // active chunks of 32
    bf8v Ph[RT][NK], Pl[RT][NK];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ks = 0; ks < NK; ++ks) {
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int bcol = 32 * ks + 8 * lhi + j;
          x[j] = (bcol < 16 * NB) ? -p_at(16 * rt + l16, bcol) : 0.0f;
        }
        split8(x, Ph[rt][ks], Pl[rt][ks], SPLIT);
      }
    const bf8v* fah = reinterpret_cast<const bf8v*>(fragA2) + (int64_t)g0 * KS * 64;
    const bf8v* fal = fah + frag_stride;
    bf8v frh[2][NK], frl[2][NK];
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (k < CT) {
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
          const uint32_t o = (uint32_t)((k * KS + ks) * 64) + lane;
          frh[k][ks] = fah[o];
          if constexpr (SPLIT) frl[k][ks] = fal[o];
        }
      }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int sl = ct & 1;
      if constexpr (RF) {
        if ((ct & 1) == 0) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const uint4 u = raw[rt][ct >> 1];
            const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t x = wv[j >> 1], y = wv[2 + (j >> 1)];
              Rreg[rt][ct][j] = __uint_as_float((j & 1) ? (x & 0xFFFF0000u) : (x << 16));
              Rreg[rt][ct + 1][j] = __uint_as_float((j & 1) ? (y & 0xFFFF0000u) : (y << 16));
            }
          }
        }
      }
#pragma unroll
      for (int ks = 0; ks < NK; ++ks) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) Rreg[rt][ct] = mfma_bf16(frh[sl][ks], Ph[rt][ks], Rreg[rt][ct]);
        if constexpr (SPLIT) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            Rreg[rt][ct] = mfma_bf16(frh[sl][ks], Pl[rt][ks], Rreg[rt][ct]);
            Rreg[rt][ct] = mfma_bf16(frl[sl][ks], Ph[rt][ks], Rreg[rt][ct]);
          }
        }
      }
      if (ct + 2 < CT) {
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
          const uint32_t o = (uint32_t)(((ct + 2) * KS + ks) * 64) + lane;
          frh[sl][ks] = fah[o];
          if constexpr (SPLIT) frl[sl][ks] = fal[o];
        }
      }
      sched_fence<FENCE>();
      if constexpr (STORER) {
        if constexpr (RIO == 0) finish_chunk(ct);
        else if (ct & 1) finish_pair16(ct >> 1);
      }
    }
  }

  // ---- squared row norms: lanes of one row, then waves in order ----
  if constexpr (!STORER) return;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    double s = nrm[rt];
    s += __shfl_xor(s, 16, kWave);
    s += __shfl_xor(s, 32, kWave);
    nrm[rt] = s;
  }
  if (lane < 16) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) Ns[w * MP + 16 * rt + lane] = nrm[rt];
  }
  __syncthreads();
  if (w == 0) {
    double dv = 0.0;
    if (lane < MP) {
      double s = 0.0;
      for (int ww = 0; ww < nw; ++ww) s += Ns[ww * MP + lane];
      const int64_t row = r0 + lane;
      const bool skel = row >= m || sb_s[lane] >= 0;
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

// Blocks wider than 128 kept columns come as two halves (bprime_p and
// bprime2_p, with their own fragments): the second half's products run on
// the residual still in registers (since Q2 is orthogonal to Q1, the
// updated residual times Q2 equals R Q2), so R is read and written once per
// block.  The kernels of 128-column blocks (BT = 8) with one BF16 product
// carry that path, the memory-bound ones where the second pass over R
// costs most; with FP32 or split products (bound by their MFMA work at 128
// columns) the longer kernel spilled registers, so they take one launch per
// half.
template <int MODE, int BT>
constexpr bool deflate_fuses() {
  return BT == 8 && MODE == kModeBF16;
}

template <int MODE, int RT, int CT, int BT, int NWMAX, int DEPTH = kDepth, int RIO = 0,
          int WPE = 2>
__global__ __launch_bounds__(64 * NWMAX) __attribute__((amdgpu_waves_per_eu(WPE))) void k_deflate(
    typename DT<MODE>::T* __restrict__ R, uint16_t* __restrict__ R16, int64_t ldr, int64_t m,
    int nw,
    const void* __restrict__ fragB1, const void* __restrict__ fragA2,
    int64_t frag_stride, const int32_t* __restrict__ bprime_p,
    const void* __restrict__ fragB1b, const void* __restrict__ fragA2b,
    const int32_t* __restrict__ bprime2_p,
    typename DT<MODE>::T* __restrict__ L, int64_t ldl, int64_t kS,
    const int32_t* __restrict__ sel_block, int32_t t, double* __restrict__ d,
    double* __restrict__ part_sum, double* __restrict__ part_max) {
  typedef typename DT<MODE>::T T;
  constexpr int MP = 16 * RT;
  constexpr int SLOT = RT * BT * kTileElems;
  constexpr int REGS = WPE == 1 ? 512 : 256;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Ps = reinterpret_cast<T*>(smem);                                            // nw * SLOT
  double* Ns = reinterpret_cast<double*>(smem + (size_t)nw * SLOT * sizeof(T));  // nw * MP
  __shared__ int32_t sb_s[MP];

  const int lane = threadIdx.x & 63;
  // wave index as a scalar, so that per-wave bases live in SGPRs and every
  // load below is a scalar base + 32-bit lane offset
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * MP;
  const int g0 = w * CT;                   // first global column tile of the wave
  T* __restrict__ Rw = R + r0 * ldr + 16 * (int64_t)g0;   // this wave's panel slice
  uint16_t* __restrict__ R16w = RIO ? R16 + r0 * ldr + 16 * (int64_t)g0 : nullptr;
  T* __restrict__ Lp = L + r0 * ldl + kS;
  // skeleton flags of the panel's rows (for the L rows and the norms)
  if (threadIdx.x < MP) {
    const int64_t row = r0 + threadIdx.x;
    sb_s[threadIdx.x] = row < m ? sel_block[row] : -2;
  }
  const int bp = *bprime_p;
  if (bp <= 0) return;
  typename DT<MODE>::V Rreg[RT][CT];
  // the body for NBV active b' tiles of one half (fragments FB, FA; bpv
  // kept columns at column offset LO of L)
#define RBRP_BODY(NBV, LD, ST, FB, FA, BPV, LO)                                             \
  deflate_body<MODE, RT, CT, BT, NBV, DEPTH, RIO, REGS, LD, ST>(                             \
      Rreg, Rw, R16w, (uint32_t)ldr, m, nw, w, lane, FB, FA, frag_stride, g0, BPV, Lp + (LO), \
      (uint32_t)ldl, t, sb_s, Ps, Ns, r0, d, part_sum, part_max)
  // the ladder of active tile counts (BF16 phase 2 works in chunks of 32
  // b'-columns: the tile count is rounded up to even)
#define RBRP_LADDER(LD, ST, FB, FA, BPV, LO)                                                \
  {                                                                                         \
    const int nbt = ((BPV) + 15) >> 4;                                                      \
    if constexpr (MODE == kModeBF16x3 || MODE == kModeBF16) {                               \
      const int nb2 = (nbt + 1) & ~1;                                                       \
      if constexpr (BT >= 8) { if (nb2 > 4) { RBRP_BODY(8, LD, ST, FB, FA, BPV, LO); return; } } \
      if constexpr (BT >= 4) { if (nb2 > 2) { RBRP_BODY(4, LD, ST, FB, FA, BPV, LO); return; } } \
      RBRP_BODY(2, LD, ST, FB, FA, BPV, LO);                                                \
    } else {                                                                                \
      if constexpr (BT >= 8) { if (nbt > 6) { RBRP_BODY(8, LD, ST, FB, FA, BPV, LO); return; } } \
      if constexpr (BT >= 8) { if (nbt > 4) { RBRP_BODY(6, LD, ST, FB, FA, BPV, LO); return; } } \
      if constexpr (BT >= 4) { if (nbt > 3) { RBRP_BODY(4, LD, ST, FB, FA, BPV, LO); return; } } \
      if constexpr (BT >= 4) { if (nbt > 2) { RBRP_BODY(3, LD, ST, FB, FA, BPV, LO); return; } } \
      if constexpr (BT >= 2) { if (nbt > 1) { RBRP_BODY(2, LD, ST, FB, FA, BPV, LO); return; } } \
      RBRP_BODY(1, LD, ST, FB, FA, BPV, LO);                                                \
    }                                                                                       \
    return;                                                                                 \
  }
  if constexpr (deflate_fuses<MODE, BT>()) {
    const int bp2 = bprime2_p ? *bprime2_p : 0;
    if (bp2 > 0) {
      // first half: all 128 columns, the residual kept in registers
      RBRP_BODY(8, true, false, fragB1, fragA2, bp, 0);
      __syncthreads();
      // second half on the updated residual, then stored with its norms
      RBRP_LADDER(false, true, fragB1b, fragA2b, bp2, 16 * BT)
    }
  }
  RBRP_LADDER(true, true, fragB1, fragA2, bp, 0)
#undef RBRP_LADDER
#undef RBRP_BODY
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
    // phase-1 operand: the column held by slot i of lane l; phase-2 operand:
    // the column assigned to result row l % 16
    const int pr = (MODE == kModeF64) ? (4 * (l16 & 3) + (l16 >> 2)) : l16;
    reinterpret_cast<T*>(fragB1)[e] = (T)q_at(16 * g + 4 * lhi + i, 16 * bt + l16);
    reinterpret_cast<T*>(fragA2)[e] = (T)q_at(16 * g + pr, 16 * bt + 4 * i + lhi);
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
// Configuration: n_pad = 16 * CT * nw.  Workgroups of up to four waves keep
// two workgroups resident per CU (registers <= 256 per lane); widths from
// 1280 to 2048 use eight waves of 16 column tiles on 32-row panels (one
// workgroup per CU, half the Q' fragment traffic per row of 16-row panels:
// measured 10-18% faster than four waves of 32 tiles at n = 2048), and the
// widest inputs eight waves of 32 column tiles.

struct DeflateCfg {
  int ct, rt, nw, nwmax;
};

struct Shape { int ct, nwmax; };
static const Shape kShapes[] = {{4, 4}, {8, 4}, {16, 4}, {16, 8}, {32, 4}, {32, 8}};

static bool shape_ok(int mode, const Shape& sh) {
  if (mode == kModeF64 && sh.ct > 16) return false;
  return true;
}

static int rt_for(int mode, int ct) {
  if (mode == kModeF64) return ct >= 16 ? 1 : 2;
  return ct >= 32 ? 1 : 2;
}

// smallest 16*CT*nw >= n; ties go to the narrower column tile (more rows per
// workgroup), then to fewer waves
static bool best_cfg(int mode, int64_t n, DeflateCfg* out) {
  int64_t best = -1;
  for (const Shape& sh : kShapes) {
    if (!shape_ok(mode, sh)) continue;
    const int lo = sh.nwmax == 8 ? 5 : 1;
    for (int nw = lo; nw <= sh.nwmax; ++nw) {
      const int64_t v = 16LL * sh.ct * nw;
      if (v < n) continue;
      if (best < 0 || v < best) {
        best = v;
        out->ct = sh.ct;
        out->nw = nw;
        out->nwmax = sh.nwmax;
        out->rt = rt_for(mode, sh.ct);
      }
    }
  }
  return best > 0;
}

static bool pick_cfg(int mode, int64_t ldr, DeflateCfg* c) {
  // FP32 products at 1536 or 2048 columns: the one-wave-per-SIMD shape
  // (measured 24 % faster per launch than eight waves of 16 tiles at 2048)
  if (mode == kModeF32 && (ldr == 1536 || ldr == 2048)) {
    c->ct = 32;
    c->rt = 2;
    c->nw = (int)(ldr / 512);
    c->nwmax = 4;
    return true;
  }
  // ldr comes from deflate_pad_cols (FP32 shapes); recover the shape for mode
  if (!best_cfg(mode, ldr, c)) return false;
  return 16LL * c->ct * c->nw == ldr;
}

int64_t deflate_pad_cols(int64_t n) {
  DeflateCfg c;
  if (!best_cfg(kModeF32, n, &c)) return -1;
  return 16LL * c.ct * c.nw;
}

static int bt_for(int mode, int bmax) {
  int bt = 1;
  while (16 * bt < bmax) bt <<= 1;
  if (is_bf16_mode(mode) && bt < 2) bt = 2;
  return bt;
}

int deflate_supported(int mode, int64_t ldr, int bmax) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return 0;
  return bmax >= 1 && bmax <= kMaxB;
}

bool deflate_fuses_halves(int mode) {
  return mode == kModeBF16 || mode == kModeBF16W || mode == kModeBF16R;
}

int deflate_rows_per_wg(int mode, int64_t ldr) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return 0;
  return 16 * c.rt;
}

int64_t deflate_num_partials(int64_t mr) { return ceil_div(mr, 16); }

int64_t frag_elems(int mode, int64_t ldr, int bmax) {
  const int bt = bt_for(mode, bmax);
  const int64_t G = ldr / 16;
  return G * bt * 64 * 4;
}

// The second half of a block wider than 128 kept columns (null bp: none).
struct Half2 {
  const void* fB;
  const void* fA;
  const int32_t* bp;
};

template <int MODE, int RT, int CT, int BT, int NWMAX, int RIO, int WPEV = 2, int DPO = 0>
static hipError_t run_deflate(const DeflateCfg& c, int64_t grid, hipStream_t s,
                              void* R, void* R16, int64_t ldr, int64_t m, const void* fB,
                              const void* fA, int64_t fstride, const int32_t* bp,
                              Half2 h2, void* L, int64_t ldl, int64_t kS,
                              const int32_t* sel,
                              int32_t t, double* d, double* ps, double* pm) {
  typedef typename DT<MODE>::T T;
  // FP32 panels of 16 column tiles keep four chunks in flight (with the
  // scheduling fences, measured 8-16% faster than three); the other shapes
  // are register-bound
  constexpr int DP = DPO ? DPO : ((MODE == kModeF32 && CT == 16 && RT == 2) ? 4 : kDepth);
  const size_t slot = (size_t)RT * BT * kTileElems * sizeof(T);
  const size_t lds = c.nw * slot + (size_t)c.nw * 16 * RT * sizeof(double);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_deflate<MODE, RT, CT, BT, NWMAX, DP, RIO, WPEV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024 - 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 160 * 1024 - 1024) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_deflate<MODE, RT, CT, BT, NWMAX, DP, RIO, WPEV>), dim3((unsigned)grid),
                     dim3(64 * c.nw), lds, s, (T*)R, (uint16_t*)R16, ldr, m, c.nw, fB, fA,
                     fstride, bp, h2.fB, h2.fA, h2.bp, (T*)L, ldl, kS, sel, t, d, ps, pm);
  return hipGetLastError();
}

template <int MODE, int BT, int RIO>
static hipError_t dispatch_ct(const DeflateCfg& c, int64_t mr, hipStream_t s, void* R,
                              void* R16, int64_t ldr, int64_t m, const void* fB,
                              const void* fA, int64_t fstride, const int32_t* bp, Half2 h2,
                              void* L, int64_t ldl, int64_t kS, const int32_t* sel, int32_t t,
                              double* d, double* ps, double* pm) {
#define RBRP_DEF_CASE(CTV, RTV, NWV)                                                   \
  if (c.ct == CTV && c.rt == RTV && c.nwmax == NWV)                                   \
    return run_deflate<MODE, RTV, CTV, BT, NWV, RIO>(c, mr / (16 * RTV), s, R, R16, ldr, \
                                                     m, fB, fA, fstride, bp, h2, L, ldl, kS, \
                                                     sel, t, d, ps, pm);
  if constexpr (MODE == kModeF64) {
    RBRP_DEF_CASE(4, 2, 4)
    RBRP_DEF_CASE(8, 2, 4)
    RBRP_DEF_CASE(16, 1, 4)
    RBRP_DEF_CASE(16, 1, 8)
  } else {
    RBRP_DEF_CASE(4, 2, 4)
    RBRP_DEF_CASE(8, 2, 4)
    RBRP_DEF_CASE(16, 2, 4)
    RBRP_DEF_CASE(16, 2, 8)
    RBRP_DEF_CASE(32, 1, 4)
    RBRP_DEF_CASE(32, 1, 8)
    // FP32 products on 1536- or 2048-column residuals: four waves of 32
    // column tiles on 32-row panels at one wave per SIMD (512 registers:
    // the residual slice in the accumulation registers), two chunks in
    // flight
    if constexpr (MODE == kModeF32 && RIO == 0)
      if (c.ct == 32 && c.rt == 2 && c.nwmax == 4)
        return run_deflate<MODE, 2, 32, BT, 4, RIO, 1, 2>(c, mr / 32, s, R, R16, ldr, m, fB, fA,
                                                          fstride, bp, h2, L, ldl, kS, sel, t, d, ps,
                                                          pm);
  }
#undef RBRP_DEF_CASE
  return hipErrorInvalidConfiguration;
}

template <int MODE, int RIO>
static hipError_t dispatch_bt(int bt, const DeflateCfg& c, int64_t mr, hipStream_t s,
                              void* R, void* R16, int64_t ldr, int64_t m, const void* fB,
                              const void* fA, int64_t fstride, const int32_t* bp,
                              Half2 h2, void* L, int64_t ldl, int64_t kS,
                              const int32_t* sel,
                              int32_t t, double* d, double* ps, double* pm) {
  switch (bt) {
    case 1:
      if constexpr (MODE == kModeF64 || MODE == kModeF32)
        return dispatch_ct<MODE, 1, RIO>(c, mr, s, R, R16, ldr, m, fB, fA, fstride, bp, h2, L,
                                         ldl, kS, sel, t, d, ps, pm);
      break;
    case 2:
      return dispatch_ct<MODE, 2, RIO>(c, mr, s, R, R16, ldr, m, fB, fA, fstride, bp, h2, L, ldl,
                                       kS, sel, t, d, ps, pm);
    case 4:
      return dispatch_ct<MODE, 4, RIO>(c, mr, s, R, R16, ldr, m, fB, fA, fstride, bp, h2, L, ldl,
                                       kS, sel, t, d, ps, pm);
    case 8:
      return dispatch_ct<MODE, 8, RIO>(c, mr, s, R, R16, ldr, m, fB, fA, fstride, bp, h2, L, ldl,
                                       kS, sel, t, d, ps, pm);
  }
  return hipErrorInvalidConfiguration;
}

hipError_t launch_deflate(int mode, void* R, void* R16, int64_t mr, int64_t ldr, int64_t m,
                          const void* fragB1, const void* fragA2,
                          const int32_t* bprime, int bmax, const void* fragB1b,
                          const void* fragA2b, const int32_t* bprime2, void* L, int64_t ldl,
                          int64_t kS, const int32_t* sel_block, int32_t t, double* d,
                          double* part_sum, double* part_max, hipStream_t s) {
  DeflateCfg c;
  if (!pick_cfg(mode, ldr, &c)) return hipErrorInvalidConfiguration;
  if (mr % (16 * c.rt)) return hipErrorInvalidValue;
  if (mode_stores_bf16(mode) && (!R16 || ldr % 32)) return hipErrorInvalidValue;
  const int bt = bt_for(mode, bmax);
  const int64_t fstride = frag_elems(mode, ldr, bmax) / (is_bf16_mode(mode) ? 8 : 4);
  // a second half only in one launch with the first (kernels of 128-column
  // blocks with one BF16 product)
  if (bprime2 && (bt != 8 || !deflate_fuses_halves(mode) || !fragB1b || !fragA2b))
    return hipErrorInvalidValue;
  const Half2 h2{fragB1b, fragA2b, bprime2};
#define RBRP_ARGS bt, c, mr, s, R, R16, ldr, m, fragB1, fragA2, fstride, bprime, h2, L, ldl, kS, \
                  sel_block, t, d, part_sum, part_max
  switch (mode) {
    case kModeF64: return dispatch_bt<kModeF64, 0>(RBRP_ARGS);
    case kModeF32: return dispatch_bt<kModeF32, 0>(RBRP_ARGS);
    case kModeBF16x3: return dispatch_bt<kModeBF16x3, 0>(RBRP_ARGS);
    case kModeBF16: return dispatch_bt<kModeBF16, 0>(RBRP_ARGS);
    case kModeBF16W: return dispatch_bt<kModeBF16, 1>(RBRP_ARGS);
    case kModeBF16R: return dispatch_bt<kModeBF16, 2>(RBRP_ARGS);
  }
#undef RBRP_ARGS
  return hipErrorInvalidValue;
}

// BF16 residual (permuted 32-column groups) back to FP32 in natural column
// order, one thread per 8 stored values.
__global__ __launch_bounds__(256) void k_r16_to_r32(const uint16_t* __restrict__ R16,
                                                    float* __restrict__ R, int64_t total8) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total8) return;
  const uint4 u = reinterpret_cast<const uint4*>(R16)[e];
  const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
  // stored positions 8 h .. 8 h + 7 of a 32-column group: h = e % 4
  const int64_t grp = e >> 2;
  const int h = (int)(e & 3);
  float* dst = R + grp * 32;
#pragma unroll
  for (int pj = 0; pj < 8; ++pj) {
    const uint32_t x = wv[pj >> 1];
    const uint32_t bits = (pj & 1) ? (x & 0xFFFF0000u) : (x << 16);
    const int p = pj >> 2, j = pj & 3;
    dst[16 * p + 4 * h + j] = __uint_as_float(bits);
  }
}

hipError_t launch_r16_to_r32(const void* R16, void* R, int64_t mr, int64_t ldr,
                             hipStream_t s) {
  if (ldr % 32) return hipErrorInvalidValue;
  const int64_t total8 = mr * ldr / 8;
  hipLaunchKernelGGL(k_r16_to_r32, dim3((unsigned)ceil_div(total8, 256)), dim3(256), 0, s,
                     (const uint16_t*)R16, (float*)R, total8);
  return hipGetLastError();
}

hipError_t launch_make_frags(const double* Qt_new, int64_t ldq, const int32_t* bprime,
                             int64_t n_pad, int bmax, int mode, void* fragB1,
                             void* fragA2, hipStream_t s) {
  const int bt = bt_for(mode, bmax);
  const int64_t G = n_pad / 16;
  const bool bf = is_bf16_mode(mode);
  const int64_t total = G * bt * 64 * 4;
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
    case kModeBF16W:
    case kModeBF16R:
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
