// Workgroup-level building blocks shared by the per-step kernels and the
// batched kernel: the exact integer block sampler of Alg. 2 (weights,
// Philox4x64-10 draws, successive sampling) and the pivoted Cholesky of the
// block filter.  Every function here is called by all threads of one
// workgroup and ends past a barrier.
#pragma once

#include "rbrp_internal.h"

#include <math.h>

namespace rbrp {

constexpr int kSampleThreads = 256;

__device__ __forceinline__ int ceil_log2_dev(int64_t m) {
  if (m <= 1) return 0;
  return 64 - __clzll((unsigned long long)(m - 1));
}

__device__ __forceinline__ int weight_shift(double dmax, int64_t m) {
  int e = 0;
  frexp(dmax, &e);
  return 62 - e - ceil_log2_dev(m);
}

__device__ __forceinline__ uint64_t weight_of(double di, int s) {
  if (!(di > 0.0)) return 0;
  return (uint64_t)floor(ldexp(di, s));
}

// ---- Philox4x64-10 ----
__device__ __forceinline__ uint64_t philox_word0(uint64_t j, uint64_t t,
                                                 uint64_t id, uint64_t seed) {
  uint64_t c0 = j, c1 = t, c2 = id, c3 = 0;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c0;
    const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
    const uint64_t lo1 = 0xCA5A826395121157ull * c2;
    const uint64_t hi1 = __umul64hi(0xCA5A826395121157ull, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// Global inclusive prefix at row i.
__device__ __forceinline__ uint64_t cdf_at(const uint64_t* cdf_local,
                                           const uint64_t* tile_excl, int64_t i) {
  return tile_excl[i / kScanTile] + cdf_local[i];
}

// Weight of row i recovered from the local prefix.
__device__ __forceinline__ uint64_t weight_at(const uint64_t* cdf_local, int64_t i) {
  const uint64_t prev = (i % kScanTile) ? cdf_local[i - 1] : 0;
  return cdf_local[i] - prev;
}

// Weights of one tile of kScanTile rows (256 threads x 8 rows) and their
// inclusive prefix within the tile; tile totals (weight and number of
// positive weights) to tile_sum / tile_pos.  wsum / wpos: 4 entries in LDS.
// Ends with every thread past a barrier.
__device__ __forceinline__ void wg_weights_scan_tile(
    const double* __restrict__ d, const int32_t* __restrict__ sel_block,
    const uint8_t* __restrict__ excluded, int64_t m, double dmax, int64_t tile,
    uint64_t* __restrict__ cdf_local, uint64_t* __restrict__ tile_sum,
    int32_t* __restrict__ tile_pos, uint64_t* wsum, int32_t* wpos) {
  const int s = dmax > 0.0 ? weight_shift(dmax, m) : 0;
  const int64_t base = tile * kScanTile + threadIdx.x * 8;
  uint64_t w[8];
  int pos = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = base + q;
    uint64_t v = 0;
    if (i < m && dmax > 0.0) {
      const bool out = (sel_block && sel_block[i] >= 0) || (excluded && excluded[i]);
      if (!out) v = weight_of(d[i], s);
    }
    w[q] = v;
    pos += v != 0;
  }
#pragma unroll
  for (int q = 1; q < 8; ++q) w[q] += w[q - 1];
  // exclusive scan of thread totals across the wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t incl = w[7];
  int ipos = pos;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t o = __shfl_up(incl, off, kWave);
    const int op = __shfl_up(ipos, off, kWave);
    if (lane >= off) {
      incl += o;
      ipos += op;
    }
  }
  if (lane == 63) {
    wsum[wv] = incl;
    wpos[wv] = ipos;
  }
  __syncthreads();
  uint64_t wave_off = 0;
  for (int i = 0; i < wv; ++i) wave_off += wsum[i];
  const uint64_t excl = incl - w[7] + wave_off;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = base + q;
    if (i < m) cdf_local[i] = w[q] + excl;
  }
  if (threadIdx.x == 0) {
    tile_sum[tile] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    tile_pos[tile] = wpos[0] + wpos[1] + wpos[2] + wpos[3];
  }
  __syncthreads();
}

// Exclusive count of the set flags before each thread of the workgroup
// (thread order) by wave ballots; *total gets the count over all threads.
// wtot: kSampleThreads / 64 ints of LDS.  Called by all threads; contains
// barriers.
__device__ __forceinline__ int wg_flag_offset(int f, int32_t* wtot, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(f != 0);
  const int pre = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wtot[w] = __popcll(bal);
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int v = 0; v < kSampleThreads / 64; ++v) {
    const int c = wtot[v];
    base += v < w ? c : 0;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + pre;
}

// LDS state of the block sampler (one workgroup of kSampleThreads threads).
template <int MAXTILES, int MAXB>
struct SampleShared {
  uint64_t tile_excl[MAXTILES + 1];
  int64_t acc_idx[MAXB];
  uint64_t acc_w[MAXB];
  int64_t cand[kSampleThreads];
  int32_t flag[kSampleThreads];
  uint64_t red[kSampleThreads];
  int32_t nacc, npos;
  uint64_t W;
};

// b rows drawn without replacement from the tiled integer CDF (weights and
// per-tile prefixes from wg_weights_scan_tile), candidates counted from 0
// with Philox counter (j, t, ident, 0) and key (seed, 0).  Writes idx[0..nt)
// and *nt_out (and *npos_out, the number of positive weights).  Called by all
// kSampleThreads threads of the workgroup; ends past a barrier.  b <= MAXB.
template <int MAXTILES, int MAXB>
__device__ __forceinline__ void wg_sample(
    const uint64_t* __restrict__ cdf_local, const uint64_t* __restrict__ tile_sum,
    const int32_t* __restrict__ tile_pos, int64_t m, int32_t b, uint64_t seed,
    uint64_t t, uint64_t ident, int64_t* __restrict__ idx, int32_t* nt_out,
    int32_t* npos_out, SampleShared<MAXTILES, MAXB>& sh) {
  int32_t& s_nacc = sh.nacc;
  int32_t& s_npos = sh.npos;
  uint64_t& s_W = sh.W;
  uint64_t* tile_excl = sh.tile_excl;
  int64_t* acc_idx = sh.acc_idx;
  uint64_t* acc_w = sh.acc_w;
  int64_t* cand = sh.cand;
  int32_t* flag = sh.flag;
  uint64_t* red = sh.red;
  const int tid = threadIdx.x;
  const int64_t ntiles = ceil_div(m, kScanTile);

  // exclusive prefix of the tile totals: each thread sums a run of tiles,
  // wave 0 scans the run sums (four per lane), each thread writes its run
  {
    const int64_t per = ceil_div(ntiles, (int64_t)kSampleThreads);
    const int64_t T0 = tid * per, T1 = min(ntiles, T0 + per);
    uint64_t rs = 0;
    int rp = 0;
    for (int64_t T = T0; T < T1; ++T) {
      rs += tile_sum[T];
      rp += tile_pos[T];
    }
    red[tid] = rs;
    flag[tid] = rp;
    __syncthreads();
    if (tid < 64) {
      uint64_t v[4];
      int np = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = red[4 * tid + u];
        np += flag[4 * tid + u];
      }
      const uint64_t mine = v[0] + v[1] + v[2] + v[3];
      uint64_t incl = mine;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(incl, off, kWave);
        if (tid >= off) incl += o;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) np += __shfl_xor(np, off, kWave);
      uint64_t run = incl - mine;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        red[4 * tid + u] = run;
        run += v[u];
      }
      if (tid == 63) {
        s_W = incl;
        s_npos = np;
        s_nacc = 0;
      }
    }
    __syncthreads();
    uint64_t run = red[tid];
    for (int64_t T = T0; T < T1; ++T) {
      tile_excl[T] = run;
      run += tile_sum[T];
    }
    if (tid == 0) tile_excl[ntiles] = s_W;
  }
  __syncthreads();
  const uint64_t W = s_W;
  const int npos = s_npos;

  if (npos <= b) {
    // every row with positive weight, in index order
    int nacc = 0;
    for (int64_t T = 0; T < ntiles; ++T) {
      if (tile_pos[T] == 0) continue;
      const int64_t r0 = T * kScanTile;
      for (int64_t c0 = r0; c0 < r0 + kScanTile && c0 < m; c0 += kSampleThreads) {
        const int64_t i = c0 + tid;
        const int pos = (i < m && i < r0 + kScanTile) ? (weight_at(cdf_local, i) != 0) : 0;
        int total;
        const int off = wg_flag_offset(pos, flag, &total);
        if (pos) idx[nacc + off] = i;
        nacc += total;
      }
    }
    if (tid == 0) {
      *nt_out = nacc;
      if (npos_out) *npos_out = npos;
    }
    __syncthreads();
    return;
  }

  // rejection form: chunks of candidates resolved in parallel
  const int64_t jmax = (int64_t)kRejectionFactor * b;
  for (int64_t j0 = 0; j0 < jmax; j0 += kSampleThreads) {
    const int nacc = s_nacc;
    if (nacc >= b) break;
    const int64_t j = j0 + tid;
    int64_t my = -1;
    if (j < jmax) {
      const uint64_t x = philox_word0((uint64_t)j, t, ident, seed);
      const uint64_t target = __umul64hi(x, W);
      // tile: smallest T with tile_excl[T+1] > target
      int64_t lo = 0, hi = ntiles - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (tile_excl[mid + 1] > target) hi = mid; else lo = mid + 1;
      }
      const uint64_t local = target - tile_excl[lo];
      // smallest i of the tile with cdf_local[i] > local (cdf_local[z] is
      // the tile total, so one exists): eight probes per round, all loaded
      // before any is compared, shrink [a, z] to a ninth
      int64_t a = lo * kScanTile, z = min(m, (lo + 1) * (int64_t)kScanTile) - 1;
      while (a < z) {
        int64_t pr[8];
        uint64_t pv[8];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
          pr[s8] = a + ((s8 + 1) * (z - a)) / 9;
          pv[s8] = cdf_local[pr[s8]];
        }
        int64_t na = a, nz = z;
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
          if (pv[s8] > local) nz = min(nz, pr[s8]);
          else na = max(na, pr[s8] + 1);
        }
        a = na;
        z = nz;
      }
      my = a;
    }
    cand[tid] = my;
    __syncthreads();
    // new if neither accepted before nor drawn by an earlier candidate of
    // the chunk (every comparison made: no data-dependent exit, so the LDS
    // reads of a loop are issued back to back)
    int dup = 0;
    for (int q = 0; q < nacc; ++q) dup |= acc_idx[q] == my;
    const int qend = tid | 63;   // the wave's last thread: a uniform bound
    for (int q = 0; q < qend; ++q) dup |= (q < tid) & (cand[q] == my);
    const int isnew = my >= 0 && !dup;
    int total;
    const int off = wg_flag_offset(isnew, flag, &total);
    if (isnew) {
      const int p = nacc + off;
      if (p < b) {
        acc_idx[p] = my;
        acc_w[p] = weight_at(cdf_local, my);
      }
    }
    if (tid == 0) s_nacc = min(b, nacc + total);
    __syncthreads();
  }

  // removal form: weights of accepted rows removed, one draw per candidate
  for (int64_t j = jmax; s_nacc < b; ++j) {
    const int nacc = s_nacc;
    // W' = W - sum of accepted weights
    uint64_t part = 0;
    for (int q = tid; q < nacc; q += kSampleThreads) part += acc_w[q];
    red[tid] = part;
    __syncthreads();
    if (tid == 0) {
      uint64_t tot = 0;
      for (int q = 0; q < kSampleThreads; ++q) tot += red[q];
      red[0] = tot;
    }
    __syncthreads();
    const uint64_t Wp = W - red[0];
    __syncthreads();
    const uint64_t x = philox_word0((uint64_t)j, t, ident, seed);
    const uint64_t target = __umul64hi(x, Wp);
    int64_t lo = 0, hi = m - 1;
    while (lo < hi) {  // uniform across the workgroup
      const int64_t mid = (lo + hi) >> 1;
      uint64_t adj = 0;
      for (int q = tid; q < nacc; q += kSampleThreads)
        if (acc_idx[q] <= mid) adj += acc_w[q];
      red[tid] = adj;
      __syncthreads();
      if (tid == 0) {
        uint64_t tot = 0;
        for (int q = 0; q < kSampleThreads; ++q) tot += red[q];
        red[0] = cdf_at(cdf_local, tile_excl, mid) - tot;
      }
      __syncthreads();
      const bool above = red[0] > target;
      __syncthreads();
      if (above) hi = mid; else lo = mid + 1;
    }
    if (tid == 0) {
      acc_idx[nacc] = lo;
      acc_w[nacc] = weight_at(cdf_local, lo);
      s_nacc = nacc + 1;
    }
    __syncthreads();
  }
  const int nt = s_nacc;
  for (int q = tid; q < nt; q += kSampleThreads) idx[q] = acc_idx[q];
  if (tid == 0) {
    *nt_out = nt;
    if (npos_out) *npos_out = npos;
  }
  __syncthreads();
}

// ---- wave-level argmax / sum without LDS traffic ----
// (value, index) pairs are ordered by value, then by the lower index; an
// index < 0 marks "no candidate".
__device__ __forceinline__ bool piv_better(double ob, int oi, double best, int bi) {
  return oi >= 0 && (bi < 0 || ob > best || (ob == best && oi < bi));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = dpp_i32<CTRL>((int)b);
  const int hi = dpp_i32<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int LANE>
__device__ __forceinline__ double readlane_f64(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, LANE);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), LANE);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ void argmax_sum_step(double& best, int& bi, double& sum) {
  const double ob = dpp_f64<CTRL>(best);
  const int oi = dpp_i32<CTRL>(bi);
  sum += dpp_f64<CTRL>(sum);   // both partners form the same sum (addition commutes)
  if (piv_better(ob, oi, best, bi)) {
    best = ob;
    bi = oi;
  }
}

template <int ROW>
__device__ __forceinline__ void argmax_sum_fold_row(double best, int bi, double sum,
                                                    double& B, int& I, double& T) {
  const double ob = readlane_f64<16 * ROW>(best);
  const int oi = __builtin_amdgcn_readlane(bi, 16 * ROW);
  T += readlane_f64<16 * ROW>(sum);
  if (piv_better(ob, oi, B, I)) {
    B = ob;
    I = oi;
  }
}

// Argmax and sum over the 64 lanes of a wave (all lanes active).  Within
// rows of 16 lanes: DPP butterflies (quad permutations, half-row and row
// mirrors), after which every lane of a row holds the row's result; the four
// rows are then folded in order through readlane.  The result is uniform and
// the summation order is fixed.
__device__ __forceinline__ void wave_argmax_sum(double& best, int& bi, double& sum) {
  argmax_sum_step<0xB1>(best, bi, sum);   // quad_perm [1,0,3,2]
  argmax_sum_step<0x4E>(best, bi, sum);   // quad_perm [2,3,0,1]
  argmax_sum_step<0x141>(best, bi, sum);  // row_half_mirror
  argmax_sum_step<0x140>(best, bi, sum);  // row_mirror
  double B = readlane_f64<0>(best);
  int I = __builtin_amdgcn_readlane(bi, 0);
  double T = readlane_f64<0>(sum);
  argmax_sum_fold_row<1>(best, bi, sum, B, I, T);
  argmax_sum_fold_row<2>(best, bi, sum, B, I, T);
  argmax_sum_fold_row<3>(best, bi, sum, B, I, T);
  best = B;
  bi = I;
  sum = T;
}

template <int CTRL>
__device__ __forceinline__ void max_sum_step(double& mx, double& sum) {
  mx = fmax(mx, dpp_f64<CTRL>(mx));
  sum += dpp_f64<CTRL>(sum);
}

// Maximum and sum over the 64 lanes of a wave (all lanes active), both
// uniform on return; the summation order is fixed (DPP butterflies within
// rows of 16 lanes, then the four rows in order).
__device__ __forceinline__ void wave_max_sum(double& mx, double& sum) {
  max_sum_step<0xB1>(mx, sum);
  max_sum_step<0x4E>(mx, sum);
  max_sum_step<0x141>(mx, sum);
  max_sum_step<0x140>(mx, sum);
  const double m0 = readlane_f64<0>(mx), m1 = readlane_f64<16>(mx);
  const double m2 = readlane_f64<32>(mx), m3 = readlane_f64<48>(mx);
  const double t0 = readlane_f64<0>(sum), t1 = readlane_f64<16>(sum);
  const double t2 = readlane_f64<32>(sum), t3 = readlane_f64<48>(sum);
  mx = fmax(fmax(m0, m1), fmax(m2, m3));
  sum = ((t0 + t1) + t2) + t3;
}

// LDS state of the pivoted Cholesky (besides the Schur complement itself).
constexpr int kPivKB = 16;   // pivot rows per delayed Schur-complement update
constexpr int kPivLd = 18;   // row stride (doubles) of the transposed pivot rows
constexpr int kPivThreads = 256;

typedef double dmfma4 __attribute__((ext_vector_type(4)));

template <int NBMAX>
struct PivShared {
  alignas(16) double rblk[NBMAX][kPivLd];  // rblk[c][q]: entry c of pivot row q of the group
  int32_t chosen[NBMAX];
  int32_t pivs[NBMAX];
  int32_t fin, bp;
};

template <int LANE_DUMMY = 0>
__device__ __forceinline__ double readlane_f64_rt(double x, int lane) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Cholesky of the block's Gram matrix G (nb x nb, nb <= NBMAX <= kPivThreads)
// by kPivThreads threads: pivoted (PIVOTED, the filter: pivot = largest
// remaining Schur diagonal, ties to the lower index, stop at the truncation
// threshold) or in natural order (the reorthogonalisation pass).
//
// The pivot steps run in wave 0 alone, so that a step needs no barrier: lane
// l owns columns l, l + 64, ... of the Schur complement S, keeps their exact
// diagonal entries in registers (downdated at every step) and forms their
// entries of each pivot row; the argmax and the sum of the diagonal are
// wave-level DPP reductions in a fixed order.  S itself is brought up to
// date only once per group of kPivKB steps, by all threads (a rank-kPivKB
// update with the group's pivot rows, the delayed update of blocked pivoted
// Cholesky); inside a group a pivot row is formed from the last update plus
// the corrections of the group's earlier pivots.  S lives in LDS (GS false:
// copied from G, row stride nb + 1) or in global memory (GS true: S is G
// itself, updated in place).
//
// Outputs: pivots (kept ones first, the rest in increasing order), b' (the
// steps done), the pivot rows of R with unpermuted columns (Rraw), R11 in
// pivoted order (Rp, nb_host x nb_host, zero outside the leading b' x b'
// upper triangle), ||V||_F^2 and the rank-guard flag (pivoted mode only).
// Ends past a barrier.
template <int NBMAX, bool GS, bool PIVOTED>
__device__ __forceinline__ void wg_piv_chol(
    const double* __restrict__ G, int64_t ldg, int32_t nb_host,
    const int32_t* __restrict__ nb_dev, double tau_b,
    const double* __restrict__ xs2_rows, int32_t* __restrict__ piv,
    double* __restrict__ Rraw, int64_t ldr, double* __restrict__ Rp, int64_t ldp,
    int32_t* __restrict__ bprime_out, double* __restrict__ tail1_out,
    int32_t* __restrict__ stop_out, double* __restrict__ S, PivShared<NBMAX>& sh,
    int nsl = 1, int64_t gstride = 0) {
  static_assert(NBMAX <= kPivThreads, "at most one column per thread in the updates");
  constexpr int NPL = (NBMAX + 63) / 64;       // columns per lane of wave 0
  constexpr int NCOLS = 64 * NPL;
  constexpr int TPC = kPivThreads / NCOLS;     // threads per column in the updates
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  int nb = nb_host;
  if (nb_dev) nb = min(nb, *nb_dev);
  const int64_t ld = GS ? ldg : nb + 1;
  if constexpr (!GS) {
    // thread (column c, part) copies rows part, part + TPC, ...; eight rows'
    // loads are issued before their stores.  G may come as nsl K slices of
    // partial sums (gstride apart), added in slice order.
    const int c = tid % NCOLS, part = tid / NCOLS;
    if (c < nb) {
      for (int r0 = part; r0 < nb; r0 += 8 * TPC) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = min(r0 + u * TPC, nb - 1);
          x[u] = G[(int64_t)r * ldg + c];
        }
        if (nsl > 1) {
          double xz[kNtMaxSlices - 1][8];
#pragma unroll
          for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int r = min(r0 + u * TPC, nb - 1);
              xz[z - 1][u] = G[min(z, nsl - 1) * gstride + (int64_t)r * ldg + c];
            }
#pragma unroll
          for (int z = 1; z < kNtMaxSlices; ++z)
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] += z < nsl ? xz[z - 1][u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (r0 + u * TPC < nb) S[(r0 + u * TPC) * ld + c] = x[u];
      }
    }
  }
  if (tid < NBMAX) sh.chosen[tid] = (tid < nb) ? 0 : 1;
  if (tid == 0) {
    sh.fin = 0;
    sh.bp = 0;
  }
  __syncthreads();
  // wave-0 state: the owned columns' diagonal entries and flags (their
  // entries of the group's pivot rows are read back from rblk)
  double dj[NPL];
  bool ch[NPL];
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int c = lane + 64 * j;
    ch[j] = c >= nb;
    dj[j] = (wv == 0 && c < nb) ? S[(int64_t)c * ld + c] : 0.0;
  }
  double thr = 0.0;
  for (int g = 0;; ++g) {
    if (wv == 0) {
      bool fin = false;
      int bp = 0;
      // fully unrolled (qb a constant in each step): the steps after the
      // last one are skipped rather than left by a break, which would keep
      // the compiler from unrolling
#pragma unroll
      for (int qb = 0; qb < kPivKB; ++qb) {
        if (fin) continue;
        const int p = g * kPivKB + qb;
        // largest remaining diagonal entry (the wave maximum, then the lowest
        // column holding it: columns l + 64 j ascend with j, then with l)
        double best = -INFINITY, sum = 0.0;
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          if (!ch[j]) {
            sum += fmax(dj[j], 0.0);
            best = fmax(best, dj[j]);
          }
        }
        wave_max_sum(best, sum);
        int bi = -1;
        if (best > -INFINITY) {
#pragma unroll
          for (int j = NPL - 1; j >= 0; --j) {
            const unsigned long long hit = __ballot(!ch[j] && dj[j] == best);
            if (hit) bi = 64 * j + (__ffsll((long long)hit) - 1);
          }
        }
        const double tail = sum;
        bool done = false;
        if (PIVOTED && p == 0) {
          thr = tau_b * tail * (1.0 - 4.0 * nb * 1.1102230246251565e-16);
          if (lane == 0 && tail1_out) *tail1_out = tail;
          if (xs2_rows) {
            // ||X(S_t,:)||_F^2: all loads at once, then a wave sum
            double xs2 = 0.0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
              const int c = lane + 64 * j;
              const double x = xs2_rows[c < nb ? c : nb - 1];   // clamped: always in range
              xs2 += c < nb ? x : 0.0;
            }
            double dmy = 0.0;
            int dmi = -1;
            wave_argmax_sum(dmy, dmi, xs2);
            if (!(tail > 1e-26 * xs2)) {
              done = true;
              if (stop_out && lane == 0) *stop_out = 1;
            }
          }
        }
        int jp = bi;
        double gv = best;
        if (!PIVOTED) {
          jp = p;
          gv = 0.0;
          if (p < nb) {
            double x = dj[0];
#pragma unroll
            for (int j = 1; j < NPL; ++j)
              if ((p >> 6) == j) x = dj[j];
            gv = readlane_f64_rt(x, p & 63);
          }
        }
        if (p >= nb || jp < 0 || !(gv > 0.0)) done = true;
        if (PIVOTED && p > 0 && tail < thr) done = true;
        if (done) {
          bp = p;
          fin = true;
          continue;
        }
        const double r = sqrt(gv);
        const double rinv = 1.0 / r;
        const double* rj = sh.rblk[jp];
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          const int c = lane + 64 * j;
          double v = 0.0;
          if (c == jp) {
            v = r;
          } else if (!ch[j]) {
            // the corrections of the group's qb earlier pivots (qb is a
            // compile-time constant in each unrolled step: straight-line LDS
            // reads, two partial sums)
            const double a = S[(int64_t)jp * ld + c];
            const double* rc = sh.rblk[c];
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q + 1 < qb; q += 2) {
              s0 += rj[q] * rc[q];
              s1 += rj[q + 1] * rc[q + 1];
            }
            if (qb & 1) s0 += rj[qb - 1] * rc[qb - 1];
            v = (a - (s0 + s1)) * rinv;
          }
          if (c < NBMAX) sh.rblk[c][qb] = v;
          if (c < nb) Rraw[(int64_t)p * ldr + c] = v;
          if (c == jp) {
            ch[j] = true;
            sh.chosen[c] = 1;
            sh.pivs[p] = jp;
          }
          dj[j] -= v * v;
        }
      }
      if (lane == 0) {
        sh.fin = fin ? 1 : 0;
        sh.bp = bp;
      }
    }
    __syncthreads();
    if (sh.fin) break;
    // delayed update of S by the group's pivot rows, S -= B B^T with
    // B(c, q) = entry c of pivot row q.  In LDS for 64 or more columns: a
    // rank-16 product on FP64 MFMA over 16 x 16 tiles of S, wave w taking
    // tiles w, w + 4, ...; a tile is skipped when its rows or its columns
    // are all chosen (entries of chosen rows and columns are never read
    // again, so the others may be updated too).  Not needed after the group
    // that reaches nb pivots.
    if constexpr (!GS && NBMAX >= 64) {
      if ((g + 1) * kPivKB < nb) {
        const int nt = (nb + 15) >> 4;
        const int l16 = lane & 15, lq = lane >> 4;
        for (int tile = wv; tile < nt * nt; tile += kPivThreads / 64) {
          const int ti = tile / nt, tj = tile - ti * nt;
          const int ra = 16 * ti + l16, rb = 16 * tj + l16;
          const bool rlive = ra < nb && !sh.chosen[ra];
          const bool clive = rb < nb && !sh.chosen[rb];
          if (__ballot(rlive) == 0ull || __ballot(clive) == 0ull) continue;
          dmfma4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < kPivKB / 4; ++s4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sh.rblk[ra][4 * s4 + lq],
                                                       sh.rblk[rb][4 * s4 + lq], acc, 0, 0, 0);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = 16 * ti + lq + 4 * q;
            if (i < nb && rb < nb) S[(int64_t)i * ld + rb] -= acc[q];
          }
        }
      }
    } else {
      // thread (column c, part) takes rows part, part + TPC, ... (the same
      // rows across a wave)
      const int c = tid % NCOLS, part = tid / NCOLS;
      if (c < nb && !sh.chosen[c]) {
        double rc[kPivKB];
#pragma unroll
        for (int q = 0; q < kPivKB; ++q) rc[q] = sh.rblk[c][q];
        constexpr int RU = GS ? 8 : 4;
        for (int i0 = part; i0 < nb; i0 += RU * TPC) {
          double a[RU];
          bool live[RU];
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int i = i0 + u * TPC;
            live[u] = i < nb && !sh.chosen[i];
            a[u] = S[(int64_t)(live[u] ? i : c) * ld + c];
          }
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            if (!live[u]) continue;
            const double* ri = sh.rblk[i0 + u * TPC];
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q < kPivKB; q += 2) {
              s0 += ri[q] * rc[q];
              s1 += ri[q + 1] * rc[q + 1];
            }
            S[(int64_t)(i0 + u * TPC) * ld + c] = a[u] - (s0 + s1);
          }
        }
      }
    }
    __syncthreads();
  }
  const int bp = sh.bp;
  // the remaining columns after the kept ones, in increasing order
  if (wv == 0) {
    int base = bp;
    for (int c0 = 0; c0 < nb; c0 += 64) {
      const int c = c0 + lane;
      const bool rest = c < nb && !sh.chosen[c];
      const unsigned long long mask = __ballot(rest);
      const int pos = __popcll(mask & ((1ull << lane) - 1ull));
      if (rest) sh.pivs[base + pos] = c;
      base += __popcll(mask);
    }
    if (lane == 0) *bprime_out = bp;
  }
  __syncthreads();
  if (tid < nb) piv[tid] = sh.pivs[tid];
  // R11 in pivoted order, zero outside the leading b' x b' upper triangle:
  // thread (column c, part) fills rows part, part + TPC2, ... of column c,
  // eight rows' loads before their stores
  {
    constexpr int TPC2 = kPivThreads / NCOLS;
    const int c = tid % NCOLS, part = tid / NCOLS;
    if (c < nb_host) {
      const int pc = c < nb ? sh.pivs[c] : 0;
      for (int a0 = part; a0 < nb_host; a0 += 8 * TPC2) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int a = a0 + u * TPC2;
          const int ar = min(a, bp > 0 ? bp - 1 : 0);
          x[u] = Rraw[(int64_t)ar * ldr + pc];
          x[u] = (a < bp && c >= a && c < nb) ? x[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (a0 + u * TPC2 < nb_host) Rp[(int64_t)(a0 + u * TPC2) * ldp + c] = x[u];
      }
    }
  }
  __syncthreads();
}

}  // namespace rbrp
