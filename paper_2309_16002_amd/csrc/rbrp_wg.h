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

// LDS state of the block sampler (one workgroup of kSampleThreads threads).
template <int MAXTILES, int MAXB>
struct SampleShared {
  uint64_t tile_excl[MAXTILES + 1];
  int64_t acc_idx[MAXB];
  uint64_t acc_w[MAXB];
  int64_t cand[kSampleThreads];
  int32_t flag[kSampleThreads];
  uint64_t red[kSampleThreads];
  int32_t nacc, npos, total_new;
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
  int32_t& s_total_new = sh.total_new;
  uint64_t& s_W = sh.W;
  uint64_t* tile_excl = sh.tile_excl;
  int64_t* acc_idx = sh.acc_idx;
  uint64_t* acc_w = sh.acc_w;
  int64_t* cand = sh.cand;
  int32_t* flag = sh.flag;
  uint64_t* red = sh.red;
  const int tid = threadIdx.x;
  const int64_t ntiles = ceil_div(m, kScanTile);

  // exclusive prefix of tile totals (serial: ntiles is small)
  if (tid == 0) {
    uint64_t run = 0;
    int npos = 0;
    for (int64_t T = 0; T < ntiles; ++T) {
      tile_excl[T] = run;
      run += tile_sum[T];
      npos += tile_pos[T];
    }
    tile_excl[ntiles] = run;
    s_W = run;
    s_npos = npos;
    s_nacc = 0;
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
        flag[tid] = pos;
        __syncthreads();
        if (tid == 0) {
          int run = nacc;
          for (int q = 0; q < kSampleThreads; ++q) {
            const int f = flag[q];
            flag[q] = run;
            run += f;
          }
          s_total_new = run;
        }
        __syncthreads();
        if (pos) idx[flag[tid]] = i;
        nacc = s_total_new;
        __syncthreads();
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
      int64_t a = lo * kScanTile, z = min(m, (lo + 1) * (int64_t)kScanTile) - 1;
      while (a < z) {
        const int64_t mid = (a + z) >> 1;
        if (cdf_local[mid] > local) z = mid; else a = mid + 1;
      }
      my = a;
    }
    cand[tid] = my;
    __syncthreads();
    int isnew = 0;
    if (my >= 0) {
      isnew = 1;
      for (int q = 0; q < nacc && isnew; ++q) isnew = acc_idx[q] != my;
      for (int q = 0; q < tid && isnew; ++q) isnew = cand[q] != my;
    }
    flag[tid] = isnew;
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int q = 0; q < kSampleThreads; ++q) {
        const int f = flag[q];
        flag[q] = run;
        run += f;
      }
      s_total_new = run;
    }
    __syncthreads();
    if (isnew) {
      const int p = nacc + flag[tid];
      if (p < b) {
        acc_idx[p] = my;
        acc_w[p] = weight_at(cdf_local, my);
      }
    }
    __syncthreads();
    if (tid == 0) s_nacc = min(b, nacc + s_total_new);
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

// LDS state of the pivoted Cholesky (besides the Schur complement itself).
constexpr int kPivKB = 16;   // pivot rows per delayed Schur-complement update
constexpr int kPivLd = 18;   // row stride (doubles) of the transposed pivot rows
constexpr int kPivThreads = 256;

template <int NBMAX>
struct PivShared {
  double rblk[NBMAX][kPivLd];  // rblk[c][q]: entry c of pivot row q of the current group
  int32_t chosen[NBMAX];
  int32_t pivs[NBMAX];
  double wbest[2][4], wsum[2][4], gdiag[2];
  int32_t wbi[2][4];
};

// Cholesky of the block's Gram matrix G (nb x nb, nb <= NBMAX <= kPivThreads)
// by kPivThreads threads: pivoted (PIVOTED, the filter: pivot = largest
// remaining Schur diagonal, ties to the lower index, stop at the truncation
// threshold) or in natural order (the reorthogonalisation pass).
//
// Thread c < nb owns column c of the Schur complement S: it keeps the exact
// diagonal S[c][c] in a register, downdated at every step, and is the only
// thread that reads or writes column c of S.  S is brought up to date only
// once per group of kPivKB steps (a rank-kPivKB update of the owned column
// with the group's pivot rows, the delayed update of blocked pivoted
// Cholesky); inside a group the pivot row is formed from the last update
// plus the corrections of the group's earlier pivots.  S lives in LDS (GS
// false: copied from G, row stride nb + 1) or in global memory (GS true: S is
// G itself, updated in place).  One barrier per step (two at a group's
// first step); the per-step argmax and the sum of the diagonal are wave-level
// DPP reductions folded across waves in a fixed order.
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
    int32_t* __restrict__ stop_out, double* __restrict__ S, PivShared<NBMAX>& sh) {
  static_assert(NBMAX <= kPivThreads, "one thread per column");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  int nb = nb_host;
  if (nb_dev) nb = min(nb, *nb_dev);
  const int64_t ld = GS ? ldg : nb + 1;
  if constexpr (!GS) {
    for (int e = tid; e < nb * nb; e += kPivThreads) {
      const int r = e / nb, c = e - r * nb;
      S[r * ld + c] = G[(int64_t)r * ldg + c];
    }
  }
  if (tid < NBMAX) sh.chosen[tid] = (tid < nb) ? 0 : 1;
  __syncthreads();
  const bool owner = tid < nb;
  double dj = owner ? S[(int64_t)tid * ld + tid] : 0.0;
  bool chosen = !owner;
  const int nwv = (nb + 63) >> 6;
  double rown[kPivKB];
#pragma unroll
  for (int q = 0; q < kPivKB; ++q) rown[q] = 0.0;
  double thr = 0.0;
  int bp = 0;
  for (int g = 0;; ++g) {
    bool fin = false;
#pragma unroll
    for (int qb = 0; qb < kPivKB; ++qb) {
      const int p = g * kPivKB + qb;
      const int par = p & 1;
      if (wv < nwv) {
        double best = chosen ? -INFINITY : dj;
        int bi = chosen ? -1 : tid;
        double sum = chosen ? 0.0 : fmax(dj, 0.0);
        wave_argmax_sum(best, bi, sum);
        if (lane == 0) {
          sh.wbest[par][wv] = best;
          sh.wbi[par][wv] = bi;
          sh.wsum[par][wv] = sum;
        }
      }
      if (!PIVOTED && tid == p) sh.gdiag[par] = dj;
      __syncthreads();
      double best = sh.wbest[par][0];
      int bi = sh.wbi[par][0];
      double tail = sh.wsum[par][0];
      for (int w2 = 1; w2 < nwv; ++w2) {
        tail += sh.wsum[par][w2];
        if (piv_better(sh.wbest[par][w2], sh.wbi[par][w2], best, bi)) {
          best = sh.wbest[par][w2];
          bi = sh.wbi[par][w2];
        }
      }
      bool done = false;
      if (PIVOTED && p == 0) {
        thr = tau_b * tail * (1.0 - 4.0 * nb * 1.1102230246251565e-16);
        if (tid == 0 && tail1_out) *tail1_out = tail;
        if (xs2_rows) {
          double xs2 = 0.0;
          for (int q = 0; q < nb; ++q) xs2 += xs2_rows[q];
          if (!(tail > 1e-26 * xs2)) {
            done = true;
            if (stop_out && tid == 0) *stop_out = 1;
          }
        }
      }
      int jp = bi;
      double gv = best;
      if (!PIVOTED) {
        jp = p;
        gv = p < nb ? sh.gdiag[par] : 0.0;
      }
      if (p >= nb || jp < 0 || !(gv > 0.0)) done = true;
      if (PIVOTED && p > 0 && tail < thr) done = true;
      if (done) {
        bp = p;
        fin = true;
        break;
      }
      if (qb == 0 && g > 0) {
        // delayed update of the owned column by the previous group's pivot rows
        if (owner && !chosen) {
          constexpr int RU = GS ? 8 : 4;
          for (int i0 = 0; i0 < nb; i0 += RU) {
            double a[RU];
            bool live[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
              const int i = i0 + u;
              live[u] = i < nb && !sh.chosen[i];
              a[u] = S[(int64_t)(live[u] ? i : tid) * ld + tid];
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
              if (!live[u]) continue;
              const double* ri = sh.rblk[i0 + u];
              double s0 = 0.0, s1 = 0.0;
#pragma unroll
              for (int q = 0; q < kPivKB; q += 2) {
                s0 += ri[q] * rown[q];
                s1 += ri[q + 1] * rown[q + 1];
              }
              S[(int64_t)(i0 + u) * ld + tid] = a[u] - (s0 + s1);
            }
          }
        }
        __syncthreads();
      }
      const double r = sqrt(gv);
      double v = 0.0;
      if (owner) {
        if (tid == jp) {
          v = r;
        } else if (!chosen) {
          double a = S[(int64_t)jp * ld + tid];
          const double* rj = sh.rblk[jp];
#pragma unroll
          for (int q = 0; q < qb; ++q) a -= rj[q] * rown[q];
          v = a / r;
        }
        sh.rblk[tid][qb] = v;
        Rraw[(int64_t)p * ldr + tid] = v;
        if (tid == jp) {
          chosen = true;
          sh.chosen[tid] = 1;
          sh.pivs[p] = jp;
        }
        dj -= v * v;
      }
      rown[qb] = v;
    }
    if (fin) break;
  }
  if (tid == 0) {
    int q = bp;
    for (int c = 0; c < nb; ++c)
      if (!sh.chosen[c]) sh.pivs[q++] = c;
    *bprime_out = bp;
  }
  __syncthreads();
  if (tid < nb) piv[tid] = sh.pivs[tid];
  // R11 in pivoted order, zero outside the leading b' x b' upper triangle
  for (int e = tid; e < nb_host * nb_host; e += kPivThreads) {
    const int a = e / nb_host, c = e - a * nb_host;
    double v = 0.0;
    if (a < bp && c >= a && c < nb) v = Rraw[(int64_t)a * ldr + sh.pivs[c]];
    Rp[(int64_t)a * ldp + c] = v;
  }
  __syncthreads();
}

}  // namespace rbrp
