// Block sampling of Alg. 2: b rows drawn without replacement from the
// residual squared-norm distribution d / ||d||_1.
//
// Probabilities are exact integers: with max d = f 2^e (f in [0.5, 1)) and
// s = 62 - e - ceil(log2 m), row i weighs w_i = floor(max(d_i, 0) 2^s) (zero
// for rows already in S), so the prefix sums are exact in uint64 and every
// draw is bit-reproducible.  Candidate j draws word 0 of
// Philox4x64-10(counter (j, t, id, 0), key (seed, 0)) (Salmon et al., SC'11),
// maps it to target = floor(x W / 2^64) and picks the smallest i with
// C_i > target.  First occurrences are accepted (successive sampling); after
// 32 b candidates the accepted rows are removed from the CDF and each further
// candidate is accepted.  With at most b positive weights, all positive rows
// are taken in index order.
//
// Kernels: (1) weights + per-tile inclusive scan, one workgroup per 2048
// rows; (2) one workgroup that scans the tile totals in LDS and resolves all
// candidates of a chunk in parallel (two-level binary search), then
// de-duplicates them in candidate order.
#include "rbrp_internal.h"

#include <math.h>

namespace rbrp {

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

// 256 threads x 8 rows per tile.
__global__ __launch_bounds__(256) void k_weights_scan(
    const double* __restrict__ d, const int32_t* __restrict__ sel_block,
    const uint8_t* __restrict__ excluded, int64_t m,
    const DevScalars* __restrict__ sc, uint64_t* __restrict__ cdf_local,
    uint64_t* __restrict__ tile_sum, int32_t* __restrict__ tile_pos) {
  __shared__ uint64_t wsum[4];
  __shared__ int32_t wpos[4];
  const double dmax = sc->max_d;
  const int s = dmax > 0.0 ? weight_shift(dmax, m) : 0;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
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
    tile_sum[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    tile_pos[blockIdx.x] = wpos[0] + wpos[1] + wpos[2] + wpos[3];
  }
}

int64_t scan_num_tiles(int64_t m) { return ceil_div(m, kScanTile); }

hipError_t launch_weights_scan(const double* d, const int32_t* sel_block,
                               const uint8_t* excluded, int64_t m,
                               const DevScalars* sc, uint64_t* cdf_local,
                               uint64_t* tile_sum, int32_t* tile_pos,
                               hipStream_t s) {
  const int64_t tiles = scan_num_tiles(m);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_weights_scan, dim3(tiles), dim3(256), 0, s, d, sel_block,
                     excluded, m, sc, cdf_local, tile_sum, tile_pos);
  return hipGetLastError();
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

constexpr int kMaxTiles = 4096;  // rows up to 4096 * 2048 per decomposition
constexpr int kSampleThreads = 256;

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

__global__ __launch_bounds__(kSampleThreads) void k_sample(
    const uint64_t* __restrict__ cdf_local, const uint64_t* __restrict__ tile_sum,
    const int32_t* __restrict__ tile_pos, int64_t m, int32_t b, uint64_t seed,
    uint64_t t, uint64_t ident, int64_t* __restrict__ idx, DevScalars* sc) {
  __shared__ uint64_t tile_excl[kMaxTiles + 1];
  __shared__ int64_t acc_idx[kMaxB];
  __shared__ uint64_t acc_w[kMaxB];
  __shared__ int64_t cand[kSampleThreads];
  __shared__ int32_t flag[kSampleThreads];
  __shared__ uint64_t red[kSampleThreads];
  __shared__ int32_t s_nacc, s_npos, s_total_new;
  __shared__ uint64_t s_W;
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
      sc->nt = nacc;
      sc->npos = npos;
    }
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
    sc->nt = nt;
    sc->npos = npos;
  }
}

hipError_t launch_sample(const uint64_t* cdf_local, const uint64_t* tile_sum,
                         const int32_t* tile_pos, int64_t m, int32_t b,
                         uint64_t seed, uint64_t t, uint64_t ident,
                         int64_t* idx, DevScalars* sc, hipStream_t s) {
  if (scan_num_tiles(m) > kMaxTiles || b > kMaxB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sample, dim3(1), dim3(kSampleThreads), 0, s, cdf_local,
                     tile_sum, tile_pos, m, b, seed, t, ident, idx, sc);
  return hipGetLastError();
}

// Greedy top-b selection (Remark 4.3): b rounds of a fixed-order argmax over
// the rows not yet in S and not yet chosen; equal values go to the lower index.
__global__ __launch_bounds__(256) void k_topb(const double* __restrict__ d,
                                              const int32_t* __restrict__ sel_block,
                                              int64_t m, int32_t b,
                                              int64_t* __restrict__ idx,
                                              DevScalars* sc) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  __shared__ int64_t chosen[kMaxB];
  __shared__ int s_n;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int r = 0; r < b; ++r) {
    const int nch = s_n;
    double best = 0.0;
    int64_t besti = -1;
    for (int64_t i = tid; i < m; i += 256) {
      const double v = d[i];
      if (!(v > 0.0) || (sel_block && sel_block[i] >= 0)) continue;
      bool taken = false;
      for (int q = 0; q < nch; ++q) taken |= chosen[q] == i;
      if (taken) continue;
      if (v > best) { best = v; besti = i; }
    }
    bv[tid] = best;
    bi[tid] = besti;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (tid < h) {
        const double v2 = bv[tid + h];
        const int64_t i2 = bi[tid + h];
        if (i2 >= 0 && (bi[tid] < 0 || v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid]))) {
          bv[tid] = v2;
          bi[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0 && bi[0] >= 0) {
      chosen[nch] = bi[0];
      s_n = nch + 1;
    }
    __syncthreads();
    if (s_n == nch) break;
  }
  const int n = s_n;
  for (int q = tid; q < n; q += 256) idx[q] = chosen[q];
  if (tid == 0) {
    sc->nt = n;
    sc->npos = n;
  }
}

hipError_t launch_topb(const double* d, const int32_t* sel_block, int64_t m,
                       int32_t b, int64_t* idx, DevScalars* sc, hipStream_t s) {
  if (b > kMaxB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_topb, dim3(1), dim3(256), 0, s, d, sel_block, m, b, idx, sc);
  return hipGetLastError();
}

}  // namespace rbrp
