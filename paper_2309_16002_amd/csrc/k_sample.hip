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
#include "rbrp_wg.h"

#include <utility>

namespace rbrp {

// 256 threads x 8 rows per tile, one workgroup per tile.
__global__ __launch_bounds__(256) void k_weights_scan(
    const double* __restrict__ d, const int32_t* __restrict__ sel_block,
    const uint8_t* __restrict__ excluded, int64_t m,
    const DevScalars* __restrict__ sc, uint64_t* __restrict__ cdf_local,
    uint64_t* __restrict__ tile_sum, int32_t* __restrict__ tile_pos) {
  __shared__ uint64_t wsum[4];
  __shared__ int32_t wpos[4];
  wg_weights_scan_tile(d, sel_block, excluded, m, sc->max_d, blockIdx.x, cdf_local, tile_sum,
                       tile_pos, wsum, wpos);
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

constexpr int kMaxTiles = kMaxScanTiles;  // rows up to kMaxRows per decomposition


__global__ __launch_bounds__(kSampleThreads) void k_sample(
    const uint64_t* __restrict__ cdf_local, const uint64_t* __restrict__ tile_sum,
    const int32_t* __restrict__ tile_pos, int64_t m, int32_t b, uint64_t seed,
    uint64_t t, uint64_t ident, int64_t* __restrict__ idx, DevScalars* sc) {
  __shared__ SampleShared<kMaxTiles, kMaxB> sh;
  wg_sample<kMaxTiles, kMaxB>(cdf_local, tile_sum, tile_pos, m, b, seed, t, ident, idx, &sc->nt,
                       &sc->npos, sh);
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

// Greedy top-b selection (Remark 4.3): the b rows not in S with the largest
// positive d, larger value first and equal values by lower row (the order of
// b rounds of argmax).  Positive doubles order like their bit patterns, so
// a row is the key (bits of d_i, i).  Each workgroup bitonic-sorts a chunk
// of kTopChunk keys in LDS and keeps its first b; passes repeat over the
// kept keys until one chunk is left, whose first b (at most the number of
// valid keys) are the selection.  Rows that cannot be chosen get the key
// (0, INT64_MAX), which sorts after every valid one.
constexpr int kTopChunk = 2048;

__device__ __forceinline__ bool key_before(uint64_t va, int64_t ia, uint64_t vb, int64_t ib) {
  return va > vb || (va == vb && ia < ib);
}

template <bool FROM_D>
__global__ __launch_bounds__(256) void k_topb_pass(
    const double* __restrict__ d, const int32_t* __restrict__ sel_block, int64_t m,
    const uint64_t* __restrict__ in_v, const int64_t* __restrict__ in_i, int64_t n_in,
    int32_t b, uint64_t* __restrict__ out_v, int64_t* __restrict__ out_i,
    int64_t* __restrict__ idx, DevScalars* sc) {
  __shared__ uint64_t kv[kTopChunk];
  __shared__ int64_t ki[kTopChunk];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTopChunk;
#pragma unroll
  for (int e = 0; e < kTopChunk / 256; ++e) {
    const int sl = e * 256 + tid;
    const int64_t g = base + sl;
    uint64_t v = 0;
    int64_t i = INT64_MAX;
    if constexpr (FROM_D) {
      if (g < m) {
        const double x = d[g];
        if (x > 0.0 && !(sel_block && sel_block[g] >= 0)) {
          v = (uint64_t)__double_as_longlong(x);
          i = g;
        }
      }
    } else if (g < n_in) {
      v = in_v[g];
      i = in_i[g];
    }
    kv[sl] = v;
    ki[sl] = i;
  }
  __syncthreads();
  for (int k = 2; k <= kTopChunk; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int e = 0; e < kTopChunk / 512; ++e) {
        const int pr = e * 256 + tid;                  // pair index
        const int lo = 2 * j * (pr / j) + (pr % j);    // bit j clear
        const int hi = lo + j;
        const uint64_t va = kv[lo], vb = kv[hi];
        const int64_t ia = ki[lo], ib = ki[hi];
        // runs with bit k clear are put in key order, the others reversed
        const bool swap = ((lo & k) == 0) ? key_before(vb, ib, va, ia)
                                          : key_before(va, ia, vb, ib);
        if (swap) {
          kv[lo] = vb;
          kv[hi] = va;
          ki[lo] = ib;
          ki[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  if (gridDim.x > 1) {
    for (int r = tid; r < b; r += 256) {
      out_v[(int64_t)blockIdx.x * b + r] = kv[r];
      out_i[(int64_t)blockIdx.x * b + r] = ki[r];
    }
    return;
  }
  // final pass: the valid keys come first
  __shared__ int s_n;
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int r = tid; r < b; r += 256)
    if (kv[r] != 0 && (r + 1 == b || kv[r + 1] == 0)) s_n = r + 1;
  __syncthreads();
  const int n = s_n;
  for (int r = tid; r < n; r += 256) idx[r] = ki[r];
  if (tid == 0) {
    sc->nt = n;
    sc->npos = n;
  }
}

// b = 1: the first key in that order is an argmax, found by a reduction
// (each workgroup over its rows, then one workgroup over the workgroups'
// winners).  The order is total on (value, row), so the result does not
// depend on the reduction's shape.
__device__ __forceinline__ void wg_first_key(uint64_t& v, int64_t& i, uint64_t* sv,
                                             int64_t* si) {
  sv[threadIdx.x] = v;
  si[threadIdx.x] = i;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h &&
        key_before(sv[threadIdx.x + h], si[threadIdx.x + h], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + h];
      si[threadIdx.x] = si[threadIdx.x + h];
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
}

__device__ __forceinline__ void top1_write(uint64_t v, int64_t i, int64_t* idx, DevScalars* sc) {
  if (threadIdx.x == 0) {
    const int n = v != 0 ? 1 : 0;
    if (n) idx[0] = i;
    sc->nt = n;
    sc->npos = n;
  }
}

__global__ __launch_bounds__(256) void k_top1_part(const double* __restrict__ d,
                                                   const int32_t* __restrict__ sel_block,
                                                   int64_t m, int64_t chunk,
                                                   uint64_t* __restrict__ out_v,
                                                   int64_t* __restrict__ out_i,
                                                   int64_t* __restrict__ idx, DevScalars* sc) {
  __shared__ uint64_t sv[256];
  __shared__ int64_t si[256];
  const int64_t rbeg = (int64_t)blockIdx.x * chunk;
  const int64_t rend = min(m, rbeg + chunk);
  uint64_t v = 0;
  int64_t i = INT64_MAX;
  for (int64_t g = rbeg + threadIdx.x; g < rend; g += 256) {
    const double x = d[g];
    if (x > 0.0 && !(sel_block && sel_block[g] >= 0)) {
      const uint64_t xv = (uint64_t)__double_as_longlong(x);
      if (key_before(xv, g, v, i)) {
        v = xv;
        i = g;
      }
    }
  }
  wg_first_key(v, i, sv, si);
  if (gridDim.x == 1) {
    top1_write(v, i, idx, sc);
  } else if (threadIdx.x == 0) {
    out_v[blockIdx.x] = v;
    out_i[blockIdx.x] = i;
  }
}

__global__ __launch_bounds__(256) void k_top1_final(const uint64_t* __restrict__ in_v,
                                                    const int64_t* __restrict__ in_i, int G,
                                                    int64_t* __restrict__ idx, DevScalars* sc) {
  __shared__ uint64_t sv[256];
  __shared__ int64_t si[256];
  uint64_t v = 0;
  int64_t i = INT64_MAX;
  for (int g = threadIdx.x; g < G; g += 256)
    if (key_before(in_v[g], in_i[g], v, i)) {
      v = in_v[g];
      i = in_i[g];
    }
  wg_first_key(v, i, sv, si);
  top1_write(v, i, idx, sc);
}

int64_t topb_scratch_words(int64_t m, int32_t b) {
  if (m <= kTopChunk) return 0;
  return 4 * ceil_div(m, (int64_t)kTopChunk) * (int64_t)b;
}

hipError_t launch_topb(const double* d, const int32_t* sel_block, int64_t m,
                       int32_t b, int64_t* idx, DevScalars* sc, uint64_t* scratch,
                       int64_t scratch_words, hipStream_t s) {
  if (b <= 0 || b > kMaxB || m <= 0) return hipErrorInvalidValue;
  if (scratch_words < topb_scratch_words(m, b)) return hipErrorInvalidValue;
  if (b == 1) {
    const int G = (int)ceil_div(m, (int64_t)kTopChunk);   // <= scratch_words / 4
    const int64_t chunk = ceil_div(m, (int64_t)G);
    hipLaunchKernelGGL(k_top1_part, dim3(G), dim3(256), 0, s, d, sel_block, m, chunk, scratch,
                       reinterpret_cast<int64_t*>(scratch + G), idx, sc);
    if (G > 1)
      hipLaunchKernelGGL(k_top1_final, dim3(1), dim3(256), 0, s, (const uint64_t*)scratch,
                         reinterpret_cast<const int64_t*>(scratch + G), G, idx, sc);
    return hipGetLastError();
  }
  // ping-pong halves of the scratch: values then rows, cap keys each
  const int64_t cap = ceil_div(m, (int64_t)kTopChunk) * b;
  uint64_t* v0 = scratch;
  int64_t* i0 = reinterpret_cast<int64_t*>(scratch + cap);
  uint64_t* v1 = scratch + 2 * cap;
  int64_t* i1 = reinterpret_cast<int64_t*>(scratch + 3 * cap);
  int64_t G = ceil_div(m, (int64_t)kTopChunk);
  hipLaunchKernelGGL(k_topb_pass<true>, dim3((unsigned)G), dim3(256), 0, s, d, sel_block, m,
                     (const uint64_t*)nullptr, (const int64_t*)nullptr, (int64_t)0, b, v0, i0,
                     idx, sc);
  int64_t n = G * b;
  while (G > 1) {
    G = ceil_div(n, (int64_t)kTopChunk);
    hipLaunchKernelGGL(k_topb_pass<false>, dim3((unsigned)G), dim3(256), 0, s, d, sel_block,
                       m, (const uint64_t*)v0, (const int64_t*)i0, n, b, v1, i1, idx, sc);
    n = G * b;
    std::swap(v0, v1);
    std::swap(i0, i1);
  }
  return hipGetLastError();
}

}  // namespace rbrp
