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

constexpr int kMaxTiles = 4096;  // rows up to 4096 * 2048 per decomposition


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
