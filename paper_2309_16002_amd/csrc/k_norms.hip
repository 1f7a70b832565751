// Initial squared row norms d^(0)_i = ||x_i||^2 (Alg. 2 initialisation) fused
// with the copy R <- X into the padded residual buffer, and the fixed-order
// reduction of per-workgroup partial sums and maxima that drives the stopping
// rule (Alg. 2 loop condition) and the fixed-point sampler scale.
//
// Layout: one wave per row, lanes stride the columns four at a time; the row
// sum is accumulated in FP64 and combined by a butterfly over the wave.
// Every reduction runs in a fixed order, so results are bit-identical from
// run to run.
#include "rbrp_internal.h"

#include <math.h>

#include <algorithm>

namespace rbrp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// VEC (FP32 X with 16-byte aligned rows and n a multiple of 4): each lane's
// four columns are one 16-byte load and one 16-byte store, and all of a
// row's loads (up to four per lane) are issued before any is used.  The
// columns each lane accumulates, and their order, are the same either way.
template <typename TX, typename TRr, bool VEC>
__global__ __launch_bounds__(256) void k_init_norms(
    const TX* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
    TRr* __restrict__ R, int64_t mr, int64_t ldr, double* __restrict__ d,
    double* __restrict__ part_sum, double* __restrict__ part_max,
    int32_t* __restrict__ nonfinite) {
  __shared__ double rs[kNormRowsPerWG];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * kNormRowsPerWG;
  int bad = 0;
  for (int rr = w; rr < kNormRowsPerWG; rr += 4) {
    const int64_t row = row0 + rr;
    double acc = 0.0;
    if (row < mr) {
      const bool live = row < m;
      const TX* xr = X + (live ? row : 0) * ldx;
      TRr* rrow = R ? R + row * ldr : nullptr;
      if constexpr (VEC) {
        typedef float f4_t __attribute__((ext_vector_type(4)));
        for (int64_t c0 = 4 * lane; c0 < ldr; c0 += 16 * kWave) {
          f4_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t c = c0 + u * 4 * kWave;
            const bool in = live && c < n;
            v[u] = *reinterpret_cast<const f4_t*>(xr + (in ? c : 0));
            if (!in) v[u] = (f4_t){0.0f, 0.0f, 0.0f, 0.0f};
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t c = c0 + u * 4 * kWave;
            if (c >= ldr) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double x = (double)v[u][q];
              if (!isfinite(x)) bad = 1;
              acc += x * x;
            }
            if (rrow) {
              if constexpr (sizeof(TRr) == 4) {
                *reinterpret_cast<f4_t*>(rrow + c) = v[u];
              } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) rrow[c + q] = (TRr)v[u][q];
              }
            }
          }
        }
      } else {
        for (int64_t c = 4 * lane; c < ldr; c += 4 * kWave) {
          TX v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t cc = c + q;
            v[q] = (live && cc < n) ? xr[cc] : (TX)0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double x = (double)v[q];
            if (!isfinite(x)) bad = 1;
            acc += x * x;
          }
          if (rrow) {
#pragma unroll
            for (int q = 0; q < 4; ++q) rrow[c + q] = (TRr)v[q];
          }
        }
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      rs[rr] = acc;
      if (row < mr) d[row] = acc;
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, mx = 0.0;
    for (int i = 0; i < kNormRowsPerWG; ++i) {
      s += rs[i];
      mx = fmax(mx, rs[i]);
    }
    part_sum[blockIdx.x] = s;
    part_max[blockIdx.x] = mx;
  }
}

int64_t norms_num_partials(int64_t mr) { return ceil_div(mr, kNormRowsPerWG); }

hipError_t launch_init_norms(const void* X, rbrp_dtype dt, int64_t m, int64_t n,
                             int64_t ldx, void* R, int r_is_f64, int64_t mr,
                             int64_t ldr, double* d, double* part_sum,
                             double* part_max, int32_t* nonfinite,
                             hipStream_t s) {
  const int64_t grid = norms_num_partials(mr);
  if (grid == 0) return hipSuccess;
  if (ldr <= 0) ldr = round_up(n, 4);
  if (dt == RBRP_F64) {
    if (r_is_f64 || !R)
      hipLaunchKernelGGL((k_init_norms<double, double, false>), dim3(grid), dim3(256), 0, s,
                         (const double*)X, m, n, ldx, (double*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
    else
      hipLaunchKernelGGL((k_init_norms<double, float, false>), dim3(grid), dim3(256), 0, s,
                         (const double*)X, m, n, ldx, (float*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
  } else {
    const bool vec = reinterpret_cast<uintptr_t>(X) % 16 == 0 && ldx % 4 == 0 && n % 4 == 0;
    if (r_is_f64 && vec)
      hipLaunchKernelGGL((k_init_norms<float, double, true>), dim3(grid), dim3(256), 0, s,
                         (const float*)X, m, n, ldx, (double*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
    else if (r_is_f64)
      hipLaunchKernelGGL((k_init_norms<float, double, false>), dim3(grid), dim3(256), 0, s,
                         (const float*)X, m, n, ldx, (double*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
    else if (vec)
      hipLaunchKernelGGL((k_init_norms<float, float, true>), dim3(grid), dim3(256), 0, s,
                         (const float*)X, m, n, ldx, (float*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
    else
      hipLaunchKernelGGL((k_init_norms<float, float, false>), dim3(grid), dim3(256), 0, s,
                         (const float*)X, m, n, ldx, (float*)R, mr, ldr, d,
                         part_sum, part_max, nonfinite);
  }
  return hipGetLastError();
}

// Sum / max of max(d_i, 0) over rows not excluded, 2048 rows per workgroup.
__global__ __launch_bounds__(256) void k_masked_partials(
    const double* __restrict__ d, const uint8_t* __restrict__ excluded, int64_t m,
    double* __restrict__ part_sum, double* __restrict__ part_max) {
  __shared__ double ss[4], sm[4];
  const int64_t base = (int64_t)blockIdx.x * 2048;
  double s = 0.0, mx = 0.0;
  for (int q = 0; q < 8; ++q) {
    const int64_t i = base + q * 256 + threadIdx.x;
    if (i < m && !(excluded && excluded[i])) {
      const double v = fmax(d[i], 0.0);
      s += v;
      mx = fmax(mx, v);
    }
  }
  s = wave_sum(s);
  mx = wave_max(mx);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    ss[w] = s;
    sm[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part_sum[blockIdx.x] = ss[0] + ss[1] + ss[2] + ss[3];
    part_max[blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  }
}

int64_t masked_num_partials(int64_t m) { return ceil_div(m, 2048); }

hipError_t launch_masked_partials(const double* d, const uint8_t* excluded,
                                  int64_t m, double* part_sum, double* part_max,
                                  hipStream_t s) {
  const int64_t g = masked_num_partials(m);
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_masked_partials, dim3((unsigned)g), dim3(256), 0, s, d, excluded,
                     m, part_sum, part_max);
  return hipGetLastError();
}

// One workgroup: thread i folds partials i, i+256, ... in order, then a fixed
// binary tree in LDS.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ ps,
                                                const double* __restrict__ pm,
                                                int64_t np, DevScalars* sc,
                                                int set_d0) {
  __shared__ double ss[256];
  __shared__ double sm[256];
  double s = 0.0, mx = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 256) {
    s += ps[i];
    mx = fmax(mx, pm[i]);
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sc->sum_d = ss[0];
    sc->max_d = sm[0];
    if (set_d0) sc->d0 = ss[0];
  }
}

hipError_t launch_reduce(const double* part_sum, const double* part_max,
                         int64_t np, DevScalars* sc, int set_d0, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, part_sum, part_max, np,
                     sc, set_d0);
  return hipGetLastError();
}

// Squared norms of the columns c0 .. c0 + nc - 1 (nc <= 256) of L (m rows,
// row-major, ld ldl).  Threads are (row lane, column) pairs: ncp, the power
// of two >= nc, columns and 256 / ncp row lanes.  Stage 1: workgroup g takes
// the rows [g chunk, (g + 1) chunk), each row lane every (256 / ncp)-th of
// them with eight loads in flight, and the row lanes of a column are added
// in lane order in LDS.  Stage 2 (one workgroup) adds the workgroups'
// partials of each column the same way.  Every sum has a fixed order, so the
// result is bit-identical from run to run.
__device__ __forceinline__ double lanes_in_order(double s, int ncp, double* red) {
  red[threadIdx.x] = s;
  __syncthreads();
  double t = 0.0;
  if ((int)threadIdx.x < ncp)
    for (int q = 0; q < 256 / ncp; ++q) t += red[q * ncp + threadIdx.x];
  return t;
}

template <typename TL>
__global__ __launch_bounds__(256) void k_col_sumsq_part(const TL* __restrict__ L, int64_t ldl,
                                                        int64_t m, int64_t c0, int nc, int ncp,
                                                        int64_t chunk,
                                                        double* __restrict__ part) {
  __shared__ double red[256];
  const int col = threadIdx.x & (ncp - 1), rl = threadIdx.x / ncp, RL = 256 / ncp;
  const int64_t rbeg = (int64_t)blockIdx.x * chunk;
  const int64_t rend = min(m, rbeg + chunk);
  double s = 0.0;
  if (col < nc) {
    const TL* lc = L + c0 + col;
    int64_t r = rbeg + rl;
    for (; r + 7 * RL < rend; r += 8 * RL) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (double)lc[(r + u * RL) * ldl];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u] * v[u];
    }
    for (; r < rend; r += RL) {
      const double v = (double)lc[r * ldl];
      s += v * v;
    }
  }
  const double t = lanes_in_order(s, ncp, red);
  if ((int)threadIdx.x < nc) part[(int64_t)blockIdx.x * nc + threadIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_col_sumsq_final(const double* __restrict__ part,
                                                         int G, int nc, int ncp,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  const int col = threadIdx.x & (ncp - 1), rl = threadIdx.x / ncp, RL = 256 / ncp;
  double s = 0.0;
  if (col < nc) {
    int g = rl;
    for (; g + 7 * RL < G; g += 8 * RL) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(g + u * RL) * nc + col];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; g < G; g += RL) s += part[(int64_t)g * nc + col];
  }
  const double t = lanes_in_order(s, ncp, red);
  if ((int)threadIdx.x < nc) out[threadIdx.x] = t;
}

int col_sumsq_groups(int64_t m) {
  return (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(m, (int64_t)256)));
}

hipError_t launch_col_sumsq(const void* L, int l_f64, int64_t ldl, int64_t m, int64_t c0,
                            int nc, double* part, double* out, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  if (nc > 256 || m <= 0) return hipErrorInvalidValue;
  int ncp = 1;
  while (ncp < nc) ncp <<= 1;
  const int G = col_sumsq_groups(m);
  const int64_t chunk = ceil_div(m, (int64_t)G);
  if (l_f64)
    hipLaunchKernelGGL(k_col_sumsq_part<double>, dim3(G), dim3(256), 0, s, (const double*)L,
                       ldl, m, c0, nc, ncp, chunk, part);
  else
    hipLaunchKernelGGL(k_col_sumsq_part<float>, dim3(G), dim3(256), 0, s, (const float*)L, ldl,
                       m, c0, nc, ncp, chunk, part);
  hipLaunchKernelGGL(k_col_sumsq_final, dim3(1), dim3(256), 0, s, part, G, nc, ncp, out);
  return hipGetLastError();
}

}  // namespace rbrp
