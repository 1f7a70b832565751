// Batched RBRP: many independent small interpolative decompositions (for
// instance the off-diagonal blocks of a hierarchical-matrix compression) in
// one persistent launch.  Each workgroup takes IDs from an atomic queue and
// runs the whole of Alg. 2 and Alg. 3 for one ID before taking the next, so
// the per-block serial steps of many IDs overlap across the chip and no host
// synchronisation is needed (the launch can be captured in a HIP graph).
//
// Per ID the steps are those of the single-ID path, in the same order and
// with the same integer sampler and pivoted-Cholesky filter (shared code):
//   d_i = ||x_i||^2, R <- X; while sum d > eps^2 sum d0: integer CDF, b draws
//   (Philox counter (j, t, id, 0) with id = the ID's index in the batch),
//   V = X(S_t,:)^T projected twice against Q in FP64, Gram + pivoted
//   Cholesky (CPQR pivots, truncation of Remark 4.2), Q' = V(:,piv) R11^{-1}
//   with one Cholesky-QR reorthogonalisation, P = R Q', L(:, new) = P (rows
//   of earlier skeletons zero), R <- R - P Q'^T, d_i = ||R_i||^2 (FP64);
//   then W = L L_1^{-1} with refinement W += (L - W L_1) L_1^{-1} (FP64).
// Sizes are small (m up to a few thousand, n <= 256), so the residual is kept
// transposed (R^T, n x m) in per-workgroup scratch that stays in cache, and
// the products run on the vector ALUs with one thread per row: a thread
// holds its row's b' projections in registers and reads Q' from LDS as
// broadcasts.  With one workgroup per CU there is little other work to hide
// memory latency, so the sampled block lives in LDS for the projections and
// the filter, the small triangular factors of the W solve live in LDS when
// they fit, and every loop over global data loads eight independent values
// before using them.
#include <type_traits>

#include "rbrp_wg.h"

namespace rbrp {

constexpr int kBT = 256;            // threads per workgroup
constexpr int kBatchMaxB = 32;      // block size limit of the batched form
constexpr int kBatchMaxTiles = 8;   // rows per ID <= 8 * kScanTile
constexpr int kBatchMaxN = 256;     // columns per ID
constexpr int kBatchMaxK = 256;     // skeletons per ID
constexpr int kChunk = 8;           // independent loads issued together

// Per-workgroup scratch geometry (byte offsets inside one workgroup's slice)
// and the dynamic LDS layout.  n8 = n_max rounded up to kChunk: R^T and Q
// carry zero columns up to n8 so that chunked loops need no tail.
struct BatchGeom {
  int64_t mpad, nmax, n8, kcap, bmax, bq;   // bq: row stride of Q'^T (bmax rounded to 8)
  int64_t off_rt, off_d, off_sel, off_cdf, off_tsum, off_tpos, off_qt, off_c, off_g,
      off_rraw, off_rp, off_idx, off_xs2, off_piv, off_l, off_l1, off_linv;
  int64_t slice;                    // bytes per workgroup
  int64_t lds_a, lds_q, lds_s, lds_w;  // LDS bytes: block, Q'^T, Schur, row buffers
};

static int64_t take(int64_t& off, int64_t bytes) {
  const int64_t o = off;
  off += round_up(bytes, 256);
  return o;
}

static BatchGeom batch_geom(rbrp_dtype dt, const rbrp_batch_shape& sh) {
  BatchGeom g;
  const int64_t ts = dt == RBRP_F64 ? 8 : 4;
  g.mpad = round_up(sh.m_max, 64);
  g.nmax = sh.n_max;
  g.n8 = round_up(sh.n_max, kChunk);
  g.kcap = sh.k_cap_max;
  g.bmax = sh.b_max;
  g.bq = round_up(sh.b_max, 8);
  int64_t off = 0;
  g.off_rt = take(off, g.n8 * g.mpad * ts);
  g.off_d = take(off, g.mpad * 8);
  g.off_sel = take(off, g.mpad * 4);
  g.off_cdf = take(off, g.mpad * 8);
  g.off_tsum = take(off, (kBatchMaxTiles + 1) * 8);
  g.off_tpos = take(off, (kBatchMaxTiles + 1) * 4);
  g.off_qt = take(off, g.kcap * g.n8 * 8);
  g.off_c = take(off, g.kcap * g.bmax * 8);
  g.off_g = take(off, g.bmax * g.bmax * 8);
  g.off_rraw = take(off, g.bmax * g.bmax * 8);
  g.off_rp = take(off, g.bmax * g.bmax * 8);
  g.off_idx = take(off, g.bmax * 8);
  g.off_xs2 = take(off, g.bmax * 8);
  g.off_piv = take(off, g.bmax * 4);
  g.off_l = take(off, g.mpad * g.kcap * ts);
  g.off_l1 = take(off, g.kcap * g.kcap * 8);
  g.off_linv = take(off, g.kcap * g.kcap * 8);
  g.slice = off;
  g.lds_a = round_up(g.bmax * g.n8 * 8, 16);
  g.lds_q = round_up(g.n8 * g.bq * ts, 16);
  // room for L_1 and L_1^{-1} of the W solve in LDS up to k = 64
  const int64_t kw = g.kcap < 64 ? g.kcap : 64;
  if (g.lds_a + g.lds_q < 2 * kw * kw * 8) g.lds_a = 2 * kw * kw * 8 - g.lds_q;
  g.lds_s = round_up(g.bmax * (g.bmax + 1) * 8, 16);
  g.lds_w = (kBT / 64) * 2 * g.kcap * 8;
  return g;
}

struct BatchParams {
  double eps, tau_b;
  uint64_t seed;
  int32_t fixed_rank, refine, count, row_depth;
};

// Workgroup reduction of (sum, max) over one value per thread, fixed order.
__device__ __forceinline__ void wg_sum_max(double s, double mx, double* red, double* red2,
                                           double* out_s, double* out_m) {
  const int tid = threadIdx.x;
  red[tid] = s;
  red2[tid] = mx;
  __syncthreads();
  for (int h = kBT / 2; h >= 1; h >>= 1) {
    if (tid < h) {
      red[tid] += red[tid + h];
      red2[tid] = fmax(red2[tid], red2[tid + h]);
    }
    __syncthreads();
  }
  *out_s = red[0];
  *out_m = red2[0];
  __syncthreads();
}

// The update As -= C^T Qt of lds_project for na <= NA rows, one thread per
// column (see there).
template <int NA>
__device__ __forceinline__ void lds_project_update(double* __restrict__ As, int na, int64_t n8,
                                                   const double* __restrict__ Qt, int64_t k,
                                                   const double* __restrict__ C,
                                                   double* __restrict__ Cs, int64_t cs_cap) {
  const int tid = threadIdx.x;
  const int64_t P = cs_cap / na > 0 ? cs_cap / na : 1;
  for (int64_t p0 = 0; p0 < k; p0 += P) {
    const int64_t pn = min(P, k - p0);
    for (int64_t e = tid; e < pn * na; e += kBT) Cs[e] = C[p0 * na + e];
    __syncthreads();
    for (int64_t c = tid; c < n8; c += kBT) {
      double v[NA];
#pragma unroll
      for (int j = 0; j < NA; ++j) v[j] = j < na ? As[j * n8 + c] : 0.0;
      for (int64_t pp = 0; pp < pn; pp += kChunk) {
        // kChunk values of Qt in flight (rows past the group clamped, unused)
        double qv[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int64_t pr = p0 + (pp + u < pn ? pp + u : pn - 1);
          qv[u] = Qt[pr * n8 + c];
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          if (pp + u < pn) {
            const double* cr = Cs + (pp + u) * na;
#pragma unroll
            for (int j = 0; j < NA; ++j)
              if (j < na) v[j] -= cr[j] * qv[u];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NA; ++j)
        if (j < na) As[j * n8 + c] = v[j];
    }
    __syncthreads();
  }
}

// Rows of the LDS block As (na rows, stride n8) minus their projection on
// the basis: C = Qt[0:k] As^T (C in global scratch, k x na), As -= C^T Qt.
// Qt rows (stride n8) are zero beyond column n, as are the rows of As.
// The update runs one thread per column (n8 <= kBT): the column's na entries
// stay in registers, each Qt value is loaded once, and C is staged in LDS
// (Cs, cs_cap doubles, free at this point) a group of rows at a time; every
// entry still subtracts its terms in order of p.
__device__ __forceinline__ void lds_project(double* __restrict__ As, int na, int64_t n8,
                                            const double* __restrict__ Qt, int64_t k,
                                            double* __restrict__ C, double* __restrict__ Cs,
                                            int64_t cs_cap) {
  const int tid = threadIdx.x;
  // thread (p, g) forms C[p][jg .. jg + JG - 1], jg = JG g: one pass over
  // row p of Qt serves JG rows of As (rows past na are clamped and unused)
  constexpr int JG = 4;
  const int ngj = (na + JG - 1) / JG;
  for (int64_t e = tid; e < k * ngj; e += kBT) {
    const int64_t p = e / ngj;
    const int jg = (int)(e - p * ngj) * JG;
    const double* q = Qt + p * n8;
    const double* a[JG];
#pragma unroll
    for (int g = 0; g < JG; ++g) a[g] = As + (int64_t)min(jg + g, na - 1) * n8;
    double s0[JG], s1[JG];
#pragma unroll
    for (int g = 0; g < JG; ++g) s0[g] = s1[g] = 0.0;
    // four chunks of Qt in flight per group (the loop is latency-bound:
    // one workgroup per CU), then the remaining chunks one at a time; each
    // entry sums its even and its odd columns in order, then adds the two
    int64_t c0 = 0;
    for (; c0 + 4 * kChunk <= n8; c0 += 4 * kChunk) {
      double qv[4 * kChunk];
#pragma unroll
      for (int u = 0; u < 4 * kChunk; ++u) qv[u] = q[c0 + u];
#pragma unroll
      for (int u = 0; u < 4 * kChunk; u += 2)
#pragma unroll
        for (int g = 0; g < JG; ++g) {
          s0[g] += qv[u] * a[g][c0 + u];
          s1[g] += qv[u + 1] * a[g][c0 + u + 1];
        }
    }
    for (; c0 < n8; c0 += kChunk) {
      double qv[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) qv[u] = q[c0 + u];
#pragma unroll
      for (int u = 0; u < kChunk; u += 2)
#pragma unroll
        for (int g = 0; g < JG; ++g) {
          s0[g] += qv[u] * a[g][c0 + u];
          s1[g] += qv[u + 1] * a[g][c0 + u + 1];
        }
    }
#pragma unroll
    for (int g = 0; g < JG; ++g)
      if (jg + g < na) C[p * na + jg + g] = s0[g] + s1[g];
  }
  __syncthreads();
  if (na <= 4) lds_project_update<4>(As, na, n8, Qt, k, C, Cs, cs_cap);
  else if (na <= 8) lds_project_update<8>(As, na, n8, Qt, k, C, Cs, cs_cap);
  else if (na <= 16) lds_project_update<16>(As, na, n8, Qt, k, C, Cs, cs_cap);
  else lds_project_update<kBatchMaxB>(As, na, n8, Qt, k, C, Cs, cs_cap);
}

// G = As As^T for na rows of the LDS block (global G, stride ldg).
__device__ __forceinline__ void lds_gram(const double* __restrict__ As, int na, int64_t n8,
                                         double* __restrict__ G, int64_t ldg) {
  for (int e = threadIdx.x; e < na * na; e += kBT) {
    const int i = e / na, j = e - i * na;
    const double* a = As + (int64_t)i * n8;
    const double* b = As + (int64_t)j * n8;
    double s0 = 0.0, s1 = 0.0;
    // n8 is a multiple of kChunk: a chunk's LDS loads are issued together
    for (int64_t c0 = 0; c0 < n8; c0 += kChunk) {
#pragma unroll
      for (int u = 0; u < kChunk; u += 2) {
        s0 += a[c0 + u] * b[c0 + u];
        s1 += a[c0 + u + 1] * b[c0 + u + 1];
      }
    }
    G[(int64_t)i * ldg + j] = s0 + s1;
  }
  __syncthreads();
}

// Deflation of the residual by the new basis block, one thread per row:
// P = R Q' (b' <= NBT values in registers), L(i, kS:kS+b') = P (zero on rows
// of earlier skeletons), R <- R - P Q'^T, d_i = ||R_i||^2 (FP64), 0 on
// skeletons.  QfT (LDS) is n8 x bq, zero outside b' columns and n rows.
// CIF: chunks of the row whose loads are issued together in the first pass
// (the depth the autotuner chooses per size class).
template <int NBT, typename T, int CIF>
__device__ __forceinline__ void deflate_rows(T* __restrict__ RT, int64_t mpad, int64_t m,
                                             int64_t n8, const T* __restrict__ QfT,
                                             int64_t bq, T* __restrict__ L, int64_t ldl,
                                             int64_t kS, int bp,
                                             const int32_t* __restrict__ sel, int32_t t,
                                             double* __restrict__ d) {
  for (int64_t i = threadIdx.x; i < m; i += kBT) {
    T acc[NBT];
#pragma unroll
    for (int j = 0; j < NBT; ++j) acc[j] = (T)0;
    // CIF chunks of the row in flight per group (the loop is bound by the
    // latency of its loads), then the remaining chunks one at a time
    int64_t c0 = 0;
    for (; c0 + CIF * kChunk <= n8; c0 += CIF * kChunk) {
      T r[CIF * kChunk];
#pragma unroll
      for (int u = 0; u < CIF * kChunk; ++u) r[u] = RT[(c0 + u) * mpad + i];
#pragma unroll
      for (int u = 0; u < CIF * kChunk; ++u) {
        const T* qc = QfT + (c0 + u) * bq;
#pragma unroll
        for (int j = 0; j < NBT; ++j) acc[j] += r[u] * qc[j];
      }
    }
    for (; c0 < n8; c0 += kChunk) {
      T r[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) r[u] = RT[(c0 + u) * mpad + i];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const T* qc = QfT + (c0 + u) * bq;
#pragma unroll
        for (int j = 0; j < NBT; ++j) acc[j] += r[u] * qc[j];
      }
    }
    const int32_t sb = sel[i];
    const bool earlier = sb >= 0 && sb < t;
    T* lr = L + i * ldl + kS;
#pragma unroll
    for (int j = 0; j < NBT; ++j)
      if (j < bp) lr[j] = earlier ? (T)0 : acc[j];
    double nrm = 0.0;
    // the next chunk is loaded before the current one is updated and stored
    // (another part of the row: no element is read after it is written)
    T r[kChunk], rn[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) r[u] = RT[(int64_t)u * mpad + i];
    for (int64_t c0 = 0; c0 < n8; c0 += kChunk) {
      const int64_t cn = c0 + kChunk < n8 ? c0 + kChunk : c0;
#pragma unroll
      for (int u = 0; u < kChunk; ++u) rn[u] = RT[(cn + u) * mpad + i];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const T* qc = QfT + (c0 + u) * bq;
#pragma unroll
        for (int j = 0; j < NBT; ++j) r[u] -= acc[j] * qc[j];
        RT[(c0 + u) * mpad + i] = r[u];
        nrm += (double)r[u] * (double)r[u];
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) r[u] = rn[u];
    }
    d[i] = sb >= 0 ? 0.0 : nrm;
  }
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_rbrp_batched(
    const rbrp_batch_desc* __restrict__ descs, const int32_t* __restrict__ order,
    BatchParams prm, BatchGeom geom, char* __restrict__ scratch, int32_t* __restrict__ queue,
    int32_t* __restrict__ k_out, int32_t* __restrict__ status_out,
    double* __restrict__ resid_out) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ SampleShared<kBatchMaxTiles, kBatchMaxB> ssh;
  __shared__ PivShared<kBatchMaxB> psh;
  __shared__ double red[kBT], red2[kBT];
  __shared__ uint64_t wsum[4];
  __shared__ int32_t wpos[4];
  __shared__ int32_t s_item, s_nt, s_bp, s_stop, s_flag;
  __shared__ double s_tail1;

  const int tid = threadIdx.x;
  const int64_t nmax = geom.nmax, n8 = geom.n8, mpad = geom.mpad, kcapw = geom.kcap;
  const int64_t bmax = geom.bmax, bq = geom.bq;
  // LDS: the sampled block / new basis rows (bmax x n8, FP64), Q'^T in the
  // deflation precision (n8 x bq), the Schur buffer of the filter, and two
  // row buffers per wave for W.  The first two regions hold L_1 and L_1^{-1}
  // during the W solve when they fit.
  double* As = reinterpret_cast<double*>(dsm);
  T* QfT = reinterpret_cast<T*>(dsm + geom.lds_a);
  double* Ss = reinterpret_cast<double*>(dsm + geom.lds_a + geom.lds_q);
  double* wrow = reinterpret_cast<double*>(dsm + geom.lds_a + geom.lds_q + geom.lds_s);
  // staging of the projection coefficients: the Q'^T, Schur and row-buffer
  // regions, none of which is live during a projection
  double* Cs = reinterpret_cast<double*>(dsm + geom.lds_a);
  const int64_t cs_cap = (geom.lds_q + geom.lds_s + geom.lds_w) / 8;

  char* base = scratch + (int64_t)blockIdx.x * geom.slice;
  T* RT = reinterpret_cast<T*>(base + geom.off_rt);
  double* d = reinterpret_cast<double*>(base + geom.off_d);
  int32_t* sel = reinterpret_cast<int32_t*>(base + geom.off_sel);
  uint64_t* cdf = reinterpret_cast<uint64_t*>(base + geom.off_cdf);
  uint64_t* tsum = reinterpret_cast<uint64_t*>(base + geom.off_tsum);
  int32_t* tpos = reinterpret_cast<int32_t*>(base + geom.off_tpos);
  double* Qt = reinterpret_cast<double*>(base + geom.off_qt);
  double* C = reinterpret_cast<double*>(base + geom.off_c);
  double* G = reinterpret_cast<double*>(base + geom.off_g);
  double* Rraw = reinterpret_cast<double*>(base + geom.off_rraw);
  double* Rp = reinterpret_cast<double*>(base + geom.off_rp);
  int64_t* idx = reinterpret_cast<int64_t*>(base + geom.off_idx);
  double* xs2 = reinterpret_cast<double*>(base + geom.off_xs2);
  int32_t* piv = reinterpret_cast<int32_t*>(base + geom.off_piv);
  T* L = reinterpret_cast<T*>(base + geom.off_l);
  double* L1g = reinterpret_cast<double*>(base + geom.off_l1);
  double* Linvg = reinterpret_cast<double*>(base + geom.off_linv);

  while (true) {
    if (tid == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= prm.count) break;
    const int32_t id = order ? order[item] : item;
    if (id < 0 || id >= prm.count) continue;  // not a permutation: nothing to write to
    const rbrp_batch_desc ds = descs[id];
    const int64_t m = ds.m, n = ds.n, ldx = ds.ldx;
    const int64_t kcap = ds.k_cap;
    const int32_t b = ds.b > 0 ? ds.b : (int32_t)bmax;
    const bool valid = ds.X && ds.S && m >= 1 && n >= 1 && m <= mpad && n <= nmax &&
                       ldx >= n && kcap >= 1 && kcap <= kcapw && kcap <= m && kcap <= n &&
                       b <= bmax && (!ds.W || ds.ldw >= kcap) &&
                       ceil_div(m, kScanTile) <= kBatchMaxTiles;
    if (!valid) {
      if (tid == 0) {
        k_out[id] = 0;
        status_out[id] = RBRP_E_INVALID;
        if (resid_out) resid_out[id] = -1.0;
      }
      continue;
    }
    const T* X = reinterpret_cast<const T*>(ds.X);
    const double tau_b = prm.tau_b < 0.0 ? 1.0 / b : prm.tau_b;
    // the deflation's row-load depth of the ID's size class (n <= 64, <= 128,
    // larger), 4-bit fields; 0 -> 2
    const int cls = n <= 64 ? 0 : (n <= 128 ? 1 : 2);
    int cif = (prm.row_depth >> (4 * cls)) & 15;
    if (cif == 0) cif = 2;
    const double tau = prm.eps * prm.eps;

    // ---- initial norms, R^T <- X^T (zero columns n..n8), skeleton flags ----
    double part = 0.0;
    int bad = 0;
    for (int64_t i = tid; i < m; i += kBT) {
      const T* xr = X + i * ldx;
      double s = 0.0;
      int64_t c0 = 0;
      for (; c0 + kChunk <= n; c0 += kChunk) {
        T xv[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) xv[u] = xr[c0 + u];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          bad |= !isfinite((double)xv[u]);
          s += (double)xv[u] * (double)xv[u];
          RT[(c0 + u) * mpad + i] = xv[u];
        }
      }
      for (; c0 < n; ++c0) {
        const T x = xr[c0];
        bad |= !isfinite((double)x);
        s += (double)x * (double)x;
        RT[c0 * mpad + i] = x;
      }
      for (int64_t c = n; c < n8; ++c) RT[c * mpad + i] = (T)0;
      d[i] = s;
      sel[i] = -1;
      part += s;
    }
    if (tid == 0) s_flag = 0;
    __syncthreads();
    if (bad) atomicOr(&s_flag, 1);
    double D0, dummy;
    wg_sum_max(part, 0.0, red, red2, &D0, &dummy);
    int32_t status = RBRP_OK;
    int64_t kS = 0;
    double sum_d = D0;
    if (s_flag) status = RBRP_E_NONFINITE;
    int32_t t = 0;
    while (status == RBRP_OK && D0 > 0.0) {
      // sum and max of d over the rows not yet selected (selected rows hold 0)
      double ps = 0.0, pm = 0.0;
      for (int64_t i = tid; i < m; i += kBT) {
        const double v = fmax(d[i], 0.0);
        ps += v;
        pm = fmax(pm, v);
      }
      double dmax;
      wg_sum_max(ps, pm, red, red2, &sum_d, &dmax);
      if (kS >= kcap) {
        if (!prm.fixed_rank && sum_d > tau * D0) status = RBRP_E_CAPACITY;
        break;
      }
      if (!prm.fixed_rank && !(sum_d > tau * D0)) break;
      ++t;
      const int32_t bt = (int32_t)((int64_t)b < kcap - kS ? b : kcap - kS);
      // ---- block sampling (exact integer CDF, Philox draws) ----
      const int64_t ntl = ceil_div(m, kScanTile);
      for (int64_t tl = 0; tl < ntl; ++tl)
        wg_weights_scan_tile(d, sel, nullptr, m, dmax, tl, cdf, tsum, tpos, wsum, wpos);
      wg_sample<kBatchMaxTiles, kBatchMaxB>(cdf, tsum, tpos, m, bt, prm.seed, (uint64_t)t, (uint64_t)id,
                                idx, &s_nt, nullptr, ssh);
      const int nt = s_nt;
      if (nt <= 0) break;
      // ---- V^T: sampled rows of X in FP64 (LDS), projected twice against Q ----
      // kChunk elements per thread loaded before any is stored (clamped
      // past the end: the load of a column >= n or an entry past the block
      // reads an element of the block that is in range, and is not used)
      for (int64_t e0 = tid; e0 < nt * n8; e0 += kChunk * kBT) {
        double xv[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int64_t e = min(e0 + u * kBT, (int64_t)nt * n8 - 1);
          const int64_t j = e / n8, c = e - j * n8;
          xv[u] = (double)X[idx[j] * ldx + (c < n ? c : n - 1)];
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int64_t e = e0 + u * kBT;
          if (e < nt * n8) {
            const int64_t c = e % n8;
            As[e] = c < n ? xv[u] : 0.0;
          }
        }
      }
      __syncthreads();
      if (tid < nt) {
        double s = 0.0;
        for (int64_t c0 = 0; c0 < n8; c0 += kChunk) {
#pragma unroll
          for (int u = 0; u < kChunk; ++u) s += As[tid * n8 + c0 + u] * As[tid * n8 + c0 + u];
        }
        xs2[tid] = s;
      }
      __syncthreads();
      if (kS > 0) {
        lds_project(As, nt, n8, Qt, kS, C, Cs, cs_cap);
        lds_project(As, nt, n8, Qt, kS, C, Cs, cs_cap);
      }
      // ---- robust blockwise filter: pivoted Cholesky of V^T V ----
      lds_gram(As, nt, n8, G, bmax);
      if (tid == 0) s_stop = 0;
      __syncthreads();
      wg_piv_chol<kBatchMaxB, false, true>(G, bmax, nt, nullptr, tau_b, xs2, piv, Rraw, bmax,
                                           Rp, bmax, &s_bp, &s_tail1, &s_stop, Ss, psh);
      const int bp = s_bp;
      if (s_stop || bp <= 0) break;
      // ---- Q' = V(:, piv(1:b')) R11^{-1}, in place in As (one thread per
      // column: the column's kept entries are read before any is written) ----
      for (int64_t c = tid; c < n8; c += kBT) {
        double q[kBatchMaxB];
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p)
          if (p < bp) q[p] = As[(int64_t)piv[p] * n8 + c];
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p) {
          if (p < bp) {
            double v = q[p];
#pragma unroll
            for (int r = 0; r < p; ++r) v -= Rp[r * bmax + p] * q[r];
            q[p] = v / Rp[p * bmax + p];
          }
        }
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p)
          if (p < bp) As[p * n8 + c] = q[p];
      }
      __syncthreads();
      // ---- reorthogonalisation: project, then Cholesky QR ----
      if (kS > 0) lds_project(As, bp, n8, Qt, kS, C, Cs, cs_cap);
      lds_gram(As, bp, n8, G, bmax);
      // Cholesky G = R2^T R2 (right-looking, in place in the upper triangle)
      if (tid == 0) s_flag = 0;
      __syncthreads();
      for (int p = 0; p < bp; ++p) {
        const double gpp = G[p * bmax + p];
        if (!(gpp > 0.0)) {
          if (tid == 0) s_flag = 1;
          __syncthreads();
          break;
        }
        const double rpp = sqrt(gpp);
        __syncthreads();
        if (tid > p && tid < bp) G[p * bmax + tid] /= rpp;
        if (tid == p) G[p * bmax + p] = rpp;
        __syncthreads();
        for (int e = tid; e < bp * bp; e += kBT) {
          const int i = e / bp, j = e - i * bp;
          if (i > p && j >= i) G[i * bmax + j] -= G[p * bmax + i] * G[p * bmax + j];
        }
        __syncthreads();
      }
      if (s_flag) {
        status = RBRP_E_HIP;  // the new block lost orthogonality beyond repair
        break;
      }
      // Qn = R2^{-T} Qtmp into Qt rows kS.. (zero beyond column n) and its
      // copy for the deflation (zero beyond b' columns and n rows)
      for (int64_t c = tid; c < n8; c += kBT) {
        double q[kBatchMaxB];
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p) {
          if (p < bp) {
            double v = As[p * n8 + c];
#pragma unroll
            for (int r = 0; r < p; ++r) v -= G[r * bmax + p] * q[r];
            q[p] = c < n ? v / G[p * bmax + p] : 0.0;
            Qt[(kS + p) * n8 + c] = q[p];
          }
        }
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p)
          if (p < bq) QfT[c * bq + p] = p < bp ? (T)q[p] : (T)0;
      }
      // append the kept skeletons
      if (tid < bp) {
        const int64_t row = idx[piv[tid]];
        ds.S[kS + tid] = row;
        sel[row] = t;
      }
      __syncthreads();
      // ---- deflation: P = R Q', L(:, kS:kS+b') = P, R <- R - P Q'^T ----
      const int nbt = (bp + 7) & ~7;
#define RBRP_DEFL(NBV)                                                                     \
  do {                                                                                     \
    if (cif == 1)                                                                          \
      deflate_rows<NBV, T, 1>(RT, mpad, m, n8, QfT, bq, L, kcapw, kS, bp, sel, t, d);      \
    else if (cif == 4)                                                                     \
      deflate_rows<NBV, T, 4>(RT, mpad, m, n8, QfT, bq, L, kcapw, kS, bp, sel, t, d);      \
    else                                                                                   \
      deflate_rows<NBV, T, 2>(RT, mpad, m, n8, QfT, bq, L, kcapw, kS, bp, sel, t, d);      \
  } while (0)
      if (bp <= 1)
        RBRP_DEFL(1);
      else if (bp <= 2)
        RBRP_DEFL(2);
      else if (bp <= 4)
        RBRP_DEFL(4);
      else if (nbt <= 8)
        RBRP_DEFL(8);
      else if (nbt <= 16)
        RBRP_DEFL(16);
      else if (nbt <= 24)
        RBRP_DEFL(24);
      else
        RBRP_DEFL(32);
#undef RBRP_DEFL
      __syncthreads();
      kS += bp;
    }
    // final tracked residual
    {
      double ps = 0.0;
      for (int64_t i = tid; i < m; i += kBT) ps += fmax(d[i], 0.0);
      double dm;
      wg_sum_max(ps, 0.0, red, red2, &sum_d, &dm);
    }
    if (tid == 0) {
      k_out[id] = (int32_t)kS;
      status_out[id] = status;
      if (resid_out) resid_out[id] = D0 > 0.0 ? sqrt(fmax(sum_d, 0.0) / D0) : 0.0;
    }
    if (status != RBRP_OK && status != RBRP_E_CAPACITY) continue;
    const int64_t k = kS;
    if (!ds.W || k == 0) continue;

    // ---- W = L L_1^{-1}, one refinement step per prm.refine, W(S,:) = I ----
    const bool wl = 2 * k * k * 8 <= geom.lds_a + geom.lds_q;
    // one copy of the solve per memory space of L_1 and L_1^{-1} (LDS when
    // they fit, else global scratch), so that every access compiles to an
    // LDS or a global instruction rather than a generic one
    auto w_solve = [&](double* L1, double* Linv) {
      for (int64_t e = tid; e < k * k; e += kBT) {
        const int64_t j = e / k, p = e - j * k;
        L1[e] = (p <= j) ? (double)L[ds.S[j] * kcapw + p] : 0.0;
      }
      __syncthreads();
      if (tid < k) {  // column tid of L_1^{-1} by forward substitution
        const int64_t j = tid;
        for (int64_t i = 0; i < j; ++i) Linv[i * k + j] = 0.0;
        for (int64_t i = j; i < k; ++i) {
          double v = (i == j) ? 1.0 : 0.0;
  #pragma unroll 8
          for (int64_t p = j; p < i; ++p) v -= L1[i * k + p] * Linv[p * k + j];
          Linv[i * k + j] = v / L1[i * k + i];
        }
      }
      __syncthreads();
      {
        const int lane = tid & 63, wv = tid >> 6;
        double* wl_row = wrow + wv * 2 * kcapw;   // this wave's copy of the row of L
        double* wbuf = wl_row + kcapw;            // and of w, then of the residual e
        // KS 64-column slots per lane, ceil(k / 64) of them: no slot's loads
        // and FMAs issue fully masked (the sums and their order are the
        // same for every KS that covers k)
        auto rows_pass = [&](auto ks_tag) {
          constexpr int KS = decltype(ks_tag)::value;
          // the row of L is loaded one row ahead (clamped to row m - 1 past
          // the end), so that its load overlaps the previous row's products
          T lnext[KS];
          auto load_row = [&](int64_t r) {
            const T* lr = L + (r < m ? r : m - 1) * kcapw;
    #pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int64_t p = lane + 64 * s;
              lnext[s] = lr[p < k ? p : k - 1];
            }
          };
          load_row(wv);
          for (int64_t i = wv; i < m; i += kBT / 64) {
    #pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int64_t p = lane + 64 * s;
              if (p < k) wl_row[p] = (double)lnext[s];
            }
            load_row(i + kBT / 64);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            double w[KS];
    #pragma unroll
            for (int s = 0; s < KS; ++s) w[s] = 0.0;
            // w = l L_1^{-1}, four p per group: the group's loads are all
            // issued before its FMAs (L_1^{-1} may be in global memory);
            // each w[s] still sums over p in order
            auto row_times_inv = [&](const double* lv) {
              int64_t p = 0;
              for (; p + 4 <= k; p += 4) {
                double a4[4], iv[4][KS];
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                  a4[u] = lv[p + u];
    #pragma unroll
                  for (int s = 0; s < KS; ++s) {
                    const int64_t j = lane + 64 * s;
                    iv[u][s] = 0.0;
                    if (j < k) iv[u][s] = Linv[(p + u) * k + j];
                  }
                }
    #pragma unroll
                for (int u = 0; u < 4; ++u)
    #pragma unroll
                  for (int s = 0; s < KS; ++s) w[s] += a4[u] * iv[u][s];
              }
              for (; p < k; ++p) {
                const double a = lv[p];
    #pragma unroll
                for (int s = 0; s < KS; ++s) {
                  const int64_t j = lane + 64 * s;
                  if (j < k) w[s] += a * Linv[p * k + j];
                }
              }
            };
            row_times_inv(wl_row);
            for (int it = 0; it < prm.refine; ++it) {
              // e = l - w L_1
    #pragma unroll
              for (int s = 0; s < KS; ++s) {
                const int64_t j = lane + 64 * s;
                if (j < k) wbuf[j] = w[s];
              }
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              double ev[KS];
    #pragma unroll
              for (int s = 0; s < KS; ++s) {
                const int64_t p = lane + 64 * s;
                double v = 0.0;
                if (p < k) {
                  v = wl_row[p];
                  int64_t j = p;
                  for (; j + 4 <= k; j += 4) {
                    double wv4[4], l4[4];
    #pragma unroll
                    for (int u = 0; u < 4; ++u) {
                      wv4[u] = wbuf[j + u];
                      l4[u] = L1[(j + u) * k + p];
                    }
    #pragma unroll
                    for (int u = 0; u < 4; ++u) v -= wv4[u] * l4[u];
                  }
                  for (; j < k; ++j) v -= wbuf[j] * L1[j * k + p];
                }
                ev[s] = v;
              }
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    #pragma unroll
              for (int s = 0; s < KS; ++s) {
                const int64_t p = lane + 64 * s;
                if (p < k) wbuf[p] = ev[s];
              }
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              // w += e L_1^{-1}
              row_times_inv(wbuf);
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
    #pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int64_t j = lane + 64 * s;
              if (j < k) ds.W[i * ds.ldw + j] = w[s];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          }
        };
        const int ksn = (int)((k + 63) >> 6);
        if (ksn <= 1) rows_pass(std::integral_constant<int, 1>());
        else if (ksn == 2) rows_pass(std::integral_constant<int, 2>());
        else if (ksn == 3) rows_pass(std::integral_constant<int, 3>());
        else rows_pass(std::integral_constant<int, 4>());
      }
    };
    if (wl) w_solve(As, As + k * k);
    else w_solve(L1g, Linvg);
    __syncthreads();
    for (int64_t e = tid; e < k * k; e += kBT) {
      const int64_t j = e / k, c = e - j * k;
      ds.W[ds.S[j] * ds.ldw + c] = (c == j) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
}

__global__ void k_batch_queue_reset(int32_t* q) {
  if (threadIdx.x == 0) *q = 0;
}

static size_t batch_lds_bytes(rbrp_dtype, const BatchGeom& g) {
  return (size_t)(g.lds_a + g.lds_q + g.lds_s + g.lds_w);
}

static int default_num_wg() { return 256 * 2; }

size_t batch_workspace_size(rbrp_dtype dt, const rbrp_batch_shape* sh) {
  const BatchGeom g = batch_geom(dt, *sh);
  const int64_t nwg = sh->num_wg > 0 ? sh->num_wg : default_num_wg();
  return 256 + 256 + (size_t)nwg * g.slice;
}

int32_t batch_default_wg() { return default_num_wg(); }

int64_t batch_max_wg(rbrp_dtype dt, const rbrp_batch_shape* sh, size_t bytes) {
  const BatchGeom g = batch_geom(dt, *sh);
  if (g.slice <= 0 || bytes < 512 + (size_t)g.slice) return 0;
  return (int64_t)((bytes - 512) / (size_t)g.slice);
}

static bool row_depth_ok(int32_t code) {
  if (code < 0 || code >= (1 << 12)) return false;
  for (int c = 0; c < 3; ++c) {
    const int v = (code >> (4 * c)) & 15;
    if (v != 0 && v != 1 && v != 2 && v != 4) return false;
  }
  return true;
}

bool batch_shape_ok(const rbrp_batch_shape* sh) {
  return sh && row_depth_ok(sh->row_depth) && sh->m_max >= 1 && sh->m_max <= (int64_t)kBatchMaxTiles * kScanTile &&
         sh->n_max >= 1 && sh->n_max <= kBatchMaxN && sh->b_max >= 1 &&
         sh->b_max <= kBatchMaxB && sh->k_cap_max >= 1 && sh->k_cap_max <= kBatchMaxK &&
         sh->num_wg >= 0 && sh->num_wg <= 65536;
}

hipError_t launch_batched(const rbrp_batch_desc* descs, const int32_t* order, int32_t count,
                          rbrp_dtype dt, double eps, uint64_t seed, const rbrp_options& o,
                          const rbrp_batch_shape& sh, int32_t* k_out, int32_t* status_out,
                          double* resid_out, void* workspace, hipStream_t s) {
  const BatchGeom g = batch_geom(dt, sh);
  const int64_t nwg = sh.num_wg > 0 ? sh.num_wg : default_num_wg();
  char* ws = (char*)(((uintptr_t)workspace + 255) / 256 * 256);
  int32_t* queue = reinterpret_cast<int32_t*>(ws);
  char* scratch = ws + 256;
  BatchParams prm;
  prm.eps = eps;
  prm.row_depth = sh.row_depth;
  prm.tau_b = o.tau_b;
  prm.seed = seed;
  prm.fixed_rank = o.fixed_rank;
  prm.refine = o.w_refine < 0 ? 1 : o.w_refine;
  prm.count = count;
  const size_t lds = batch_lds_bytes(dt, g);
  hipLaunchKernelGGL(k_batch_queue_reset, dim3(1), dim3(64), 0, s, queue);
  if (dt == RBRP_F64) {
    static bool attr = false;
    if (!attr) {
      hipError_t e = hipFuncSetAttribute((const void*)k_rbrp_batched<double>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         128 * 1024);
      if (e != hipSuccess) return e;
      attr = true;
    }
    hipLaunchKernelGGL(k_rbrp_batched<double>, dim3((unsigned)nwg), dim3(kBT), lds, s, descs,
                       order, prm, g, scratch, queue, k_out, status_out, resid_out);
  } else {
    static bool attr = false;
    if (!attr) {
      hipError_t e = hipFuncSetAttribute((const void*)k_rbrp_batched<float>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         128 * 1024);
      if (e != hipSuccess) return e;
      attr = true;
    }
    hipLaunchKernelGGL(k_rbrp_batched<float>, dim3((unsigned)nwg), dim3(kBT), lds, s, descs,
                       order, prm, g, scratch, queue, k_out, status_out, resid_out);
  }
  return hipGetLastError();
}

size_t batch_lds_needed(rbrp_dtype dt, const rbrp_batch_shape* sh) {
  return batch_lds_bytes(dt, batch_geom(dt, *sh));
}

}  // namespace rbrp
