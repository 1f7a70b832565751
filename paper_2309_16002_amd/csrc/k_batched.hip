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
// broadcasts.
#include "rbrp_wg.h"

namespace rbrp {

constexpr int kBT = 256;            // threads per workgroup
constexpr int kBatchMaxB = 32;      // block size limit of the batched form
constexpr int kBatchMaxTiles = 8;   // rows per ID <= 8 * kScanTile
constexpr int kBatchMaxN = 256;     // columns per ID
constexpr int kBatchMaxK = 256;     // skeletons per ID

// Per-workgroup scratch geometry (bytes offsets inside one workgroup's slice).
struct BatchGeom {
  int64_t mpad, nmax, kcap, bmax;
  int64_t off_rt, off_d, off_sel, off_cdf, off_tsum, off_tpos, off_qt, off_vt, off_qtmp,
      off_c, off_g, off_rraw, off_rp, off_idx, off_xs2, off_piv, off_l, off_l1, off_linv;
  int64_t slice;   // bytes per workgroup
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
  g.kcap = sh.k_cap_max;
  g.bmax = sh.b_max;
  int64_t off = 0;
  g.off_rt = take(off, g.nmax * g.mpad * ts);
  g.off_d = take(off, g.mpad * 8);
  g.off_sel = take(off, g.mpad * 4);
  g.off_cdf = take(off, g.mpad * 8);
  g.off_tsum = take(off, (kBatchMaxTiles + 1) * 8);
  g.off_tpos = take(off, (kBatchMaxTiles + 1) * 4);
  g.off_qt = take(off, g.kcap * g.nmax * 8);
  g.off_vt = take(off, g.bmax * g.nmax * 8);
  g.off_qtmp = take(off, g.bmax * g.nmax * 8);
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
  return g;
}

struct BatchParams {
  double eps, tau_b;
  uint64_t seed;
  int32_t fixed_rank, refine, count, pad;
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

// A (na rows of length n, row stride ldv) -= Q^T-projection: C = Qt[0:k] A^T,
// A -= C^T Qt[0:k] (FP64).
__device__ __forceinline__ void wg_project(double* __restrict__ A, int64_t ldv, int na,
                                           const double* __restrict__ Qt, int64_t ldq,
                                           int64_t k, int64_t n, double* __restrict__ C) {
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < k * na; e += kBT) {
    const int64_t p = e / na, j = e - p * na;
    const double* q = Qt + p * ldq;
    const double* a = A + j * ldv;
    double s = 0.0;
    for (int64_t c = 0; c < n; ++c) s += q[c] * a[c];
    C[p * na + j] = s;
  }
  __syncthreads();
  for (int64_t e = tid; e < na * n; e += kBT) {
    const int64_t j = e / n, c = e - j * n;
    double v = A[j * ldv + c];
    for (int64_t p = 0; p < k; ++p) v -= C[p * na + j] * Qt[p * ldq + c];
    A[j * ldv + c] = v;
  }
  __syncthreads();
}

// G = A A^T for na rows of A (FP64).
__device__ __forceinline__ void wg_gram(const double* __restrict__ A, int64_t ldv, int na,
                                        int64_t n, double* __restrict__ G, int64_t ldg) {
  for (int e = threadIdx.x; e < na * na; e += kBT) {
    const int i = e / na, j = e - i * na;
    const double* a = A + (int64_t)i * ldv;
    const double* b = A + (int64_t)j * ldv;
    double s = 0.0;
    for (int64_t c = 0; c < n; ++c) s += a[c] * b[c];
    G[(int64_t)i * ldg + j] = s;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_rbrp_batched(
    const rbrp_batch_desc* __restrict__ descs, const int32_t* __restrict__ order,
    BatchParams prm, BatchGeom geom, char* __restrict__ scratch, int32_t* __restrict__ queue,
    int32_t* __restrict__ k_out, int32_t* __restrict__ status_out,
    double* __restrict__ resid_out) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ SampleShared<kBatchMaxTiles> ssh;
  __shared__ PivShared psh;
  __shared__ double red[kBT], red2[kBT];
  __shared__ uint64_t wsum[4];
  __shared__ int32_t wpos[4];
  __shared__ int32_t s_item, s_nt, s_bp, s_stop, s_flag;
  __shared__ double s_sum, s_max, s_tail1;

  const int tid = threadIdx.x;
  const int64_t nmax = geom.nmax, mpad = geom.mpad, kcapw = geom.kcap, bmax = geom.bmax;
  // LDS: Q'^T in the deflation precision (n x bmax), the Schur buffer of the
  // filter ((bmax) x (bmax + 1)), and a per-wave row buffer for W (4 x kcap)
  T* QfT = reinterpret_cast<T*>(dsm);
  double* Ss = reinterpret_cast<double*>(dsm + round_up(nmax * bmax * sizeof(T), 16));
  double* wrow = Ss + bmax * (bmax + 1);

  char* base = scratch + (int64_t)blockIdx.x * geom.slice;
  T* RT = reinterpret_cast<T*>(base + geom.off_rt);
  double* d = reinterpret_cast<double*>(base + geom.off_d);
  int32_t* sel = reinterpret_cast<int32_t*>(base + geom.off_sel);
  uint64_t* cdf = reinterpret_cast<uint64_t*>(base + geom.off_cdf);
  uint64_t* tsum = reinterpret_cast<uint64_t*>(base + geom.off_tsum);
  int32_t* tpos = reinterpret_cast<int32_t*>(base + geom.off_tpos);
  double* Qt = reinterpret_cast<double*>(base + geom.off_qt);
  double* Vt = reinterpret_cast<double*>(base + geom.off_vt);
  double* Qtmp = reinterpret_cast<double*>(base + geom.off_qtmp);
  double* C = reinterpret_cast<double*>(base + geom.off_c);
  double* G = reinterpret_cast<double*>(base + geom.off_g);
  double* Rraw = reinterpret_cast<double*>(base + geom.off_rraw);
  double* Rp = reinterpret_cast<double*>(base + geom.off_rp);
  int64_t* idx = reinterpret_cast<int64_t*>(base + geom.off_idx);
  double* xs2 = reinterpret_cast<double*>(base + geom.off_xs2);
  int32_t* piv = reinterpret_cast<int32_t*>(base + geom.off_piv);
  T* L = reinterpret_cast<T*>(base + geom.off_l);
  double* L1 = reinterpret_cast<double*>(base + geom.off_l1);
  double* Linv = reinterpret_cast<double*>(base + geom.off_linv);

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
    const double tau_b = prm.tau_b > 0.0 ? prm.tau_b : 1.0 / b;
    const double tau = prm.eps * prm.eps;

    // ---- initial norms, R^T <- X^T, skeleton flags ----
    double part = 0.0;
    int bad = 0;
    for (int64_t i = tid; i < m; i += kBT) {
      const T* xr = X + i * ldx;
      double s = 0.0;
      for (int64_t c = 0; c < n; ++c) {
        const T x = xr[c];
        bad |= !isfinite((double)x);
        s += (double)x * (double)x;
        RT[c * mpad + i] = x;
      }
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
      wg_sample<kBatchMaxTiles>(cdf, tsum, tpos, m, bt, prm.seed, (uint64_t)t, (uint64_t)id,
                                idx, &s_nt, nullptr, ssh);
      const int nt = s_nt;
      if (nt <= 0) break;
      // ---- V^T: sampled rows of X in FP64, projected twice against Q ----
      for (int64_t e = tid; e < nt * n; e += kBT) {
        const int64_t j = e / n, c = e - j * n;
        Vt[j * nmax + c] = (double)X[idx[j] * ldx + c];
      }
      __syncthreads();
      if (tid < nt) {
        double s = 0.0;
        for (int64_t c = 0; c < n; ++c) s += Vt[tid * nmax + c] * Vt[tid * nmax + c];
        xs2[tid] = s;
      }
      __syncthreads();
      if (kS > 0) {
        wg_project(Vt, nmax, nt, Qt, nmax, kS, n, C);
        wg_project(Vt, nmax, nt, Qt, nmax, kS, n, C);
      }
      // ---- robust blockwise filter: pivoted Cholesky of V^T V ----
      wg_gram(Vt, nmax, nt, n, G, bmax);
      if (tid == 0) s_stop = 0;
      __syncthreads();
      wg_piv_chol(G, bmax, nt, nullptr, tau_b, xs2, piv, Rraw, bmax, Rp, bmax, &s_bp, &s_tail1,
                  &s_stop, Ss, psh);
      const int bp = s_bp;
      if (s_stop || bp <= 0) break;
      // ---- Q' = V(:, piv(1:b')) R11^{-1}: one thread per column ----
      for (int64_t c = tid; c < n; c += kBT) {
        double q[kBatchMaxB];
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p) {
          if (p < bp) {
            double v = Vt[(int64_t)piv[p] * nmax + c];
#pragma unroll
            for (int r = 0; r < p; ++r) v -= Rp[r * bmax + p] * q[r];
            q[p] = v / Rp[p * bmax + p];
            Qtmp[p * nmax + c] = q[p];
          }
        }
      }
      __syncthreads();
      // ---- reorthogonalisation: project, then Cholesky QR ----
      if (kS > 0) wg_project(Qtmp, nmax, bp, Qt, nmax, kS, n, C);
      wg_gram(Qtmp, nmax, bp, n, G, bmax);
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
      // Qn = R2^{-T} Qtmp into Qt rows kS.., and its copy for the deflation
      for (int64_t c = tid; c < n; c += kBT) {
        double q[kBatchMaxB];
#pragma unroll
        for (int p = 0; p < kBatchMaxB; ++p) {
          if (p < bp) {
            double v = Qtmp[p * nmax + c];
#pragma unroll
            for (int r = 0; r < p; ++r) v -= G[r * bmax + p] * q[r];
            q[p] = v / G[p * bmax + p];
            Qt[(kS + p) * nmax + c] = q[p];
            QfT[c * bmax + p] = (T)q[p];
          }
        }
      }
      // append the kept skeletons
      if (tid < bp) {
        const int64_t row = idx[piv[tid]];
        ds.S[kS + tid] = row;
        sel[row] = t;
      }
      __syncthreads();
      // ---- deflation: P = R Q', L(:, kS:kS+b') = P, R <- R - P Q'^T ----
      for (int64_t i = tid; i < m; i += kBT) {
        T acc[kBatchMaxB];
#pragma unroll
        for (int j = 0; j < kBatchMaxB; ++j) acc[j] = (T)0;
        for (int64_t c = 0; c < n; ++c) {
          const T r = RT[c * mpad + i];
          const T* qc = QfT + c * bmax;
#pragma unroll
          for (int j = 0; j < kBatchMaxB; ++j)
            if (j < bp) acc[j] += r * qc[j];
        }
        const int32_t sb = sel[i];
        const bool earlier = sb >= 0 && sb < t;
        T* lr = L + i * kcapw + kS;
#pragma unroll
        for (int j = 0; j < kBatchMaxB; ++j)
          if (j < bp) lr[j] = earlier ? (T)0 : acc[j];
        double nrm = 0.0;
        for (int64_t c = 0; c < n; ++c) {
          T r = RT[c * mpad + i];
          const T* qc = QfT + c * bmax;
#pragma unroll
          for (int j = 0; j < kBatchMaxB; ++j)
            if (j < bp) r -= acc[j] * qc[j];
          RT[c * mpad + i] = r;
          nrm += (double)r * (double)r;
        }
        d[i] = sb >= 0 ? 0.0 : nrm;
      }
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
        for (int64_t p = j; p < i; ++p) v -= L1[i * k + p] * Linv[p * k + j];
        Linv[i * k + j] = v / L1[i * k + i];
      }
    }
    __syncthreads();
    {
      const int lane = tid & 63, wv = tid >> 6;
      double* wr = wrow + wv * kcapw;          // this wave's row buffer
      constexpr int KS = kBatchMaxK / 64;
      for (int64_t i = wv; i < m; i += kBT / 64) {
        const T* lr = L + i * kcapw;
        double w[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) w[s] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
          const double lp = (double)lr[p];
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const int64_t j = lane + 64 * s;
            if (j < k) w[s] += lp * Linv[p * k + j];
          }
        }
        for (int it = 0; it < prm.refine; ++it) {
          // e = l - w L_1
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const int64_t j = lane + 64 * s;
            if (j < k) wr[j] = w[s];
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          double ev[KS];
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const int64_t p = lane + 64 * s;
            double v = 0.0;
            if (p < k) {
              v = (double)lr[p];
              for (int64_t j = p; j < k; ++j) v -= wr[j] * L1[j * k + p];
            }
            ev[s] = v;
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const int64_t p = lane + 64 * s;
            if (p < k) wr[p] = ev[s];
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          // w += e L_1^{-1}
          for (int64_t p = 0; p < k; ++p) {
            const double ep = wr[p];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int64_t j = lane + 64 * s;
              if (j < k) w[s] += ep * Linv[p * k + j];
            }
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int64_t j = lane + 64 * s;
          if (j < k) ds.W[i * ds.ldw + j] = w[s];
        }
      }
    }
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

static size_t batch_lds_bytes(rbrp_dtype dt, const BatchGeom& g) {
  const size_t ts = dt == RBRP_F64 ? 8 : 4;
  return round_up(g.nmax * g.bmax * ts, 16) + (size_t)g.bmax * (g.bmax + 1) * 8 +
         (size_t)(kBT / 64) * g.kcap * 8;
}

static int default_num_wg() { return 256 * 2; }

size_t batch_workspace_size(rbrp_dtype dt, const rbrp_batch_shape* sh) {
  const BatchGeom g = batch_geom(dt, *sh);
  const int64_t nwg = sh->num_wg > 0 ? sh->num_wg : default_num_wg();
  return 256 + 256 + (size_t)nwg * g.slice;
}

bool batch_shape_ok(const rbrp_batch_shape* sh) {
  return sh && sh->m_max >= 1 && sh->m_max <= (int64_t)kBatchMaxTiles * kScanTile &&
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
  prm.tau_b = o.tau_b;
  prm.seed = seed;
  prm.fixed_rank = o.fixed_rank;
  prm.refine = o.w_refine < 0 ? 1 : o.w_refine;
  prm.count = count;
  prm.pad = 0;
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
