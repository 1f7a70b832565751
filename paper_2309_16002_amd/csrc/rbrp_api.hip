// C ABI of the RBRP library: argument validation, workspace layout, and the
// host loop of Algorithm 2 (one stop test per block), followed by
// Algorithm 3 for W.
#include "rbrp_internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

using namespace rbrp;

namespace {

constexpr size_t kAlign = 256;

struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Plan {
  rbrp_dtype dt;
  int64_t m, n, mr, ldr, k_max, ldl, ntiles, nparts;
  int32_t b;
  int32_t bdef;      // columns of one deflation launch: min(b, kDeflateMaxB)
  int native_mode;   // deflation mode of the NATIVE precision
  bool bf16;
  bool r_f64;
  int32_t refine;    // refinement steps of the W solve
  bool w_pinv;       // W through the truncated-SVD pseudo-inverse of L_1
};

struct Work {
  DevScalars* sc;
  void* R;
  void* R16;   // BF16 residual of the BF16 form (permuted 32-column groups)
  double* d;
  double* part_sum;
  double* part_max;
  int32_t* sel_block;
  uint64_t* cdf;
  uint64_t* tile_sum;
  int32_t* tile_pos;
  int64_t* idx;
  double* xs2;
  double* Vt;
  double* C;
  double* G;
  int32_t* piv;
  int32_t* piv2;
  double* Rraw;
  double* R2raw;
  double* Mc;
  double* Mc2;
  double* Rinv;
  double* Qtmp;
  double* Qt;
  void* fragB1;
  void* fragA2;
  void* fragB1b;   // the second half of blocks wider than kDeflateMaxB
  void* fragA2b;
  void* L;
  double* interp;
};

void fill_defaults(rbrp_options* o) {
  memset(o, 0, sizeof(*o));
  o->tau_b = -1.0;
  o->k_max = 0;
  o->fixed_rank = 0;
  o->greedy = 0;
  o->precision = RBRP_PREC_NATIVE;
  o->w_refine = -1;
  o->theta = 0.0;
}

bool make_plan(rbrp_dtype dt, int64_t m, int64_t n, int32_t b, const rbrp_options* opt,
               Plan* p) {
  if (dt != RBRP_F32 && dt != RBRP_F64) return false;
  if (m <= 0 || n <= 0 || b < 1 || b > kMaxB) return false;
  if (m > kMaxRows) return false;   // the sampler's integer CDF tiles
  rbrp_options o;
  if (opt) o = *opt; else fill_defaults(&o);
  if (o.precision != RBRP_PREC_NATIVE && o.precision != RBRP_PREC_BF16) return false;
  if (!(o.tau_b <= 1.0)) return false;   // NaN or above 1
  p->dt = dt;
  p->m = m;
  p->n = n;
  p->b = b;
  p->bdef = b < kDeflateMaxB ? b : kDeflateMaxB;
  p->mr = round_up(m, kRowPad);
  p->ldr = deflate_pad_cols(n);
  if (p->ldr <= 0) return false;
  p->k_max = (o.k_max > 0) ? o.k_max : (m < n ? m : n);
  if (p->k_max > m || p->k_max > n) return false;
  p->ldl = round_up(p->k_max, 16);  // rows of L 64-byte aligned, padded to whole GEMM K steps
  p->bf16 = o.precision == RBRP_PREC_BF16;
  p->r_f64 = dt == RBRP_F64;
  p->native_mode = p->r_f64 ? kModeF64 : kModeF32;
  p->refine = o.w_refine < 0 ? 1 : o.w_refine;
  if (o.w_method != 0 && o.w_method != 1) return false;
  if (!(o.w_clip < 1.0)) return false;   // NaN or 1 and above: nothing could be kept
  p->w_pinv = o.w_method == 1;
  p->ntiles = scan_num_tiles(m);
  const int64_t a = norms_num_partials(p->mr), c = deflate_num_partials(p->mr);
  p->nparts = a > c ? a : c;
  return true;
}

size_t layout(const Plan& p, char* base, Work* w) {
  Carver cv;
  cv.base = base;
  const size_t rs = p.r_f64 ? sizeof(double) : sizeof(float);
  const int mode = p.bf16 ? kModeBF16x3 : p.native_mode;
  w->sc = cv.take<DevScalars>(1);
  w->R = cv.take<char>((size_t)p.mr * p.ldr * rs);
  w->R16 = p.bf16 ? cv.take<char>((size_t)p.mr * p.ldr * 2) : nullptr;
  w->d = cv.take<double>(p.mr);
  w->part_sum = cv.take<double>(p.nparts);
  w->part_max = cv.take<double>(p.nparts);
  w->sel_block = cv.take<int32_t>(p.m);
  w->cdf = cv.take<uint64_t>(p.m);
  w->tile_sum = cv.take<uint64_t>(p.ntiles + 1);
  w->tile_pos = cv.take<int32_t>(p.ntiles + 1);
  w->idx = cv.take<int64_t>(kMaxB);
  w->xs2 = cv.take<double>(kMaxB);
  w->Vt = cv.take<double>((size_t)p.b * p.ldr);
  w->C = cv.take<double>((size_t)kNtMaxSlices * p.k_max * p.b);  // K slices of C
  w->G = cv.take<double>((size_t)kNtMaxSlices * p.b * p.b);  // K slices of the Gram
  w->piv = cv.take<int32_t>(kMaxB);
  w->piv2 = cv.take<int32_t>(kMaxB);
  w->Rraw = cv.take<double>((size_t)p.b * p.b);
  w->R2raw = cv.take<double>((size_t)p.b * p.b);
  w->Mc = cv.take<double>((size_t)p.b * p.b);
  w->Mc2 = cv.take<double>((size_t)p.b * p.b);
  w->Rinv = cv.take<double>((size_t)p.b * p.b);
  w->Qtmp = cv.take<double>((size_t)p.b * p.ldr);
  w->Qt = cv.take<double>((size_t)p.k_max * p.ldr);
  w->fragB1 = cv.take<char>(frag_bytes(mode, p.ldr, p.bdef));
  w->fragA2 = cv.take<char>(frag_bytes(mode, p.ldr, p.bdef));
  const bool halves = p.b > kDeflateMaxB;
  w->fragB1b = halves ? cv.take<char>(frag_bytes(mode, p.ldr, p.bdef)) : nullptr;
  w->fragA2b = halves ? cv.take<char>(frag_bytes(mode, p.ldr, p.bdef)) : nullptr;
  w->L = cv.take<char>((size_t)p.m * p.ldl * rs);
  const size_t nint = p.w_pinv ? pinv_workspace_doubles(p.k_max)
                               : interp_workspace_doubles(p.m, p.k_max, p.refine);
  w->interp = cv.take<double>(nint);
  return cv.off + kAlign;
}

// Pinned host copy of the device scalars (one per host thread).
DevScalars* host_scalars() {
  static thread_local DevScalars* h = nullptr;
  if (!h) {
    if (hipHostMalloc((void**)&h, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess)
      h = nullptr;
  }
  return h;
}

// ---- running bound on the deflation rounding (the precision controller) ----
//
// Block s replaces the stored residual R by R - P Q'^T, P = R Q'.  Rounding
// that falls in span(Q') (the product R Q' itself, and the operand rounding of
// P in the update) stays orthogonal to X (I - Q Q^T) for every later basis, so
// it can only raise the tracked norm.  The rest can lower it: the operand
// rounding of Q' in the update (sd s_q |P|), the lo*lo product a split form
// drops (sd s_x |P|), the same rounding of Q' applied to the error of R Q'
// (at most u_op |R|), and the FP32 accumulator (sd s_a per rounding, about
// bprime / kstep + 1 roundings of values of size |R|).  With independent,
// mean-zero relative errors uniform in [-u, u] the squared Frobenius norm of
// that part has expectation at most v below; blocks add (orthogonal
// projections do not enlarge earlier errors), and the bound is kErrLambda
// standard deviations of the sum.
constexpr double kErrLambda = 3.0;
constexpr double kErrBudget = 0.25;   // default controller: E <= eps / 4

// ss: deviation of the storage rounding of the block's output residual
// (BF16 storage; 0 when R keeps FP32).
struct ModeDev { double sq, sx, sa, uop, ss; int kstep; };

bool mode_dev(int mode, ModeDev* d) {
  const double r3 = 1.0 / sqrt(3.0);
  const double u64 = ldexp(1.0, -53), u32 = ldexp(1.0, -24), ub = ldexp(1.0, -8);
  switch (mode) {
    case kModeF64: *d = {u64 * r3, 0.0, u64 * r3, 2 * u64, 0.0, 4}; return true;
    case kModeF32: *d = {u32 * r3, 0.0, u32 * r3, 2 * u32, 0.0, 4}; return true;
    case kModeBF16x3:
      *d = {ub * ub * r3, ub * ub * r3, u32 * r3, 3 * ub * ub, 0.0, 32};
      return true;
    case kModeBF16: *d = {ub * r3, 0.0, u32 * r3, 2 * ub, 0.0, 32}; return true;
    case kModeBF16W:
    case kModeBF16R: *d = {ub * r3, 0.0, u32 * r3, 2 * ub, ub * r3, 32}; return true;
  }
  return false;
}

// Variance increment of one block (relative to ||X||_F^2); -1 on bad input.
// A residual stored in BF16 adds the rounding of every stored value: it lies
// in all directions, so the part of it that later blocks move into L (and
// out of the tracked norm) is at most all of it, sd ss |R_new|.
double err_var_increment(int mode, int bprime, double r_prev_sq, double r_new_sq) {
  ModeDev md;
  if (!mode_dev(mode, &md) || bprime < 0) return -1.0;
  const double p2 = fmax(r_prev_sq - r_new_sq, 0.0);
  const double rp2 = fmax(r_prev_sq, 0.0);
  return (md.sq * md.sq + md.sx * md.sx) * p2 +
         (md.sq * md.uop * md.sq * md.uop +
          md.sa * md.sa * ((double)bprime / md.kstep + 1.0)) * rp2 +
         md.ss * md.ss * fmax(r_new_sq, 0.0);
}

// Contribution of keeping ``mode`` for every later block, starting from the
// relative squared residual r_sq: the later blocks remove at most r_sq in
// total; the product terms in |R| are allowed for up to 64 more blocks, the
// storage term for n_future blocks (the controller's estimate of the blocks
// left; a wrong estimate costs time, not accuracy, since the bound itself
// sums the increments of the blocks actually run).
double err_var_future(int mode, int b, double r_sq, int n_future) {
  ModeDev md;
  if (!mode_dev(mode, &md)) return 1e300;
  return (md.sq * md.sq + md.sx * md.sx) * r_sq +
         64.0 * (md.sq * md.uop * md.sq * md.uop +
                 md.sa * md.sa * ((double)b / md.kstep + 1.0)) * r_sq +
         (double)n_future * md.ss * md.ss * r_sq;
}

#define RBRP_HIP(expr)                             \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) {                        \
      if (getenv("RBRP_LOG"))                      \
        fprintf(stderr, "rbrp: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(e_), \
                __FILE__, __LINE__);               \
      return RBRP_E_HIP;                           \
    }                                              \
  } while (0)

// Phase timing with HIP events recorded on the caller's stream.  Events come
// from a per-thread pool that is created once and reused by later calls.
// level 1 times every phase; level 2 only the deflation launches (phase 3),
// the least intrusive way to measure the dominant kernel inside a timed loop.
struct Profiler {
  int level = 0;
  hipStream_t s = nullptr;
  struct Span { hipEvent_t a, b; int phase; };
  static constexpr int kMaxSpans = 1100;
  Span spans[kMaxSpans];
  int n = 0;
  bool open = false;
  static hipEvent_t pool_event(int i) {
    static thread_local std::vector<hipEvent_t> pool;
    while ((int)pool.size() <= i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[i];
  }
  void begin(int phase) {
    open = false;
    if (level == 0 || n >= kMaxSpans || (level == 2 && phase != 3)) return;
    Span& sp = spans[n];
    sp.a = pool_event(2 * n);
    sp.b = pool_event(2 * n + 1);
    if (!sp.a || !sp.b) { level = 0; return; }
    sp.phase = phase;
    (void)hipEventRecord(sp.a, s);
    open = true;
  }
  void end() {
    if (!open) return;
    (void)hipEventRecord(spans[n].b, s);
    ++n;
    open = false;
  }
  // phases: 0 init, 1 select, 2 filter, 3 deflate, 4 interp
  void collect(double* ms5, int* ndeflate) {
    for (int i = 0; i < 5; ++i) ms5[i] = 0.0;
    *ndeflate = 0;
    for (int i = 0; i < n; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, spans[i].a, spans[i].b) == hipSuccess) ms5[spans[i].phase] += t;
      if (spans[i].phase == 3) ++*ndeflate;
    }
  }
};

// Event marking the copy of a block's scalars (one per host thread).
hipEvent_t scalars_event() {
  static thread_local hipEvent_t e = nullptr;
  if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  return e;
}

rbrp_status fetch(DevScalars* h, const DevScalars* dsc, hipStream_t s) {
  RBRP_HIP(hipMemcpyAsync(h, dsc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  RBRP_HIP(hipStreamSynchronize(s));
  return RBRP_OK;
}

}  // namespace

extern "C" {

void rbrp_default_options(rbrp_options* opt) {
  if (opt) fill_defaults(opt);
}

double rbrp_err_bound_increment(int32_t mode, int32_t bprime, double r_prev_sq,
                                double r_new_sq) {
  return err_var_increment(mode, bprime, r_prev_sq, r_new_sq);
}

const char* rbrp_status_string(rbrp_status s) {
  switch (s) {
    case RBRP_OK: return "ok";
    case RBRP_E_INVALID: return "invalid argument";
    case RBRP_E_WORKSPACE: return "workspace too small";
    case RBRP_E_HIP: return "HIP runtime error";
    case RBRP_E_NONFINITE: return "input holds NaN or Inf";
    case RBRP_E_CAPACITY: return "tolerance not met within k_max skeletons";
    case RBRP_E_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

size_t rbrp_workspace_size(rbrp_dtype dtype, int64_t m, int64_t n, int32_t b,
                           const rbrp_options* opt) {
  Plan p;
  if (!make_plan(dtype, m, n, b, opt, &p)) return 0;
  Work w;
  return layout(p, nullptr, &w);
}

rbrp_status rbrp_id(const void* X, rbrp_dtype dtype, int64_t m, int64_t n, int64_t ldx,
                    double eps, int32_t b, uint64_t seed, const rbrp_options* opt,
                    int64_t* S, int64_t* k_host, double* W, int64_t ldw,
                    rbrp_stats* stats_host, void* workspace, size_t ws_bytes,
                    void* stream) {
  rbrp_options o;
  if (opt) o = *opt; else fill_defaults(&o);
  Plan p;
  if (!X || !S || !k_host || !workspace) return RBRP_E_INVALID;
  if (m > kMaxRows && (dtype == RBRP_F32 || dtype == RBRP_F64)) return RBRP_E_UNSUPPORTED;
  if (!make_plan(dtype, m, n, b, &o, &p)) return RBRP_E_INVALID;
  if (ldx < n) return RBRP_E_INVALID;
  if (!o.fixed_rank && !(eps > 0.0 && eps < 1.0)) return RBRP_E_INVALID;
  if (W && ldw < p.k_max) return RBRP_E_INVALID;
  if (o.replay_blocks < 0 || (o.replay_blocks > 0 && !o.replay_d)) return RBRP_E_INVALID;
  if (p.bf16 && dtype != RBRP_F32) return RBRP_E_UNSUPPORTED;
  const int mode_hi = p.bf16 ? kModeBF16x3 : p.native_mode;
  const int mode_lo = p.bf16 ? kModeBF16 : p.native_mode;
  if (!deflate_supported(mode_hi, p.ldr, p.bdef) || !deflate_supported(mode_lo, p.ldr, p.bdef) ||
      !deflate_supported(p.native_mode, p.ldr, p.bdef))
    return RBRP_E_UNSUPPORTED;
  Work w;
  const size_t need = layout(p, nullptr, &w);
  if (ws_bytes < need) return RBRP_E_WORKSPACE;
  layout(p, (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign), &w);
  if (((uintptr_t)workspace % kAlign) != 0 && ws_bytes < need) return RBRP_E_WORKSPACE;

  hipStream_t s = (hipStream_t)stream;
  DevScalars* h = host_scalars();
  if (!h) return RBRP_E_HIP;
  hipEvent_t ev_scalars = scalars_event();
  if (!ev_scalars) return RBRP_E_HIP;
  const double tau_b = o.tau_b < 0.0 ? 1.0 / b : o.tau_b;
  const double theta = o.theta;   // > 0: fixed split/plain switch; else the budget
  const int refine = p.refine;
  const int64_t k_max = p.k_max;
  const int64_t ldr = p.ldr;
  rbrp_stats st;
  memset(&st, 0, sizeof(st));
  Profiler prof;
  prof.level = (o.profile == 1 || o.profile == 2) ? o.profile : 0;
  prof.s = s;
  double flops = 0.0;
  double dbytes = 0.0;   // algorithmic HBM bytes of the deflation launches
  bool r16 = false;      // the residual is held in BF16 (BF16 form)

  RBRP_HIP(hipMemsetAsync(w.sc, 0, sizeof(DevScalars), s));
  RBRP_HIP(hipMemsetAsync(w.sel_block, 0xFF, sizeof(int32_t) * p.m, s));
  prof.begin(0);
  RBRP_HIP(launch_init_norms(X, dtype, m, n, ldx, w.R, p.r_f64, p.mr, ldr, w.d,
                             w.part_sum, w.part_max, &w.sc->nonfinite, s));
  RBRP_HIP(launch_reduce(w.part_sum, w.part_max, norms_num_partials(p.mr), w.sc, 1, s));
  prof.end();
  rbrp_status rs = fetch(h, w.sc, s);
  if (rs != RBRP_OK) return rs;
  if (h->nonfinite) return RBRP_E_NONFINITE;
  const double D0 = h->d0;
  st.norm_x_fro = sqrt(D0);
  *k_host = 0;
  if (D0 == 0.0) {
    st.resid_tracked = 0.0;
    if (stats_host) *stats_host = st;
    return RBRP_OK;
  }
  int64_t kS = 0;
  int32_t t = 0;
  rbrp_status final_status = RBRP_OK;
  double sum_d = h->sum_d;
  // running variance of the rounding bound; the stopping rule of Alg. 2 is
  // applied to the tracked residual plus the bound
  double err_var = 0.0;
  auto err_bound = [&]() { return kErrLambda * sqrt(err_var); };
  auto met = [&](double sd) {
    const double e = eps - err_bound();
    return e > 0.0 && sd <= e * e * D0;
  };
  const int def_rows = deflate_rows_per_wg(mode_hi, ldr);
  // test hook: block tt draws from the supplied norms and the loop runs
  // exactly replay_blocks blocks
  const bool replay = o.replay_blocks > 0;
  auto select_block = [&](int32_t tt, int32_t bsz) -> hipError_t {
    prof.begin(1);
    hipError_t e;
    const double* dsrc = replay ? o.replay_d + (int64_t)(tt - 1) * m : w.d;
    if (o.greedy) {
      e = launch_topb(dsrc, w.sel_block, m, bsz, w.idx, w.sc, w.cdf, p.m, s);
    } else {
      e = launch_weights_scan(dsrc, w.sel_block, nullptr, m, w.sc, w.cdf, w.tile_sum,
                              w.tile_pos, s);
      if (e == hipSuccess)
        e = launch_sample(w.cdf, w.tile_sum, w.tile_pos, m, bsz, seed, (uint64_t)tt, 0, w.idx,
                          w.sc, s);
    }
    if (e == hipSuccess) e = launch_gather_rows(X, dtype, n, ldx, w.idx, w.sc, bsz, w.Vt, ldr,
                                                w.xs2, s);
    prof.end();
    return e;
  };
  bool preselected = false;
  int64_t k_last = 0;        // skeletons before the last counted block
  double sum_last = sum_d;   // tracked squared residual before that block
  while (true) {
    if (kS >= k_max) {
      if (!o.fixed_rank && !replay && !met(sum_d)) final_status = RBRP_E_CAPACITY;
      break;
    }
    if (replay) {
      if (t >= o.replay_blocks) break;
    } else if (!o.fixed_rank && met(sum_d)) {
      break;
    }
    ++t;
    const int32_t bt = (int32_t)((int64_t)b < k_max - kS ? b : k_max - kS);
    // sampling (or greedy top-b) and V^T, the sampled rows of X in FP64 --
    // already queued behind the previous block's deflation when its size
    // was certain
    if (!preselected) RBRP_HIP(select_block(t, bt));
    preselected = false;
    // project twice against the basis
    prof.begin(2);
    // C = Q V^T in K slices when it has few output tiles (the update adds
    // the slices)
    const int nsl = kS > 0 ? nt_slice_count(kS, bt, ldr) : 1;
    const int64_t cstride = (int64_t)k_max * p.b;
    if (kS > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        RBRP_HIP(launch_gemm_nt_small(kS, bt, ldr, 1.0, w.Qt, ldr, w.Vt, ldr, 0.0, w.C, bt,
                                      nullptr, nullptr, s, nsl, cstride));
        RBRP_HIP(launch_gemm_tn_small(bt, ldr, kS, -1.0, w.C, bt, w.Qt, ldr, 1.0, w.Vt, ldr,
                                      s, nullptr, nullptr, nsl, cstride));
      }
    }
    // robust blockwise filter: pivoted Cholesky of V^T V, then the kept columns'
    // orthonormal basis Q' = V(:, piv(1:b')) R11^{-1}
    // the filter's Gram matrix in K slices too when it has few output tiles
    // (the pivoted Cholesky adds them while copying G in); the second Gram
    // below stays whole (its first-order check reads each entry, where the
    // slices cost more than they save: measured)
    const int nslg = nt_slice_count(bt, bt, ldr);
    const int64_t gstride = (int64_t)p.b * p.b;
    RBRP_HIP(launch_gemm_nt_small(bt, bt, ldr, 1.0, w.Vt, ldr, w.Vt, ldr, 0.0, w.G, bt, nullptr,
                                  nullptr, s, nslg, gstride));
    RBRP_HIP(launch_cpqr_piv(w.G, bt, bt, &w.sc->nt, tau_b, w.xs2, w.piv, w.Rraw, bt, w.Mc, bt,
                             &w.sc->bprime, &w.sc->tail1, &w.sc->stop_rank, s, nslg, gstride));
    RBRP_HIP(launch_qsolve(w.Vt, ldr, w.piv, w.Mc, bt, &w.sc->bprime, bt, ldr, w.Qtmp, ldr,
                           w.Rinv, s));
    // second pass: project against the basis, then Cholesky QR
    if (kS > 0) {
      RBRP_HIP(launch_gemm_nt_small(kS, bt, ldr, 1.0, w.Qt, ldr, w.Qtmp, ldr, 0.0, w.C, bt,
                                    nullptr, nullptr, s, nsl, cstride));
      RBRP_HIP(launch_gemm_tn_small(bt, ldr, kS, -1.0, w.C, bt, w.Qt, ldr, 1.0, w.Qtmp, ldr,
                                    s, nullptr, nullptr, nsl, cstride));
    }
    RBRP_HIP(launch_gemm_nt_small(bt, bt, ldr, 1.0, w.Qtmp, ldr, w.Qtmp, ldr, 0.0, w.G, bt,
                                  nullptr, nullptr, s));
    RBRP_HIP(launch_ortho_first_order(w.G, bt, &w.sc->bprime, bt, w.Mc2, bt,
                                      &w.sc->need_exact, s));
    RBRP_HIP(launch_ortho_exact(w.G, bt, &w.sc->bprime, bt, w.piv2, w.R2raw, w.Mc, w.Mc2, bt,
                                &w.sc->b2, &w.sc->need_exact, s));
    double* Qn = w.Qt + kS * ldr;
    RBRP_HIP(launch_gemm_tn_small(bt, ldr, bt, 1.0, w.Mc2, bt, w.Qtmp, ldr, 0.0, Qn, ldr, s,
                                  nullptr, &w.sc->bprime));
    RBRP_HIP(launch_append(w.idx, w.piv, &w.sc->bprime, kS, t, S, w.sel_block, w.sc->bchunk,
                           s));
    // deflation of the residual, in launches of at most kDeflateMaxB columns
    int mode = p.native_mode;
    bool to_fp32_storage = false;
    if (p.bf16) {
      const double r_sq = sum_d / D0;
      if (theta > 0.0) {
        mode = sqrt(r_sq) > theta ? kModeBF16x3 : kModeBF16;
      } else {
        // the cheapest deflation whose contribution, kept for every later
        // block, holds the bound within the budget: one BF16 product on a
        // BF16-stored residual, then on the FP32 residual, the split
        // products, the FP32 product
        const double lim = kErrBudget * eps / kErrLambda;
        const int64_t left = (k_max - kS + b - 1) / b;
        const int n_future = (int)(left < 1 ? 1 : (left > 64 ? 64 : left));
        mode = p.native_mode;
        for (int cand : {r16 ? kModeBF16R : kModeBF16W, kModeBF16, kModeBF16x3}) {
          if (err_var + err_var_future(cand, b, r_sq, n_future) <= lim * lim) {
            mode = cand;
            break;
          }
        }
      }
      // a BF16-stored residual that the budget no longer allows goes back to
      // FP32 (exactly: every BF16 value is an FP32 value)
      if (r16 && !mode_reads_bf16(mode)) to_fp32_storage = true;
      if (mode == kModeBF16x3) st.blocks_split++;
      if (mode == p.native_mode) st.blocks_native++;
      if (mode_stores_bf16(mode)) st.blocks_bf16_stored++;
    }
    // blocks wider than kDeflateMaxB columns: both halves in one launch
    // where the mode allows it (the count of the second half stays on the
    // device), else one launch per half
    const bool fuse = b > kDeflateMaxB && deflate_fuses_halves(mode);
    int nchunk = 1;
    if (b > kDeflateMaxB && !fuse) {
      rs = fetch(h, w.sc, s);
      if (rs != RBRP_OK) return rs;
      nchunk = h->bprime > kDeflateMaxB ? 2 : 1;
    }
    if (to_fp32_storage) {
      RBRP_HIP(launch_r16_to_r32(w.R16, w.R, p.mr, ldr, s));
      r16 = false;
    }
    prof.end();
    const double s_in = mode_reads_bf16(mode) ? 2.0 : (p.r_f64 ? 8.0 : 4.0);
    if (fuse) {
      prof.begin(2);
      RBRP_HIP(launch_make_frags(Qn, ldr, &w.sc->bchunk[0], ldr, p.bdef, mode, w.fragB1,
                                 w.fragA2, s));
      RBRP_HIP(launch_make_frags(Qn + (int64_t)kDeflateMaxB * ldr, ldr, &w.sc->bchunk[1], ldr,
                                 p.bdef, mode, w.fragB1b, w.fragA2b, s));
      prof.end();
      prof.begin(3);
      RBRP_HIP(launch_deflate(mode, w.R, w.R16, p.mr, ldr, m, w.fragB1, w.fragA2,
                              &w.sc->bchunk[0], p.bdef, w.fragB1b, w.fragA2b,
                              &w.sc->bchunk[1], w.L, p.ldl, kS, w.sel_block, t, w.d,
                              w.part_sum, w.part_max, s));
      prof.end();
      const double sw = mode_stores_bf16(mode) ? 2.0 : (p.r_f64 ? 8.0 : 4.0);
      dbytes += (double)m * (double)n * (s_in + sw) + 8.0 * (double)m;
    }
    for (int c = 0; c < (fuse ? 0 : nchunk); ++c) {
      const int32_t* bcnt = b > kDeflateMaxB ? &w.sc->bchunk[c] : &w.sc->bprime;
      // the first launch of a block that switches to BF16 storage writes the
      // BF16 residual, a second one reads it
      const int cm = (mode == kModeBF16W && c > 0) ? kModeBF16R : mode;
      prof.begin(2);
      RBRP_HIP(launch_make_frags(Qn + (int64_t)c * kDeflateMaxB * ldr, ldr, bcnt, ldr, p.bdef,
                                 cm, w.fragB1, w.fragA2, s));
      prof.end();
      prof.begin(3);
      RBRP_HIP(launch_deflate(cm, w.R, w.R16, p.mr, ldr, m, w.fragB1, w.fragA2, bcnt, p.bdef,
                              nullptr, nullptr, nullptr, w.L, p.ldl,
                              kS + (int64_t)c * kDeflateMaxB, w.sel_block, t, w.d,
                              w.part_sum, w.part_max, s));
      prof.end();
      // algorithmic bytes: R read and written, d written (L below)
      const double sr = mode_reads_bf16(cm) ? 2.0 : s_in;
      const double sw = mode_stores_bf16(cm) ? 2.0 : (p.r_f64 ? 8.0 : 4.0);
      dbytes += (double)m * (double)n * (sr + sw) + 8.0 * (double)m;
    }
    if (mode_stores_bf16(mode)) r16 = true;
    RBRP_HIP(launch_reduce(w.part_sum, w.part_max, p.mr / def_rows, w.sc, 0, s));
    // This block's scalars are copied out first; the next block's selection
    // needs only d, S and the block size, so when the size is certain (b
    // rows, whatever b' turns out to be) it is queued behind the copy, and
    // the host, waiting for the copy alone, decides and queues the next
    // steps while the GPU samples.  If the loop stops instead, the queued
    // work is simply not used.
    RBRP_HIP(hipMemcpyAsync(h, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    RBRP_HIP(hipEventRecord(ev_scalars, s));
    if (k_max - kS - bt >= b && (!replay || t < o.replay_blocks)) {
      RBRP_HIP(select_block(t + 1, b));
      preselected = true;
    }
    RBRP_HIP(hipEventSynchronize(ev_scalars));
    const int bp = h->bprime;
    flops += 4.0 * (double)m * (double)n * (double)(bp > 0 ? bp : 0);
    dbytes += (double)m * (double)(bp > 0 ? bp : 0) * (p.r_f64 ? 8.0 : 4.0);   // L columns
    if (t <= 256) st.bprime[t - 1] = bp;
    st.blocks = t;
    if (h->stop_rank || bp <= 0) break;
    if (h->b2 != bp) return RBRP_E_HIP;  // basis lost orthogonality beyond repair
    k_last = kS;
    sum_last = sum_d;
    kS += bp;
    {
      // a second half rounds the accumulator once more per row; in its own
      // launch with BF16 storage it also rounds the (larger) intermediate
      // residual to BF16
      const int halves = bp > kDeflateMaxB ? 2 : 1;
      double v = err_var_increment(mode, bp + 32 * (halves - 1), sum_d / D0, h->sum_d / D0);
      if (v > 0.0 && !fuse && nchunk > 1 && mode_stores_bf16(mode))
        v += (nchunk - 1) * err_var_increment(mode, 0, 0.0, sum_d / D0);
      if (v > 0.0) err_var += v;
    }
    sum_d = h->sum_d;
  }
  // Rank trimming: with Q' orthogonal to the earlier basis, the error of the
  // prefix that ends j columns into the last block is its starting residual
  // minus the squared norms of its first j columns of L (L-hat = X Q'); the
  // shortest prefix that meets the stopping rule is kept.  The partial sums
  // use the residual buffer (no longer needed), the column norms C.  Not in
  // the BF16 form: its tracked residual carries the BF16 rounding, and the
  // whole last block keeps the slack that covers it.
  if (o.trim && !o.fixed_rank && !replay && !p.bf16 && kS - k_last > 1 && met(sum_d)) {
    const int nc = (int)(kS - k_last);
    const int G = col_sumsq_groups(m);
    const size_t rsz = (size_t)p.mr * p.ldr * (p.r_f64 ? sizeof(double) : sizeof(float));
    if ((size_t)G * nc * sizeof(double) > rsz) return RBRP_E_HIP;
    double* part = reinterpret_cast<double*>(w.R);
    RBRP_HIP(launch_col_sumsq(w.L, p.r_f64, p.ldl, m, k_last, nc, part, w.C, s));
    double colsq[kMaxB];
    RBRP_HIP(hipMemcpyAsync(colsq, w.C, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
    RBRP_HIP(hipStreamSynchronize(s));
    double e = sum_last;
    for (int j = 0; j < nc; ++j) {
      e -= colsq[j];
      if (met(e)) {
        if (j + 1 < nc) {
          kS = k_last + j + 1;
          sum_d = e;
        }
        break;
      }
    }
  }
  *k_host = kS;
  st.resid_tracked = sqrt(fmax(sum_d, 0.0) / D0);
  st.err_bound = err_bound();
  st.w_rank = (int32_t)kS;
  if (W && kS > 0) {
    prof.begin(4);
    if (p.w_pinv) {
      const double clip = o.w_clip > 0.0 ? o.w_clip : 1e-12;
      RBRP_HIP(launch_interp_pinv(w.L, p.r_f64, p.ldl, m, kS, S, W, ldw, clip, w.interp,
                                  &st.w_rank, s));
    } else {
      RBRP_HIP(launch_interp(w.L, p.r_f64, p.ldl, m, kS, S, W, ldw, refine, w.interp, s));
    }
    prof.end();
  }
  RBRP_HIP(hipStreamSynchronize(s));
  if (prof.level) {
    double ms5[5];
    int nd = 0;
    prof.collect(ms5, &nd);
    st.ms_init = ms5[0];
    st.ms_select = ms5[1];
    st.ms_filter = ms5[2];
    st.ms_deflate = ms5[3];
    st.ms_interp = ms5[4];
    st.deflate_launches = nd;
    st.deflate_flops = flops;
    st.deflate_bytes = dbytes;
  }
  if (stats_host) *stats_host = st;
  return final_status;
}

// ---- single-step entry points ----

size_t rbrp_row_norms_workspace_size(int64_t m) {
  if (m <= 0) return 0;
  return 2 * kAlign + sizeof(DevScalars) + 2 * sizeof(double) * norms_num_partials(m);
}

rbrp_status rbrp_row_norms(const void* X, rbrp_dtype dtype, int64_t m, int64_t n,
                           int64_t ldx, double* d, double* sum_host, double* max_host,
                           void* workspace, size_t ws_bytes, void* stream) {
  if (!X || !d || !workspace) return RBRP_E_INVALID;
  if (dtype != RBRP_F32 && dtype != RBRP_F64) return RBRP_E_INVALID;
  if (m <= 0 || n <= 0 || ldx < n) return RBRP_E_INVALID;
  if (ws_bytes < rbrp_row_norms_workspace_size(m)) return RBRP_E_WORKSPACE;
  Carver cv;
  cv.base = (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  DevScalars* sc = cv.take<DevScalars>(1);
  const int64_t np = norms_num_partials(m);
  double* ps = cv.take<double>(np);
  double* pm = cv.take<double>(np);
  hipStream_t s = (hipStream_t)stream;
  DevScalars* h = host_scalars();
  if (!h) return RBRP_E_HIP;
  RBRP_HIP(hipMemsetAsync(sc, 0, sizeof(DevScalars), s));
  RBRP_HIP(launch_init_norms(X, dtype, m, n, ldx, nullptr, 0, m, 0, d, ps, pm,
                             &sc->nonfinite, s));
  RBRP_HIP(launch_reduce(ps, pm, np, sc, 1, s));
  rbrp_status rs = fetch(h, sc, s);
  if (rs != RBRP_OK) return rs;
  if (h->nonfinite) return RBRP_E_NONFINITE;
  if (sum_host) *sum_host = h->sum_d;
  if (max_host) *max_host = h->max_d;
  return RBRP_OK;
}

size_t rbrp_sample_workspace_size(int64_t m) {
  if (m <= 0) return 0;
  const int64_t np = masked_num_partials(m), nt = scan_num_tiles(m);
  return 8 * kAlign + sizeof(DevScalars) + 2 * sizeof(double) * np +
         sizeof(uint64_t) * m + (sizeof(uint64_t) + sizeof(int32_t)) * (nt + 1);
}

rbrp_status rbrp_sample_block(const double* d, const uint8_t* excluded, int64_t m,
                              int32_t b, uint64_t seed, uint64_t t, uint64_t ident,
                              int64_t* idx, int32_t* n_host, void* workspace,
                              size_t ws_bytes, void* stream) {
  if (!d || !idx || !n_host || !workspace) return RBRP_E_INVALID;
  if (m <= 0 || b < 1 || b > kMaxB) return RBRP_E_INVALID;
  if (scan_num_tiles(m) > 4096) return RBRP_E_UNSUPPORTED;
  if (ws_bytes < rbrp_sample_workspace_size(m)) return RBRP_E_WORKSPACE;
  Carver cv;
  cv.base = (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  DevScalars* sc = cv.take<DevScalars>(1);
  const int64_t np = masked_num_partials(m), nt = scan_num_tiles(m);
  double* ps = cv.take<double>(np);
  double* pm = cv.take<double>(np);
  uint64_t* cdf = cv.take<uint64_t>(m);
  uint64_t* ts = cv.take<uint64_t>(nt + 1);
  int32_t* tp = cv.take<int32_t>(nt + 1);
  hipStream_t s = (hipStream_t)stream;
  DevScalars* h = host_scalars();
  if (!h) return RBRP_E_HIP;
  RBRP_HIP(hipMemsetAsync(sc, 0, sizeof(DevScalars), s));
  RBRP_HIP(launch_masked_partials(d, excluded, m, ps, pm, s));
  RBRP_HIP(launch_reduce(ps, pm, np, sc, 0, s));
  RBRP_HIP(launch_weights_scan(d, nullptr, excluded, m, sc, cdf, ts, tp, s));
  RBRP_HIP(launch_sample(cdf, ts, tp, m, b, seed, t, ident, idx, sc, s));
  rbrp_status rs = fetch(h, sc, s);
  if (rs != RBRP_OK) return rs;
  *n_host = h->nt;
  return RBRP_OK;
}

size_t rbrp_block_cpqr_workspace_size(int64_t n, int32_t nb) {
  if (n <= 0 || nb < 1 || nb > kMaxB) return 0;
  return 11 * kAlign + sizeof(DevScalars) + sizeof(double) * (6 * (size_t)nb * nb) +
         sizeof(double) * (size_t)nb * n + sizeof(int32_t) * kMaxB;
}

rbrp_status rbrp_block_cpqr(const double* Vt, int64_t n, int32_t nb, int64_t ldv,
                            double tau_b, int32_t* piv, double* R, double* Qt,
                            int64_t ldq, int32_t* bprime_host, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!Vt || !piv || !R || !Qt || !bprime_host || !workspace) return RBRP_E_INVALID;
  if (n <= 0 || nb < 1 || nb > kMaxB || ldv < n || ldq < n) return RBRP_E_INVALID;
  if (!(tau_b >= 0.0 && tau_b <= 1.0)) return RBRP_E_INVALID;
  if (ws_bytes < rbrp_block_cpqr_workspace_size(n, nb)) return RBRP_E_WORKSPACE;
  Carver cv;
  cv.base = (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  DevScalars* sc = cv.take<DevScalars>(1);
  double* G = cv.take<double>((size_t)nb * nb);
  double* Rraw = cv.take<double>((size_t)nb * nb);
  double* R2 = cv.take<double>((size_t)nb * nb);
  double* Mc = cv.take<double>((size_t)nb * nb);
  double* Mc2 = cv.take<double>((size_t)nb * nb);
  double* Rinv = cv.take<double>((size_t)nb * nb);
  double* Qtmp = cv.take<double>((size_t)nb * n);
  int32_t* piv2 = cv.take<int32_t>(kMaxB);
  hipStream_t s = (hipStream_t)stream;
  DevScalars* h = host_scalars();
  if (!h) return RBRP_E_HIP;
  RBRP_HIP(hipMemsetAsync(sc, 0, sizeof(DevScalars), s));
  RBRP_HIP(launch_gemm_nt_small(nb, nb, n, 1.0, Vt, ldv, Vt, ldv, 0.0, G, nb, nullptr,
                                nullptr, s));
  RBRP_HIP(launch_cpqr_piv(G, nb, nb, nullptr, tau_b, nullptr, piv, Rraw, nb, R, nb,
                           &sc->bprime, &sc->tail1, nullptr, s));
  RBRP_HIP(launch_qsolve(Vt, ldv, piv, R, nb, &sc->bprime, nb, n, Qtmp, n, Rinv, s));
  RBRP_HIP(launch_gemm_nt_small(nb, nb, n, 1.0, Qtmp, n, Qtmp, n, 0.0, G, nb, nullptr,
                                nullptr, s));
  RBRP_HIP(launch_ortho_first_order(G, nb, &sc->bprime, nb, Mc2, nb, &sc->need_exact, s));
  RBRP_HIP(launch_ortho_exact(G, nb, &sc->bprime, nb, piv2, R2, Mc, Mc2, nb, &sc->b2,
                              &sc->need_exact, s));
  RBRP_HIP(launch_gemm_tn_small(nb, n, nb, 1.0, Mc2, nb, Qtmp, n, 0.0, Qt, ldq, s, nullptr,
                                &sc->bprime));
  rbrp_status rs = fetch(h, sc, s);
  if (rs != RBRP_OK) return rs;
  *bprime_host = h->bprime;
  return RBRP_OK;
}


size_t rbrp_batch_workspace_size(rbrp_dtype dtype, const rbrp_batch_shape* shape) {
  if ((dtype != RBRP_F32 && dtype != RBRP_F64) || !rbrp::batch_shape_ok(shape)) return 0;
  return rbrp::batch_workspace_size(dtype, shape);
}

static rbrp_status batch_check(int32_t count, rbrp_dtype dtype, double eps,
                               const rbrp_options* opt, const rbrp_batch_shape* shape,
                               const void* descs, const int32_t* k_out,
                               const int32_t* status_out, const void* workspace,
                               size_t ws_bytes, rbrp_options* o) {
  if (count < 0 || !descs || !k_out || !status_out || !workspace) return RBRP_E_INVALID;
  if (dtype != RBRP_F32 && dtype != RBRP_F64) return RBRP_E_INVALID;
  if (!(eps >= 0.0) || !(eps < 1.0)) return RBRP_E_INVALID;
  if (!rbrp::batch_shape_ok(shape)) return RBRP_E_INVALID;
  rbrp_default_options(o);
  if (opt) *o = *opt;
  if (!(o->tau_b <= 1.0)) return RBRP_E_INVALID;
  if (o->greedy || o->precision != RBRP_PREC_NATIVE || o->w_method != 0)
    return RBRP_E_UNSUPPORTED;
  if (ws_bytes < rbrp::batch_workspace_size(dtype, shape)) return RBRP_E_WORKSPACE;
  if (rbrp::batch_lds_needed(dtype, shape) > 128 * 1024) return RBRP_E_UNSUPPORTED;
  return RBRP_OK;
}

rbrp_status rbrp_id_batched(const rbrp_batch_desc* descs, const int32_t* order,
                            int32_t count, rbrp_dtype dtype, double eps, uint64_t seed,
                            const rbrp_options* opt, const rbrp_batch_shape* shape,
                            int32_t* k_out, int32_t* status_out, double* resid_out,
                            void* workspace, size_t ws_bytes, void* stream) {
  rbrp_options o;
  const rbrp_status v = batch_check(count, dtype, eps, opt, shape, descs, k_out, status_out,
                                    workspace, ws_bytes, &o);
  if (v != RBRP_OK) return v;
  if (count == 0) return RBRP_OK;
  RBRP_HIP(rbrp::launch_batched(descs, order, count, dtype, eps, seed, o, *shape, k_out,
                                status_out, resid_out, workspace, (hipStream_t)stream));
  return RBRP_OK;
}

// ---- sketchy pivoting and the oversampled sketchy ID ----

static bool sketchy_args_ok(rbrp_dtype dtype, int64_t m, int64_t n, int32_t k, int32_t l) {
  if (dtype != RBRP_F32 && dtype != RBRP_F64) return false;
  if (m < 1 || n < 1 || m > kMaxRows || l < 1 || l > 65536) return false;
  return k >= 1 && k <= l && (int64_t)k <= m;
}

size_t rbrp_sketchy_workspace_size(rbrp_dtype dtype, int64_t m, int64_t n, int32_t k,
                                   int32_t l) {
  if (!sketchy_args_ok(dtype, m, n, k, l)) return 0;
  return rbrp::sketchy_workspace_bytes(m, k, l);
}

rbrp_status rbrp_sketchy_id(const void* X, rbrp_dtype dtype, int64_t m, int64_t n, int64_t ldx,
                            int32_t k, int32_t l, const double* Omega, int64_t ldo,
                            int64_t* S, double* W, int64_t ldw, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!X || !Omega || !S || !workspace) return RBRP_E_INVALID;
  if (!sketchy_args_ok(dtype, m, n, k, l) || ldx < n || ldo < l) return RBRP_E_INVALID;
  if (W && ldw < k) return RBRP_E_INVALID;
  if (ws_bytes < rbrp::sketchy_workspace_bytes(m, k, l)) return RBRP_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  RBRP_HIP(rbrp::launch_sketchy(X, dtype == RBRP_F32 ? 1 : 0, m, n, ldx, k, l, Omega, ldo, S, W,
                                ldw, workspace, s));
  return RBRP_OK;
}

// ---- batched form on a static scratch array (no allocation) ----
//
// The array lives in the library's code object: each GPU that loads the
// library holds one copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only names the symbol); the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and is cached here.
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchMaxDevices];

// Device address of ``scratch`` on the current device (looked up on the
// first call on that device).
rbrp_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RBRP_E_HIP;
  if (dev < 0 || dev >= kScratchMaxDevices) return RBRP_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      if (getenv("RBRP_LOG"))
        fprintf(stderr, "rbrp: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
                hipGetErrorString(e));
      return RBRP_E_HIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return RBRP_OK;
}
}  // namespace

rbrp_status rbrp_id_batched_noalloc(const rbrp_batch_desc* descs, const int32_t* order,
                                    int32_t count, rbrp_dtype dtype, double eps,
                                    uint64_t seed, const rbrp_options* opt,
                                    const rbrp_batch_shape* shape, int32_t* k_out,
                                    int32_t* status_out, double* resid_out, void* stream) {
  if (dtype != RBRP_F32 && dtype != RBRP_F64) return RBRP_E_INVALID;
  if (!rbrp::batch_shape_ok(shape)) return RBRP_E_INVALID;
  // as many persistent workgroups as the array holds, up to the requested
  // count (the queue hands out the IDs, so the count changes no result); a
  // shape whose single workgroup needs more than the array is rejected
  rbrp_batch_shape sh = *shape;
  const int64_t fit = rbrp::batch_max_wg(dtype, &sh, kNoAllocScratchBytes);
  if (fit < 1) return RBRP_E_WORKSPACE;
  const int64_t want = sh.num_wg > 0 ? sh.num_wg : rbrp::batch_default_wg();
  sh.num_wg = (int32_t)(want < fit ? want : fit);
  if (stream) {
    int cur = -1, sdev = -1;
    if (hipGetDevice(&cur) != hipSuccess ||
        hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess)
      return RBRP_E_HIP;
    if (cur != sdev) return RBRP_E_INVALID;   // the array of the current device only
  }
  void* ws = nullptr;
  rbrp_status v = scratch_address(&ws);
  if (v != RBRP_OK) return v;
  rbrp_options o;
  v = batch_check(count, dtype, eps, opt, &sh, descs, k_out, status_out, ws,
                  kNoAllocScratchBytes, &o);
  if (v != RBRP_OK) return v;
  if (count == 0) return RBRP_OK;
  RBRP_HIP(rbrp::launch_batched(descs, order, count, dtype, eps, seed, o, sh, k_out,
                                status_out, resid_out, ws, (hipStream_t)stream));
  return RBRP_OK;
}

rbrp_status rbrp_batch_autotune(const rbrp_batch_desc* descs_host, rbrp_batch_desc* descs,
                                int32_t count, rbrp_dtype dtype, double eps, uint64_t seed,
                                const rbrp_options* opt, rbrp_batch_shape* shape,
                                int32_t* order, int32_t* k_out, int32_t* status_out,
                                double* resid_out, void* workspace, size_t ws_bytes,
                                void* stream, int32_t* b_class_host) {
  rbrp_options o;
  const rbrp_status v = batch_check(count, dtype, eps, opt, shape, descs, k_out, status_out,
                                    workspace, ws_bytes, &o);
  if (v != RBRP_OK) return v;
  if (!descs_host || !order || !b_class_host) return RBRP_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  constexpr int kClasses = 3;
  auto cls = [](int64_t n) { return n <= 64 ? 0 : (n <= 128 ? 1 : 2); };
  // largest-first queue order by the work estimate m n min(m, n)
  std::vector<int32_t> ord(count);
  for (int32_t i = 0; i < count; ++i) ord[i] = i;
  auto work = [&](int32_t i) {
    const rbrp_batch_desc& d = descs_host[i];
    return (double)d.m * (double)d.n * (double)(d.m < d.n ? d.m : d.n);
  };
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int32_t a, int32_t b) { return work(a) > work(b); });
  std::vector<rbrp_batch_desc> cur(descs_host, descs_host + count);
  hipEvent_t e0, e1;
  RBRP_HIP(hipEventCreate(&e0));
  RBRP_HIP(hipEventCreate(&e1));
  rbrp_status st = RBRP_OK;
  auto timed = [&](const std::vector<int32_t>& ord_c, const rbrp_batch_shape& sh,
                   float* ms) -> rbrp_status {
    RBRP_HIP(hipMemcpyAsync(descs, cur.data(), sizeof(rbrp_batch_desc) * count,
                            hipMemcpyHostToDevice, s));
    RBRP_HIP(hipMemcpyAsync(order, ord_c.data(), sizeof(int32_t) * ord_c.size(),
                            hipMemcpyHostToDevice, s));
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      RBRP_HIP(hipEventRecord(e0, s));
      RBRP_HIP(rbrp::launch_batched(descs, order, (int32_t)ord_c.size(), dtype, eps, seed, o,
                                    sh, k_out, status_out, resid_out, workspace, s));
      RBRP_HIP(hipEventRecord(e1, s));
      RBRP_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      RBRP_HIP(hipEventElapsedTime(&t, e0, e1));
      if (t < best) best = t;
    }
    *ms = best;
    return RBRP_OK;
  };
  const int32_t cand_b[3] = {8, 16, 32};
  for (int c = 0; c < kClasses && st == RBRP_OK; ++c) {
    std::vector<int32_t> members;
    for (int32_t i : ord)
      if (cls(descs_host[i].n) == c) members.push_back(i);
    b_class_host[c] = 0;
    if (members.empty()) continue;
    float best_ms = 1e30f;
    int32_t best_b = 0;
    for (int32_t bc : cand_b) {
      if (bc > shape->b_max) continue;
      for (int32_t i : members) cur[i].b = bc;
      float ms = 0.f;
      st = timed(members, *shape, &ms);
      if (st != RBRP_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_b = bc;
      }
    }
    for (int32_t i : members) cur[i].b = best_b;
    b_class_host[c] = best_b;
    // then the deflation's row-load depth of the class
    const int32_t cand_depth[3] = {1, 2, 4};
    best_ms = 1e30f;
    int32_t best_depth = 2;
    for (int32_t dep : cand_depth) {
      if (st != RBRP_OK) break;
      rbrp_batch_shape sh = *shape;
      sh.row_depth = (sh.row_depth & ~(15 << (4 * c))) | (dep << (4 * c));
      float ms = 0.f;
      st = timed(members, sh, &ms);
      if (st != RBRP_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_depth = dep;
      }
    }
    shape->row_depth = (shape->row_depth & ~(15 << (4 * c))) | (best_depth << (4 * c));
  }
  if (st == RBRP_OK) {
    const int32_t cand_wg[3] = {256, 512, 768};
    float best_ms = 1e30f;
    int32_t best_wg = shape->num_wg;
    for (int32_t nwg : cand_wg) {
      rbrp_batch_shape sh = *shape;
      sh.num_wg = nwg;
      if (rbrp::batch_workspace_size(dtype, &sh) > ws_bytes) continue;
      float ms = 0.f;
      st = timed(ord, sh, &ms);
      if (st != RBRP_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_wg = nwg;
      }
    }
    shape->num_wg = best_wg;
  }
  if (st == RBRP_OK) {
    hipError_t e = hipMemcpyAsync(descs, cur.data(), sizeof(rbrp_batch_desc) * count,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(order, ord.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice,
                         s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = RBRP_E_HIP;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // extern "C"
