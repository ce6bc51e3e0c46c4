// Host side of libddcal: contexts, workspace, argument checks and the drivers that enqueue
// the kernels of predict, residual, normal equations, damped solve, LM and SAGE calibration.
// Every public entry point catches nothing and throws nothing: failures become ddc_status
// codes with a message kept in the context.
#include "../../include/ddcal.h"
#include "common.h"
#include "host_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace ddc;

namespace {

constexpr int kMaxTiles = 512;                  // n_pad <= 32768 (N <= 4096 stations)
constexpr size_t kSyncBytes = 2u << 20;        // [0, 1 MiB) zeroed; [1 MiB, 2 MiB) solve messages

enum Timer { T_CHOL = 0, T_PREDICT, T_BUILD, T_TRSV, T_TRIAL, T_MODEL, T_REFINE, T_ADJOINT,
             T_PREDICT_FACTORED, T_COUNT };

struct TimerAcc {
  int64_t launches = 0;
  double ms = 0.0;
  double work = 0.0;
};

struct Pending {
  int which;
  hipEvent_t a, b;
  double work;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct ddc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_external = false;      // workspace lent by a server arena (not owned, never grown)
  char* sync = nullptr;          // fixed region: LM state, sync areas, flags (zeroed once)
  int tab_N = 0;
  int32_t* ant = nullptr;        // [2][B] canonical baseline table
  const void* h_ptr = nullptr;   // matrix storage initialised for (address, n_pad, n, elem size)
  int h_npad = -1, h_n = -1, h_es = -1;
  uint32_t timing = 0u;          // bit k set: launches of timer k are bracketed with events
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  TimerAcc acc[T_COUNT];
  int chol_wg = 512;
  uint32_t chol_seq = 0;         // tag of the factorisation's partial-sum messages

  LMState* lm() { return reinterpret_cast<LMState*>(sync); }
  SyncArea* area(int i) { return reinterpret_cast<SyncArea*>(sync + 512 + 64 * i); }
  uint32_t* chol_flags() { return reinterpret_cast<uint32_t*>(sync + 1024); }
  uint32_t* fwd_flags() { return chol_flags() + kMaxTiles * (kMaxTiles + 1) / 2 + 2 * kMaxTiles; }
  uint32_t* bwd_flags() { return fwd_flags() + 2 * kMaxTiles; }
  // triangular-solve message arrays (partial sums, solution blocks), kEmpty between solves
  uint64_t* solve_psum() { return reinterpret_cast<uint64_t*>(sync + (1u << 20)); }
  uint64_t* solve_xpub() { return solve_psum() + 64 * kMaxTiles; }
  uint64_t* refine_norms() { return solve_xpub() + 64 * kMaxTiles; }
};

namespace {

ddc_status fail(ddc_ctx* c, ddc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCK(expr)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(c, DDC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

#define DDCCK(expr)                   \
  do {                                \
    ddc_status s_ = (expr);           \
    if (s_ != DDC_OK) return s_;      \
  } while (0)

hipEvent_t get_event(ddc_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events on the context stream when timing is on.
template <typename F>
ddc_status timed(ddc_ctx* c, int which, double work, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  const bool on = (c->timing >> which) & 1u;
  if (on) {
    a = get_event(c);
    b = get_event(c);
    if (a) HIPCK(hipEventRecord(a, c->stream));
  }
  HIPCK(launch());
  if (on && a && b) {
    HIPCK(hipEventRecord(b, c->stream));
    c->pending.push_back({which, a, b, work});
  }
  return DDC_OK;
}

ddc_status collect_timing(ddc_ctx* c) {
  if (c->pending.empty()) return DDC_OK;
  HIPCK(hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, p.a, p.b));
    c->acc[p.which].launches += 1;
    c->acc[p.which].ms += ms;
    c->acc[p.which].work += p.work;
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return DDC_OK;
}

// Workspace: one device allocation carved into aligned pieces by a bump layout.
struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  }
};

ddc_status ensure_ws(ddc_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return DDC_OK;
  if (c->ws_external)
    return fail(c, DDC_ENOMEM, "lent workspace of %zu bytes is smaller than the %zu needed", c->ws_bytes, bytes);
  HIPCK(hipStreamSynchronize(c->stream));
  if (c->ws && !c->ws_external) HIPCK(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->h_ptr = nullptr;
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, DDC_ENOMEM, "workspace allocation of %zu bytes failed", want);
  }
  c->ws_bytes = want;
  HIPCK(hipMemsetAsync(c->ws, 0, want, c->stream));
  return DDC_OK;
}

// Workspace for a call outside the solve layout (predict phasors, residual, cost gradient).
// Such a call may overwrite the matrix storage, whose zeros and padding diagonal are written
// once per (address, size), so the next solve writes them again.
ddc_status ensure_ws_other(ddc_ctx* c, size_t bytes) {
  DDCCK(ensure_ws(c, bytes));
  c->h_ptr = nullptr;
  return DDC_OK;
}

ddc_status check_prec(ddc_ctx* c, int32_t p) {
  if (p != DDC_FP64 && p != DDC_MIXED) return fail(c, DDC_EINVAL, "precision must be DDC_FP64 or DDC_MIXED");
  return DDC_OK;
}

ddc_status check_obs(ddc_ctx* c, const ddc_obs* o) {
  if (!c) return DDC_EINVAL;
  if (!o) return fail(c, DDC_EINVAL, "obs is NULL");
  if (o->n_stations < 2) return fail(c, DDC_EINVAL, "n_stations must be >= 2");
  if (8 * (int64_t)o->n_stations > 64 * kMaxTiles)
    return fail(c, DDC_EINVAL, "n_stations must be <= %d", 8 * kMaxTiles);
  if (o->n_times < 1 || o->n_chans < 1) return fail(c, DDC_EINVAL, "n_times and n_chans must be >= 1");
  if (!o->u || !o->v || !o->w || !o->freq_hz) return fail(c, DDC_EINVAL, "obs arrays must not be NULL");
  const int64_t B = (int64_t)o->n_stations * (o->n_stations - 1) / 2;
  if ((int64_t)o->n_times * o->n_chans * B > (int64_t)1 << 40)
    return fail(c, DDC_EINVAL, "problem too large");
  return DDC_OK;
}

// Canonical baseline table of the context's current N (rebuilt when N changes).
ddc_status obs_dev(ddc_ctx* c, const ddc_obs* o, ObsDev& d) {
  DDCCK(check_obs(c, o));
  const int N = o->n_stations;
  const int64_t B = (int64_t)N * (N - 1) / 2;
  if (c->tab_N != N) {
    HIPCK(hipStreamSynchronize(c->stream));
    if (c->ant) HIPCK(hipFree(c->ant));
    c->ant = nullptr;
    c->tab_N = 0;
    std::vector<int32_t> h(2 * B);
    int64_t b = 0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q, ++b) {
        h[b] = p;
        h[B + b] = q;
      }
    HIPCK(hipMalloc(&c->ant, 2 * B * sizeof(int32_t)));
    HIPCK(hipMemcpyAsync(c->ant, h.data(), 2 * B * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    c->tab_N = N;
  }
  d.N = N;
  d.T = o->n_times;
  d.F = o->n_chans;
  d.B = B;
  d.u = o->u;
  d.v = o->v;
  d.w = o->w;
  d.freq = o->freq_hz;
  d.ant_p = c->ant;
  d.ant_q = c->ant + B;
  return DDC_OK;
}

// Buffers of one damped solve / LM solve in the workspace.
struct SolveBufs {
  int n, n_pad, T, ld;
  void *Hc, *Lt, *Linv, *part, *cpart, *LtT, *LinvT;
  double *g, *diag, *d, *y, *s, *e, *cost_part, *scalar, *prow, *pcol;
  size_t h_off;
};

void layout_solve(Bump& bp, SolveBufs& b, int n, size_t es, int64_t B, int64_t nblk_max,
                  std::vector<size_t>& offs) {
  b.n = n;
  b.n_pad = (n + 63) / 64 * 64;
  b.T = b.n_pad / 64;
  b.ld = b.n_pad;
  const size_t np = b.n_pad;
  offs.clear();
  offs.push_back(bp.take(np * np * es));                                // Hc
  offs.push_back(bp.take((size_t)b.T * (b.T + 1) / 2 * 4096 * es));    // Lt
  offs.push_back(bp.take((size_t)b.T * 4096 * es));                    // Linv
  offs.push_back(bp.take((size_t)kPartials * (B > 0 ? B : 1) * es));   // part
  for (int i = 0; i < 6; ++i) offs.push_back(bp.take(np * sizeof(double)));  // g diag d y s e
  offs.push_back(bp.take((size_t)(nblk_max > 0 ? nblk_max : 1) * sizeof(double)));  // cost_part
  offs.push_back(bp.take(64 * sizeof(double)));                         // scalars
  const size_t ntiles = (size_t)b.T * (b.T + 1) / 2;
  offs.push_back(bp.take(ntiles * 64 * sizeof(double)));               // prow
  offs.push_back(bp.take(ntiles * 64 * sizeof(double)));               // pcol
  // Cholesky messages: look-ahead tiles (T x 2), tagged copies of the lower tiles, y blocks
  offs.push_back(bp.take(((size_t)b.T * 2 * 4096 + (size_t)b.T * (b.T + 1) / 2 * 4096 +
                          (size_t)64 * b.T) * 8));
  offs.push_back(bp.take((size_t)b.T * (b.T + 1) / 2 * 4096 * es));    // LtT (transposed tiles)
  offs.push_back(bp.take((size_t)b.T * 4096 * es));                    // LinvT
}

void bind_solve(ddc_ctx* c, SolveBufs& b, const std::vector<size_t>& o) {
  char* w = c->ws;
  b.Hc = w + o[0];
  b.Lt = w + o[1];
  b.Linv = w + o[2];
  b.part = w + o[3];
  b.g = reinterpret_cast<double*>(w + o[4]);
  b.diag = reinterpret_cast<double*>(w + o[5]);
  b.d = reinterpret_cast<double*>(w + o[6]);
  b.y = reinterpret_cast<double*>(w + o[7]);
  b.s = reinterpret_cast<double*>(w + o[8]);
  b.e = reinterpret_cast<double*>(w + o[9]);
  b.cost_part = reinterpret_cast<double*>(w + o[10]);
  b.scalar = reinterpret_cast<double*>(w + o[11]);
  b.prow = reinterpret_cast<double*>(w + o[12]);
  b.pcol = reinterpret_cast<double*>(w + o[13]);
  b.cpart = w + o[14];
  // the factorisation's FP32 tagged messages carry nonzero tags (zeroed scratch holds none);
  // its y messages start empty
  const size_t ntag = (size_t)b.T * 2 * 4096 + (size_t)b.T * (b.T + 1) / 2 * 4096;
  (void)hipMemsetAsync(b.cpart, 0, ntag * 8, c->stream);
  (void)launch_fill_empty(reinterpret_cast<uint64_t*>(b.cpart) + ntag, 64 * b.T, c->stream);
  b.LtT = w + o[15];
  b.LinvT = w + o[16];
  b.h_off = o[0];
}

// (Re)initialise the matrix storage (zeros, identity on the padding) when its place or
// shape changed; builds overwrite only the 8N x 8N lower part afterwards.
template <typename R>
ddc_status prepare_matrix(ddc_ctx* c, SolveBufs& b) {
  if (c->h_ptr == b.Hc && c->h_npad == b.n_pad && c->h_n == b.n && c->h_es == (int)sizeof(R))
    return DDC_OK;
  HIPCK(launch_init_matrix<R>(reinterpret_cast<R*>(b.Hc), b.ld, b.n, c->stream));
  c->h_ptr = b.Hc;
  c->h_npad = b.n_pad;
  c->h_n = b.n;
  c->h_es = (int)sizeof(R);
  return DDC_OK;
}

double chol_flop(int n) { return (double)n * n * n / 3.0; }

// Factor, solve and (optionally) refine: d = (H + mu_eff I)^{-1} g, all on the device.
template <typename R>
ddc_status enqueue_solve(ddc_ctx* c, SolveBufs& b, LMState* lm, int refine_max, double tol) {
  hipStream_t st = c->stream;
  R* Hc = reinterpret_cast<R*>(b.Hc);
  R* Lt = reinterpret_cast<R*>(b.Lt);
  R* Li = reinterpret_cast<R*>(b.Linv);
  R* LtT = reinterpret_cast<R*>(b.LtT);
  R* LiT = reinterpret_cast<R*>(b.LinvT);
  // the factorisation also runs the forward substitution y = L^{-1} g
  DDCCK(timed(c, T_CHOL, chol_flop(b.n), [&] {
    return launch_cholesky<R>(Hc, b.ld, b.n_pad, &lm->mu_eff, 0.0, b.g, b.y, Lt, Li, b.cpart,
                              ++c->chol_seq, c->area(0), c->chol_flags(), c->fwd_flags(),
                              &lm->notpd, st, c->chol_wg);
  }));
  // transposed copies of the factor and inverse tiles: the backward solves read them by rows
  HIPCK(launch_transpose_tiles<R>(Lt, LtT, b.T * (b.T + 1) / 2, Li, LiT, b.T, lm, st));
  const double tri_bytes = (double)b.n_pad * (b.n_pad + 64) / 2 * sizeof(R);
  DDCCK(timed(c, T_TRSV, tri_bytes, [&] {
    return launch_trsv<R>(false, LtT, LiT, b.n_pad, b.y, b.d, nullptr, c->solve_psum(),
                          c->solve_xpub(), c->area(2), &lm->timeout, lm, 1, st);
  }));
  for (int r = 0; r < refine_max; ++r) {
    DDCCK(timed(c, T_REFINE, (double)b.n_pad * b.n_pad * sizeof(R), [&] {
      return launch_refine_resid<R>(Hc, b.ld, b.n_pad, &lm->mu_eff, b.g, b.d, b.s,
                                    c->refine_norms(), b.prow, b.pcol, lm, 2, c->area(3),
                                    tol * tol, st);
    }));
    DDCCK(timed(c, T_TRSV, tri_bytes, [&] {
      return launch_trsv<R>(true, Lt, Li, b.n_pad, b.s, b.y, nullptr, c->solve_psum(),
                            c->solve_xpub(), c->area(1), &lm->timeout, lm, 2, st);
    }));
    DDCCK(timed(c, T_TRSV, tri_bytes, [&] {
      return launch_trsv<R>(false, LtT, LiT, b.n_pad, b.y, b.e, b.d, c->solve_psum(),
                            c->solve_xpub(), c->area(2), &lm->timeout, lm, 2, st);
    }));
  }
  return DDC_OK;
}

// n_iter LM iterations for one cluster; Jones updated in place on the device.
template <typename R>
ddc_status enqueue_lm(ddc_ctx* c, const ObsDev& o, const R* y, const R* coh, double* jones,
                      const ddc_lm_opts& opt, SolveBufs& b, int fresh, double mu, double nu,
                      ddc_lm_step* trace) {
  hipStream_t st = c->stream;
  LMState* lm = c->lm();
  const int refine_max = opt.precision == DDC_MIXED ? opt.refine_max : 0;
  const int n8 = 8 * o.N;
  HIPCK(launch_lm_init(lm, fresh, mu, nu, st));
  HIPCK(hipMemsetAsync(b.g, 0, (size_t)b.n_pad * sizeof(double), st));
  const double vis = (double)o.T * o.F * o.B;
  const double es = sizeof(R);
  const double build_bytes = vis * 16 * es + (double)o.B * (64 + kPartials) * es;
  for (int it = 0; it < opt.n_iter; ++it) {
    int nblk = 0;
    DDCCK(timed(c, T_BUILD, build_bytes, [&] {
      return launch_build_neq<R>(o, y, coh, jones, reinterpret_cast<R*>(b.Hc), b.ld,
                                 reinterpret_cast<R*>(b.part), b.cost_part, &nblk, lm, st);
    }));
    HIPCK(launch_neq_station<R>(o, reinterpret_cast<const R*>(b.part), reinterpret_cast<R*>(b.Hc),
                                b.ld, b.g, b.diag, lm, st));
    HIPCK(launch_lm_pre(lm, b.cost_part, nblk, b.diag, n8, b.g, opt.tau, opt.mu_floor,
                        refine_max, st));
    DDCCK(enqueue_solve<R>(c, b, lm, refine_max, opt.refine_tol));
    DDCCK(timed(c, T_TRIAL, vis * 16 * es, [&] {
      return launch_trial_cost<R>(o, y, coh, jones, b.d, b.cost_part, &nblk, lm, st);
    }));
    HIPCK(launch_lm_post(lm, b.cost_part, nblk, b.d, b.g, n8, jones, trace, st));
  }
  return DDC_OK;
}

ddc_status check_lm_opts(ddc_ctx* c, const ddc_lm_opts* opt) {
  if (!opt) return fail(c, DDC_EINVAL, "opts is NULL");
  DDCCK(check_prec(c, opt->precision));
  if (opt->n_iter < 0) return fail(c, DDC_EINVAL, "n_iter must be >= 0");
  if (!(opt->tau > 0.0) || !(opt->mu_floor >= 0.0) || !(opt->refine_tol >= 0.0))
    return fail(c, DDC_EINVAL, "tau must be > 0, mu_floor and refine_tol >= 0");
  if (opt->refine_max < 0 || opt->refine_max > 8) return fail(c, DDC_EINVAL, "refine_max must be in 0..8");
  return DDC_OK;
}

// Status of a finished solve from its device state: a timed-out wait first (its results are
// incomplete), then a non-finite cost.
ddc_status solve_status(ddc_ctx* c, const LMState& h) {
  if (h.timeout || (h.notpd & 2)) return fail(c, DDC_ETIMEOUT, "an inter-workgroup wait timed out");
  if (h.nonfinite) return fail(c, DDC_ENONFINITE, "the cost is not finite (NaN/Inf in the data, coherencies or Jones)");
  return DDC_OK;
}

void fill_info(const LMState& s, ddc_lm_info* info) {
  info->cost0 = s.f0;
  info->cost = s.f;
  info->n_accept = s.n_accept;
  info->n_reject = s.n_reject;
  info->n_notpd = s.n_notpd;
  info->max_refine = s.max_refine;
}

size_t esize(int32_t prec) { return prec == DDC_MIXED ? sizeof(float) : sizeof(double); }

}  // namespace

// ---------------------------------------------------------------------------------------
// Public ABI
// ---------------------------------------------------------------------------------------
extern "C" {

void ddc_default_lm_opts(ddc_lm_opts* o) {
  if (!o) return;
  o->n_iter = 10;
  o->precision = DDC_FP64;
  o->tau = 1e-3;
  o->mu_floor = 1e-6;
  o->refine_tol = 1e-10;
  o->refine_max = 5;
}

ddc_status ddc_create(ddc_ctx** out, int32_t device) {
  if (!out) return DDC_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return DDC_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return DDC_EDEVICE;
  ddc_ctx* c = new ddc_ctx();
  c->device = device;
  if (hipMalloc(&c->sync, kSyncBytes) != hipSuccess ||
      hipMemset(c->sync, 0, 1u << 20) != hipSuccess ||
      launch_fill_empty(c->solve_psum(), 2 * 64 * kMaxTiles + kMaxTiles, nullptr) != hipSuccess ||
      set_chol_smem_attr() != hipSuccess || noalloc_setup(device) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    if (c->sync) (void)hipFree(c->sync);
    delete c;
    return DDC_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->chol_wg = prop.multiProcessorCount;
  *out = c;
  return DDC_OK;
}

ddc_status ddc_destroy(ddc_ctx* c) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->ws && !c->ws_external) (void)hipFree(c->ws);
  if (c->ant) (void)hipFree(c->ant);
  if (c->sync) (void)hipFree(c->sync);
  delete c;
  return DDC_OK;
}

ddc_status ddc_set_stream(ddc_ctx* c, void* s) {
  if (!c) return DDC_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(s);
  return DDC_OK;
}

const char* ddc_last_error(const ddc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int64_t ddc_workspace_bytes(const ddc_ctx* c) { return c ? (int64_t)c->ws_bytes : 0; }

ddc_status ddc_predict(ddc_ctx* c, const ddc_obs* obs, const ddc_sky* sky, int32_t prec,
                       void* coh) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (!sky || !coh) return fail(c, DDC_EINVAL, "sky and coh must not be NULL");
  const int K = sky->n_clusters;
  if (K < 1 || !sky->cluster_offset) return fail(c, DDC_EINVAL, "n_clusters must be >= 1 with offsets");
  if (sky->cluster_offset[0] != 0) return fail(c, DDC_EINVAL, "cluster_offset[0] must be 0");
  for (int k = 0; k < K; ++k)
    if (sky->cluster_offset[k + 1] < sky->cluster_offset[k])
      return fail(c, DDC_EINVAL, "cluster_offset must be non-decreasing");
  const int S = sky->cluster_offset[K];
  if (S > 0 && (!sky->l || !sky->m || !sky->I || !sky->Q || !sky->U || !sky->V))
    return fail(c, DDC_EINVAL, "sky arrays must not be NULL");
  Bump bp;
  const size_t off = bp.take((size_t)(K + 1) * sizeof(int32_t));
  DDCCK(ensure_ws_other(c, bp.off));
  int32_t* offs = reinterpret_cast<int32_t*>(c->ws + off);
  HIPCK(hipMemcpyAsync(offs, sky->cluster_offset, (K + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                       c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  const double terms = (double)S * o.T * o.F * o.B;
  if (prec == DDC_MIXED)
    return timed(c, T_PREDICT, terms, [&] {
      return launch_predict<float>(o, K, offs, sky->cluster_offset, sky->l, sky->m, sky->I, sky->Q,
                                   sky->U, sky->V, reinterpret_cast<float*>(coh), c->stream);
    });
  return timed(c, T_PREDICT, terms, [&] {
    return launch_predict<double>(o, K, offs, sky->cluster_offset, sky->l, sky->m, sky->I, sky->Q,
                                  sky->U, sky->V, reinterpret_cast<double*>(coh), c->stream);
  });
}

ddc_status ddc_predict_factored(ddc_ctx* c, const ddc_obs* obs, const double* su,
                                const double* sv, const double* sw, const ddc_sky* sky,
                                int32_t prec, void* coh) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (!su || !sv || !sw) return fail(c, DDC_EINVAL, "station coordinates must not be NULL");
  if (!sky || !coh) return fail(c, DDC_EINVAL, "sky and coh must not be NULL");
  const int K = sky->n_clusters;
  if (K < 1 || K > 65535 || !sky->cluster_offset)
    return fail(c, DDC_EINVAL, "n_clusters must be in 1..65535 with offsets");
  if (sky->cluster_offset[0] != 0) return fail(c, DDC_EINVAL, "cluster_offset[0] must be 0");
  for (int k = 0; k < K; ++k)
    if (sky->cluster_offset[k + 1] < sky->cluster_offset[k])
      return fail(c, DDC_EINVAL, "cluster_offset must be non-decreasing");
  const int S = sky->cluster_offset[K];
  if (S > 0 && (!sky->l || !sky->m || !sky->I || !sky->Q || !sky->U || !sky->V))
    return fail(c, DDC_EINVAL, "sky arrays must not be NULL");
  const size_t es = prec == DDC_MIXED ? sizeof(float) : sizeof(double);
  Bump bp;
  const size_t off = bp.take((size_t)(K + 1) * sizeof(int32_t));
  const size_t off_e = bp.take(phasor_bytes(o.N, S, o.T, o.F, es));
  DDCCK(ensure_ws_other(c, bp.off));
  int32_t* offs = reinterpret_cast<int32_t*>(c->ws + off);
  void* E = c->ws + off_e;
  HIPCK(hipMemcpyAsync(offs, sky->cluster_offset, (K + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                       c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  const double vis = (double)K * o.T * o.F * o.B;
  if (prec == DDC_MIXED)
    return timed(c, T_PREDICT_FACTORED, vis, [&] {
      return launch_predict_factored<float>(o, su, sv, sw, K, S, offs, sky->l, sky->m, sky->I,
                                            sky->Q, sky->U, sky->V, E,
                                            reinterpret_cast<float*>(coh), c->stream);
    });
  return timed(c, T_PREDICT_FACTORED, vis, [&] {
    return launch_predict_factored<double>(o, su, sv, sw, K, S, offs, sky->l, sky->m, sky->I,
                                           sky->Q, sky->U, sky->V, E,
                                           reinterpret_cast<double*>(coh), c->stream);
  });
}

}  // extern "C"

namespace {
template <typename R>
ddc_status add_model_impl(ddc_ctx* c, const ObsDev& o, int K, const void* in, const void* coh,
                          const double* jones, double alpha, void* out, double* cost) {
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  const int64_t nblk = (plane + 255) / 256;
  double* parts = nullptr;
  double* total = nullptr;
  R* jplanes = nullptr;
  {
    // cost partials, and the Jones matrices as component planes when K >= 2 (left out, and
    // the Jones matrices read in place, when a lent workspace has no room for them)
    Bump bp;
    const size_t o1 = cost ? bp.take((size_t)nblk * sizeof(double)) : 0;
    const size_t o2 = cost ? bp.take(64) : 0;
    const size_t without = bp.off;
    bool planar = K >= 2;
    const size_t o3 = planar ? bp.take((size_t)K * 8 * o.N * sizeof(R)) : 0;
    if (planar && c->ws_external && bp.off > c->ws_bytes) {
      planar = false;
      bp.off = without;
    }
    if (bp.off) DDCCK(ensure_ws_other(c, bp.off));
    if (cost) {
      parts = reinterpret_cast<double*>(c->ws + o1);
      total = reinterpret_cast<double*>(c->ws + o2);
    }
    if (planar) jplanes = reinterpret_cast<R*>(c->ws + o3);
  }
  int nb = 0;
  const double bytes = (double)plane * (16.0 + 8.0 * K) * sizeof(R);
  DDCCK(timed(c, T_MODEL, bytes, [&] {
    return launch_add_model<R>(o, 0, K, reinterpret_cast<const R*>(in), reinterpret_cast<const R*>(coh),
                               jones, alpha, reinterpret_cast<R*>(out), parts, &nb, c->stream,
                               jplanes);
  }));
  if (cost) {
    HIPCK(launch_sum(parts, nb, total, c->stream));
    HIPCK(hipMemcpyAsync(cost, total, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    if (!std::isfinite(*cost)) return fail(c, DDC_ENONFINITE, "the cost is not finite");
  }
  return DDC_OK;
}
}  // namespace

extern "C" {

ddc_status ddc_residual(ddc_ctx* c, const ddc_obs* obs, int32_t K, const void* vis,
                        const void* coh, const double* jones, int32_t prec, void* res,
                        double* cost) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (K < 1 || !vis || !coh || !jones) return fail(c, DDC_EINVAL, "bad residual arguments");
  if (!res && !cost) return DDC_OK;
  if (prec == DDC_MIXED) return add_model_impl<float>(c, o, K, vis, coh, jones, -1.0, res, cost);
  return add_model_impl<double>(c, o, K, vis, coh, jones, -1.0, res, cost);
}

ddc_status ddc_residual_noalloc(ddc_ctx* c, const ddc_obs* obs, int32_t K, const void* vis,
                                const void* coh, const double* jones, int32_t prec, void* res,
                                double* cost) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  DDCCK(check_obs(c, obs));
  DDCCK(check_prec(c, prec));
  if (K < 1 || !vis || !coh || !jones) return fail(c, DDC_EINVAL, "bad residual arguments");
  if (obs->n_stations > kNoAllocMaxStations)
    return fail(c, DDC_EINVAL, "n_stations %d exceeds the no-allocation limit of %d",
                obs->n_stations, kNoAllocMaxStations);
  const int64_t B = (int64_t)obs->n_stations * (obs->n_stations - 1) / 2;
  const int64_t plane = (int64_t)obs->n_times * obs->n_chans * B;
  if ((plane + 255) / 256 > kNoAllocMaxBlocks)
    return fail(c, DDC_EINVAL, "%lld visibilities per plane exceed the no-allocation limit of %lld",
                (long long)plane, (long long)(kNoAllocMaxBlocks * 256));
  if (!res && !cost) return DDC_OK;
  const NoAllocScratch sc = noalloc_scratch(c->device);
  if (!sc.ant) return fail(c, DDC_EDEVICE, "no-allocation scratch not set up on device %d", c->device);
  // the baseline table lives in the scratch too (the context's own table may need an
  // allocation when N changes), rebuilt by every call
  ObsDev o;
  o.N = obs->n_stations;
  o.T = obs->n_times;
  o.F = obs->n_chans;
  o.B = B;
  o.u = obs->u;
  o.v = obs->v;
  o.w = obs->w;
  o.freq = obs->freq_hz;
  o.ant_p = sc.ant;
  o.ant_q = sc.ant + B;
  hipStream_t st = c->stream;
  HIPCK(launch_baseline_table(o.N, B, sc.ant, sc.ant + B, st));
  double* parts = cost ? sc.parts : nullptr;
  int nb = 0;
  if (prec == DDC_MIXED)
    HIPCK(launch_add_model<float>(o, 0, K, reinterpret_cast<const float*>(vis),
                                  reinterpret_cast<const float*>(coh), jones, -1.0,
                                  reinterpret_cast<float*>(res), parts, &nb, st));
  else
    HIPCK(launch_add_model<double>(o, 0, K, reinterpret_cast<const double*>(vis),
                                   reinterpret_cast<const double*>(coh), jones, -1.0,
                                   reinterpret_cast<double*>(res), parts, &nb, st));
  if (cost) {
    HIPCK(launch_sum(parts, nb, sc.total, st));
    HIPCK(hipMemcpyAsync(cost, sc.total, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (!std::isfinite(*cost)) return fail(c, DDC_ENONFINITE, "the cost is not finite");
  }
  return DDC_OK;
}

ddc_status ddc_add_model(ddc_ctx* c, const ddc_obs* obs, int32_t K, const void* in,
                         const void* coh, const double* jones, double alpha, int32_t prec,
                         void* out) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (K < 1 || !in || !coh || !jones || !out) return fail(c, DDC_EINVAL, "bad add_model arguments");
  if (alpha != 1.0 && alpha != -1.0) return fail(c, DDC_EINVAL, "alpha must be +1 or -1");
  if (prec == DDC_MIXED) return add_model_impl<float>(c, o, K, in, coh, jones, alpha, out, nullptr);
  return add_model_impl<double>(c, o, K, in, coh, jones, alpha, out, nullptr);
}

}  // extern "C"

namespace {
template <typename R>
ddc_status build_neq_impl(ddc_ctx* c, const ObsDev& o, const void* y, const void* coh_k,
                          const double* jones, void* JtJ, void* Jtr, double* cost) {
  Bump bp;
  SolveBufs b;
  std::vector<size_t> offs;
  layout_solve(bp, b, 8 * o.N, sizeof(R), o.B, (o.B + 255) / 256, offs);
  DDCCK(ensure_ws(c, bp.off));
  bind_solve(c, b, offs);
  DDCCK(prepare_matrix<R>(c, b));
  hipStream_t st = c->stream;
  int nblk = 0;
  const double vis = (double)o.T * o.F * o.B;
  const double bytes = vis * 16 * sizeof(R) + (double)o.B * (64 + kPartials) * sizeof(R);
  DDCCK(timed(c, T_BUILD, bytes, [&] {
    return launch_build_neq<R>(o, reinterpret_cast<const R*>(y), reinterpret_cast<const R*>(coh_k),
                               jones, reinterpret_cast<R*>(b.Hc), b.ld, reinterpret_cast<R*>(b.part),
                               b.cost_part, &nblk, nullptr, st);
  }));
  HIPCK(launch_neq_station<R>(o, reinterpret_cast<const R*>(b.part), reinterpret_cast<R*>(b.Hc), b.ld,
                              b.g, b.diag, nullptr, st));
  if (JtJ) HIPCK(launch_expand_sym<R>(reinterpret_cast<const R*>(b.Hc), b.ld, b.n, reinterpret_cast<R*>(JtJ), st));
  if (Jtr) HIPCK((launch_convert<double, R>(b.g, b.n, b.n, reinterpret_cast<R*>(Jtr), st)));
  if (cost) {
    HIPCK(launch_sum(b.cost_part, nblk, b.scalar, st));
    HIPCK(hipMemcpyAsync(cost, b.scalar, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (!std::isfinite(*cost)) return fail(c, DDC_ENONFINITE, "the cost is not finite");
  }
  return DDC_OK;
}
}  // namespace

extern "C" {

ddc_status ddc_build_normal_eq(ddc_ctx* c, const ddc_obs* obs, const void* y, const void* coh_k,
                               const double* jones_k, int32_t prec, void* JtJ, void* Jtr,
                               double* cost) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (!y || !coh_k || !jones_k) return fail(c, DDC_EINVAL, "y, coh_k and jones_k must not be NULL");
  if (prec == DDC_MIXED) return build_neq_impl<float>(c, o, y, coh_k, jones_k, JtJ, Jtr, cost);
  return build_neq_impl<double>(c, o, y, coh_k, jones_k, JtJ, Jtr, cost);
}

}  // extern "C"

namespace {
template <typename R>
ddc_status damped_solve_impl(ddc_ctx* c, int n, const void* H, const void* g, double mu,
                             int refine_max, double tol, double* d, int32_t* steps) {
  Bump bp;
  SolveBufs b;
  std::vector<size_t> offs;
  layout_solve(bp, b, n, sizeof(R), 0, 1, offs);
  DDCCK(ensure_ws(c, bp.off));
  bind_solve(c, b, offs);
  hipStream_t st = c->stream;
  // the caller's matrix becomes the column-major lower storage: row r of H is column r
  c->h_ptr = nullptr;
  HIPCK(launch_init_matrix<R>(reinterpret_cast<R*>(b.Hc), b.ld, n, st));
  HIPCK(hipMemcpy2DAsync(b.Hc, (size_t)b.ld * sizeof(R), H, (size_t)n * sizeof(R),
                         (size_t)n * sizeof(R), (size_t)n, hipMemcpyDeviceToDevice, st));
  HIPCK((launch_convert<R, double>(reinterpret_cast<const R*>(g), n, b.n_pad, b.g, st)));
  LMState* lm = c->lm();
  HIPCK(launch_solve_setup(lm, b.g, b.n_pad, mu, refine_max, st));
  DDCCK(enqueue_solve<R>(c, b, lm, refine_max, tol));
  HIPCK(hipMemcpyAsync(d, b.d, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  LMState h;
  HIPCK(hipMemcpyAsync(&h, lm, sizeof h, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (steps) *steps = h.refine_steps;
  if ((h.notpd & 2) || h.timeout) return fail(c, DDC_ETIMEOUT, "an inter-workgroup wait timed out");
  if (h.notpd & 1) return fail(c, DDC_ENOTPD, "matrix + mu I is not positive definite");
  return DDC_OK;
}
}  // namespace

extern "C" {

ddc_status ddc_damped_solve(ddc_ctx* c, int32_t n, const void* H, const void* g, double mu,
                            int32_t prec, double tol, int32_t refine_max, double* d,
                            int32_t* steps) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  DDCCK(check_prec(c, prec));
  if (n < 1 || n > 64 * kMaxTiles) return fail(c, DDC_EINVAL, "n must be in 1..%d", 64 * kMaxTiles);
  if (!H || !g || !d) return fail(c, DDC_EINVAL, "H, g and d must not be NULL");
  if (!(mu >= 0.0) || !(tol >= 0.0) || refine_max < 0 || refine_max > 8)
    return fail(c, DDC_EINVAL, "mu, tol >= 0 and refine_max in 0..8 required");
  if (prec == DDC_MIXED) return damped_solve_impl<float>(c, n, H, g, mu, refine_max, tol, d, steps);
  return damped_solve_impl<double>(c, n, H, g, mu, 0, tol, d, steps);
}

}  // extern "C"

namespace {
template <typename R>
ddc_status lm_solve_impl(ddc_ctx* c, const ObsDev& o, const void* y, const void* coh_k,
                         double* jones, const ddc_lm_opts& opt, ddc_lm_state* state,
                         ddc_lm_info* info, ddc_lm_step* trace) {
  Bump bp;
  SolveBufs b;
  std::vector<size_t> offs;
  layout_solve(bp, b, 8 * o.N, sizeof(R), o.B, (o.B + 255) / 256, offs);
  const size_t o_trace = bp.take((size_t)(opt.n_iter > 0 ? opt.n_iter : 1) * sizeof(ddc_lm_step));
  DDCCK(ensure_ws(c, bp.off));
  bind_solve(c, b, offs);
  DDCCK(prepare_matrix<R>(c, b));
  ddc_lm_step* dtrace = reinterpret_cast<ddc_lm_step*>(c->ws + o_trace);
  const int fresh = (!state || state->fresh) ? 1 : 0;
  DDCCK(enqueue_lm<R>(c, o, reinterpret_cast<const R*>(y), reinterpret_cast<const R*>(coh_k), jones,
                      opt, b, fresh, fresh ? 0.0 : state->mu, fresh ? 2.0 : state->nu,
                      trace ? dtrace : nullptr));
  // the solve's status is always read back (one small copy), so a timed-out wait or a
  // non-finite cost is reported even when the caller asks for no report
  LMState h;
  HIPCK(hipMemcpyAsync(&h, c->lm(), sizeof h, hipMemcpyDeviceToHost, c->stream));
  if (trace && opt.n_iter > 0)
    HIPCK(hipMemcpyAsync(trace, dtrace, (size_t)opt.n_iter * sizeof(ddc_lm_step),
                         hipMemcpyDeviceToHost, c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  if (state) {
    state->mu = h.mu;
    state->nu = h.nu;
    state->fresh = 0;
  }
  if (info) fill_info(h, info);
  return solve_status(c, h);
}
}  // namespace

extern "C" {

ddc_status ddc_lm_solve(ddc_ctx* c, const ddc_obs* obs, const void* y, const void* coh_k,
                        double* jones_k, const ddc_lm_opts* opts, ddc_lm_state* state,
                        ddc_lm_info* info, ddc_lm_step* trace) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_lm_opts(c, opts));
  if (!y || !coh_k || !jones_k) return fail(c, DDC_EINVAL, "y, coh_k and jones_k must not be NULL");
  if (state && !state->fresh && !(state->mu > 0.0 && state->nu >= 2.0))
    return fail(c, DDC_EINVAL, "resumed state needs mu > 0 and nu >= 2");
  if (opts->precision == DDC_MIXED)
    return lm_solve_impl<float>(c, o, y, coh_k, jones_k, *opts, state, info, trace);
  return lm_solve_impl<double>(c, o, y, coh_k, jones_k, *opts, state, info, trace);
}

}  // extern "C"

namespace {

// Workspace layout of one calibration (shared by ddc_calibrate and the server's footprint).
struct CalLayout {
  std::vector<size_t> solve_offs;
  size_t o_coh, o_R, o_Y, o_off, o_info, o_trace, total;
};

CalLayout layout_calibrate(const ObsDev& o, int K, int n_sweeps, int n_iter, size_t es,
                           SolveBufs& b) {
  CalLayout L;
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  Bump bp;
  layout_solve(bp, b, 8 * o.N, es, o.B, (o.B + 255) / 256, L.solve_offs);
  L.o_coh = bp.take((size_t)K * 8 * plane * es);
  L.o_R = bp.take((size_t)8 * plane * es);
  L.o_Y = bp.take((size_t)8 * plane * es);
  L.o_off = bp.take((size_t)(K + 1) * sizeof(int32_t));
  const int n_info = n_sweeps * K;
  L.o_info = bp.take((size_t)(n_info > 0 ? n_info : 1) * sizeof(LMState));
  const int64_t n_trace = (int64_t)n_info * (n_iter > 0 ? n_iter : 0);
  L.o_trace = bp.take((size_t)(n_trace > 0 ? n_trace : 1) * sizeof(ddc_lm_step));
  L.total = bp.off;
  return L;
}

}  // namespace

namespace ddc {
namespace host {

int64_t calibrate_footprint(const ObsDev& o, int K, int n_sweeps, int n_iter, int prec) {
  SolveBufs b;
  return (int64_t)layout_calibrate(o, K, n_sweeps, n_iter, esize(prec), b).total;
}

ddc_status prepare_calibrate(ddc_ctx* c, const ObsDev& o, const ddc_sky* sky, int n_sweeps,
                             int n_iter, int prec, CalBufs& cb) {
  const int K = sky->n_clusters;
  SolveBufs b;
  const CalLayout L = layout_calibrate(o, K, n_sweeps, n_iter, esize(prec), b);
  DDCCK(ensure_ws(c, L.total));
  bind_solve(c, b, L.solve_offs);
  if (prec == DDC_MIXED) DDCCK(prepare_matrix<float>(c, b));
  else DDCCK(prepare_matrix<double>(c, b));
  cb.solve = new SolveBufs(b);
  cb.coh = c->ws + L.o_coh;
  cb.Rb = c->ws + L.o_R;
  cb.Yb = c->ws + L.o_Y;
  cb.doffs = reinterpret_cast<int32_t*>(c->ws + L.o_off);
  cb.dinfo = reinterpret_cast<LMState*>(c->ws + L.o_info);
  cb.dtrace = reinterpret_cast<ddc_lm_step*>(c->ws + L.o_trace);
  cb.n_info = n_sweeps * K;
  cb.n_iter = n_iter;
  cb.K = K;
  cb.prec = prec;
  cb.offs_host.assign(sky->cluster_offset, sky->cluster_offset + K + 1);
  HIPCK(hipMemcpyAsync(cb.doffs, cb.offs_host.data(), (K + 1) * sizeof(int32_t),
                       hipMemcpyHostToDevice, c->stream));
  return DDC_OK;
}

void release_calibrate(CalBufs& cb) {
  delete reinterpret_cast<SolveBufs*>(cb.solve);
  cb.solve = nullptr;
}

template <typename R>
ddc_status enqueue_sage_t(ddc_ctx* c, const ObsDev& o, const void* vis, double* jones,
                          const ddc_cal_opts& opt, CalBufs& cb, bool residual_ready) {
  const int K = cb.K;
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  SolveBufs& b = *reinterpret_cast<SolveBufs*>(cb.solve);
  R* coh = reinterpret_cast<R*>(cb.coh);
  R* Rb = reinterpret_cast<R*>(cb.Rb);
  R* Yb = reinterpret_cast<R*>(cb.Yb);
  hipStream_t st = c->stream;
  const double es = sizeof(R);
  if (!residual_ready)
    DDCCK(timed(c, T_MODEL, (double)plane * (16.0 + 8.0 * K) * es, [&] {
      return launch_add_model<R>(o, 0, K, reinterpret_cast<const R*>(vis), coh, jones, -1.0, Rb,
                                 nullptr, nullptr, st);
    }));
  for (int e = 0; e < opt.n_sweeps; ++e) {
    for (int k = 0; k < K; ++k) {
      const R* ck = coh + (int64_t)k * 8 * plane;
      double* jk = jones + (int64_t)k * 8 * o.N;
      DDCCK(timed(c, T_MODEL, (double)plane * 24.0 * es, [&] {
        return launch_add_model<R>(o, k, k + 1, Rb, coh, jones, 1.0, Yb, nullptr, nullptr, st);
      }));
      DDCCK(enqueue_lm<R>(c, o, Yb, ck, jk, opt.lm, b, 1, 0.0, 2.0,
                          cb.dtrace + (int64_t)(e * K + k) * opt.lm.n_iter));
      DDCCK(timed(c, T_MODEL, (double)plane * 24.0 * es, [&] {
        return launch_add_model<R>(o, k, k + 1, Yb, coh, jones, -1.0, Rb, nullptr, nullptr, st);
      }));
      HIPCK(launch_copy_state(c->lm(), cb.dinfo + e * K + k, st));
    }
  }
  return DDC_OK;
}

ddc_status enqueue_sage(ddc_ctx* c, const ObsDev& o, const void* vis, double* jones,
                        const ddc_cal_opts& opt, CalBufs& cb, bool residual_ready) {
  if (cb.prec == DDC_MIXED) return enqueue_sage_t<float>(c, o, vis, jones, opt, cb, residual_ready);
  return enqueue_sage_t<double>(c, o, vis, jones, opt, cb, residual_ready);
}

ddc_status collect_infos(ddc_ctx* c, CalBufs& cb, ddc_lm_info* info, ddc_lm_step* trace) {
  if (cb.n_info <= 0) return DDC_OK;
  // every visit's state is read back whether or not reports are wanted: it carries the
  // timeout and non-finite flags that decide the call's status
  std::vector<LMState> h(cb.n_info);
  HIPCK(hipMemcpyAsync(h.data(), cb.dinfo, cb.n_info * sizeof(LMState), hipMemcpyDeviceToHost, c->stream));
  const size_t n_trace = (size_t)cb.n_info * (cb.n_iter > 0 ? cb.n_iter : 0);
  if (trace && n_trace > 0)
    HIPCK(hipMemcpyAsync(trace, cb.dtrace, n_trace * sizeof(ddc_lm_step), hipMemcpyDeviceToHost,
                         c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  ddc_status st = DDC_OK;
  for (int i = 0; i < cb.n_info; ++i) {
    if (info) fill_info(h[i], info + i);
    const ddc_status si = solve_status(c, h[i]);
    if (si == DDC_ETIMEOUT || (si != DDC_OK && st == DDC_OK)) st = si;
  }
  if (st == DDC_ETIMEOUT) return fail(c, st, "an inter-workgroup wait timed out");
  if (st != DDC_OK)
    return fail(c, st, "the cost is not finite (NaN/Inf in the data, coherencies or Jones)");
  return DDC_OK;
}

ddc_status ctx_obs(ddc_ctx* c, const ddc_obs* obs, ObsDev& o) { return obs_dev(c, obs, o); }
hipStream_t ctx_stream(ddc_ctx* c) { return c->stream; }
void ctx_lend_workspace(ddc_ctx* c, void* ws, size_t bytes) {
  c->ws = reinterpret_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->ws_external = ws != nullptr;
  c->h_ptr = nullptr;
}
const char* ctx_error(ddc_ctx* c) { return c->err.c_str(); }

}  // namespace host
}  // namespace ddc

namespace {
template <typename R>
ddc_status calibrate_impl(ddc_ctx* c, const ObsDev& o, const ddc_sky* sky, const void* vis,
                          double* jones, const ddc_cal_opts& opt, void* res, ddc_lm_info* info,
                          ddc_lm_step* trace) {
  using namespace ddc::host;
  const int K = sky->n_clusters;
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  CalBufs cb;
  DDCCK(prepare_calibrate(c, o, sky, opt.n_sweeps, opt.lm.n_iter, opt.lm.precision, cb));
  struct Guard { CalBufs& cb; ~Guard() { release_calibrate(cb); } } guard{cb};
  hipStream_t st = c->stream;
  const double terms = (double)sky->cluster_offset[K] * plane;
  DDCCK(timed(c, T_PREDICT, terms, [&] {
    return launch_predict<R>(o, K, cb.doffs, sky->cluster_offset, sky->l, sky->m, sky->I, sky->Q,
                             sky->U, sky->V, reinterpret_cast<R*>(cb.coh), st);
  }));
  DDCCK(enqueue_sage(c, o, vis, jones, opt, cb));
  if (res) HIPCK(hipMemcpyAsync(res, cb.Rb, (size_t)8 * plane * sizeof(R), hipMemcpyDeviceToDevice, st));
  return collect_infos(c, cb, info, trace);
}
}  // namespace

extern "C" {

ddc_status ddc_calibrate(ddc_ctx* c, const ddc_obs* obs, const ddc_sky* sky, const void* vis,
                         double* jones, const ddc_cal_opts* opts, void* res, ddc_lm_info* info,
                         ddc_lm_step* trace) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  if (!opts) return fail(c, DDC_EINVAL, "opts is NULL");
  DDCCK(check_lm_opts(c, &opts->lm));
  if (opts->n_sweeps < 0) return fail(c, DDC_EINVAL, "n_sweeps must be >= 0");
  if (!sky || !vis || !jones) return fail(c, DDC_EINVAL, "sky, vis and jones must not be NULL");
  const int K = sky->n_clusters;
  if (K < 1 || !sky->cluster_offset || sky->cluster_offset[0] != 0)
    return fail(c, DDC_EINVAL, "n_clusters >= 1 and cluster_offset[0] = 0 required");
  for (int k = 0; k < K; ++k)
    if (sky->cluster_offset[k + 1] < sky->cluster_offset[k])
      return fail(c, DDC_EINVAL, "cluster_offset must be non-decreasing");
  if (sky->cluster_offset[K] > 0 && (!sky->l || !sky->m || !sky->I || !sky->Q || !sky->U || !sky->V))
    return fail(c, DDC_EINVAL, "sky arrays must not be NULL");
  if (opts->lm.precision == DDC_MIXED)
    return calibrate_impl<float>(c, o, sky, vis, jones, *opts, res, info, trace);
  return calibrate_impl<double>(c, o, sky, vis, jones, *opts, res, info, trace);
}

}  // extern "C"

namespace {
template <typename R>
ddc_status cost_gradient_impl(ddc_ctx* c, const ObsDev& o, int K, const void* vis, const void* coh,
                              const double* jones, double* grad, double* cost) {
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  const int64_t nblk = (plane + 255) / 256;
  Bump bp;
  const size_t o_res = bp.take((size_t)8 * plane * sizeof(R));
  const size_t o_part = bp.take((size_t)K * 16 * o.B * sizeof(R));
  const size_t o_cp = bp.take((size_t)nblk * sizeof(double));
  const size_t o_tot = bp.take(64);
  DDCCK(ensure_ws_other(c, bp.off));
  R* res = reinterpret_cast<R*>(c->ws + o_res);
  R* part = reinterpret_cast<R*>(c->ws + o_part);
  double* cp = reinterpret_cast<double*>(c->ws + o_cp);
  double* tot = reinterpret_cast<double*>(c->ws + o_tot);
  hipStream_t st = c->stream;
  int nb = 0;
  const double es = sizeof(R);
  DDCCK(timed(c, T_MODEL, (double)plane * (16.0 + 8.0 * K) * es, [&] {
    return launch_add_model<R>(o, 0, K, reinterpret_cast<const R*>(vis), reinterpret_cast<const R*>(coh),
                               jones, -1.0, res, cp, &nb, st);
  }));
  DDCCK(timed(c, T_ADJOINT, (double)plane * 16.0 * K * es, [&] {
    return launch_cost_adjoint<R>(o, K, res, reinterpret_cast<const R*>(coh), jones, part, grad, st);
  }));
  if (cost) {
    HIPCK(launch_sum(cp, nb, tot, st));
    HIPCK(hipMemcpyAsync(cost, tot, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
  }
  return DDC_OK;
}
}  // namespace

extern "C" {

ddc_status ddc_cost_gradient(ddc_ctx* c, const ddc_obs* obs, int32_t K, const void* vis,
                             const void* coh, const double* jones, int32_t prec, double* grad,
                             double* cost) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  ObsDev o;
  DDCCK(obs_dev(c, obs, o));
  DDCCK(check_prec(c, prec));
  if (K < 1 || !vis || !coh || !jones || !grad) return fail(c, DDC_EINVAL, "bad cost_gradient arguments");
  if (prec == DDC_MIXED) return cost_gradient_impl<float>(c, o, K, vis, coh, jones, grad, cost);
  return cost_gradient_impl<double>(c, o, K, vis, coh, jones, grad, cost);
}

ddc_status ddc_enable_timers(ddc_ctx* c, uint32_t mask) {
  if (!c) return DDC_EINVAL;
  DDCCK(collect_timing(c));
  c->timing = mask;
  for (auto& a : c->acc) a = TimerAcc();
  return DDC_OK;
}

ddc_status ddc_set_wait_limit(ddc_ctx* c, uint32_t polls) {
  if (!c) return DDC_EINVAL;
  (void)hipSetDevice(c->device);
  HIPCK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 4; ++i)
    HIPCK(hipMemcpy(&c->area(i)->pad, &polls, sizeof polls, hipMemcpyHostToDevice));
  return DDC_OK;
}

ddc_status ddc_enable_timing(ddc_ctx* c, int32_t on) {
  return ddc_enable_timers(c, on ? 0xffffffffu : 0u);
}

ddc_status ddc_get_timing(ddc_ctx* c, int32_t which, int64_t* launches, double* total_ms,
                          double* total_work) {
  if (!c) return DDC_EINVAL;
  if (which < 0 || which >= T_COUNT) return fail(c, DDC_EINVAL, "timer index out of range");
  DDCCK(collect_timing(c));
  if (launches) *launches = c->acc[which].launches;
  if (total_ms) *total_ms = c->acc[which].ms;
  if (total_work) *total_work = c->acc[which].work;
  return DDC_OK;
}

}  // extern "C"
