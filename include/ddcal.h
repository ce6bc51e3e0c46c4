/*
 * ddcal.h - C ABI of the direction-dependent calibration hot path on AMD MI355X (gfx950).
 *
 * Problem (paper, Sections 2 and 3): N stations observe N(N-1)/2 baselines; the sky model
 * is grouped into K clusters (calibration directions) and one calibration solution - a
 * 2x2 complex Jones matrix per station - is found per cluster.  The measurement equation
 * (Hamaker, Bregman & Sault 1996) for baseline p<q, timeslot t, channel f is
 *
 *     V_pq = sum_k J_{p,k} C_{pq,k} J_{q,k}^H + noise,
 *     C_{pq,k} = sum_{s in k} B_s exp(-2 pi i (u l_s + v m_s + w (n_s - 1)) f / c),
 *     B_s = [[I+Q, U+iV], [U-iV, I-Q]],   n_s - 1 = sqrt(1 - l^2 - m^2) - 1,
 *
 * with (u, v, w) the baseline p - q in metres.  Calibration minimises
 * f = sum ||V_pq - J_p C_pq J_q^H||_F^2 one cluster at a time (SAGE sweep) with
 * Levenberg-Marquardt on the 8N x 8N Gauss-Newton normal equations (Madsen, Nielsen &
 * Tingleff 2004, Algorithm 3.16).
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory: every array pointer is DEVICE memory owned by the caller unless marked "host".
 *   The library never frees caller memory; it owns only the workspace inside a context.
 * Baselines: canonical order, p < q, p-major: b = p(2N-p-1)/2 + (q-p-1), B = N(N-1)/2.
 * Visibility-like buffers (data V, cluster data Y, residual R, coherencies C): 8 planes
 *   {xx.re, xx.im, xy.re, xy.im, yx.re, yx.im, yy.re, yy.im}, each [T][F][B] with the
 *   baseline index fastest.  Element type: double for DDC_FP64, float for DDC_MIXED.
 *   Coherencies of several clusters are stacked as [K][8][T][F][B].
 * Jones: always double, [K][N][8] = (re, im) of the entries 00, 01, 10, 11 (row-major),
 *   i.e. the parameter vector x in R^{8N} of one cluster is jones + 8N*k.
 * Streams: every call enqueues on the context's stream (ddc_set_stream; default: the
 *   null stream of the context's device).  Calls that return host results (cost, info,
 *   state) synchronise that stream before returning; the others do not.
 * Errors: a call returns a ddc_status; on failure ddc_last_error() describes it.  No
 *   exception or abort crosses the ABI.  Invalid sizes or null required pointers give
 *   DDC_EINVAL before any work is enqueued.
 * Threading: a context is not thread-safe; use one context per host thread / stream.
 */
#ifndef DDCAL_H
#define DDCAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DDC_OK = 0,
  DDC_EINVAL = -1,      /* bad size, null pointer, unsupported option */
  DDC_ENOMEM = -2,      /* workspace allocation failed */
  DDC_EDEVICE = -3,     /* HIP runtime error (message in ddc_last_error) */
  DDC_ENOTPD = -4,      /* damped normal matrix not positive definite (ddc_damped_solve) */
  DDC_ENONFINITE = -5,  /* NaN/Inf in the inputs, seen as a non-finite cost */
  DDC_ETIMEOUT = -6     /* an internal inter-workgroup wait exceeded its bound */
} ddc_status;

typedef enum {
  DDC_FP64 = 0,   /* all arithmetic and storage in double */
  DDC_MIXED = 1   /* FP32 storage, predict, residual and J^T J accumulation; FP64 phase
                     argument, cost, accept/reject and refinement of the LM step */
} ddc_precision;

typedef struct ddc_ctx ddc_ctx;

/* Observation geometry.  u, v, w: [T][B] metres (baseline p - q); freq_hz: [F] Hz. */
typedef struct {
  int32_t n_stations;     /* N >= 2 */
  int32_t n_times;        /* T >= 1 */
  int32_t n_chans;        /* F >= 1 */
  const double* u;
  const double* v;
  const double* w;
  const double* freq_hz;
} ddc_obs;

/* Sky model: point sources grouped into clusters; cluster k owns sources
 * [cluster_offset[k], cluster_offset[k+1]).  l, m: direction cosines; I, Q, U, V: Jy. */
typedef struct {
  int32_t n_clusters;              /* K >= 1 */
  const int32_t* cluster_offset;   /* HOST, [K+1], non-decreasing, cluster_offset[0] = 0 */
  const double* l;
  const double* m;
  const double* I;
  const double* Q;
  const double* U;
  const double* V;
} ddc_sky;

/* Levenberg-Marquardt options (Madsen-Nielsen-Tingleff, Algorithm 3.16, Levenberg damping). */
typedef struct {
  int32_t n_iter;        /* iterations; a rejected step counts as one */
  int32_t precision;     /* ddc_precision */
  double tau;            /* fresh start: mu_0 = tau * max diag(J^T J) */
  double mu_floor;       /* mu_eff = max(mu, mu_floor * max diag(J^T J)) */
  double refine_tol;     /* DDC_MIXED: stop refining when ||g - (H+mu_eff I) d|| <= tol ||g|| */
  int32_t refine_max;    /* DDC_MIXED: at most this many FP64 refinement steps (0..8) */
} ddc_lm_opts;

/* Damping state; pass it back to resume an iteration exactly.  fresh != 0 starts anew. */
typedef struct {
  double mu;
  double nu;
  int32_t fresh;
} ddc_lm_state;

/* Record of one LM iteration (host), in iteration order; a rejected step is recorded too. */
typedef struct {
  double cost;           /* f at the Jones held after the iteration (the trial's f if accepted) */
  double mu_eff;         /* damping the step was solved with: max(mu, mu_floor * max diag) */
  double mu;             /* mu after the iteration's update */
  double nu;             /* nu after the iteration's update */
  int32_t accepted;      /* 1 if the step was taken */
  int32_t refine_steps;  /* FP64 refinement steps of the iteration (DDC_MIXED) */
} ddc_lm_step;

/* Per-solve report (host). */
typedef struct {
  double cost0;          /* cost at the starting Jones */
  double cost;           /* cost at the returned Jones */
  int32_t n_accept;
  int32_t n_reject;      /* includes n_notpd */
  int32_t n_notpd;       /* factorisation failures (counted as rejections) */
  int32_t max_refine;    /* most refinement steps taken in one iteration (DDC_MIXED) */
} ddc_lm_info;

typedef struct {
  int32_t n_sweeps;      /* SAGE sweeps over all clusters, in index order */
  ddc_lm_opts lm;        /* LM options for each cluster visit (mu restarts from tau) */
} ddc_cal_opts;

/* Fills opts with the defaults: n_iter 10, DDC_FP64, tau 1e-3, mu_floor 1e-6,
 * refine_tol 1e-10, refine_max 5. */
void ddc_default_lm_opts(ddc_lm_opts* opts);

/* Context on HIP device `device`; owns the workspace.  DDC_EDEVICE if the device is absent. */
ddc_status ddc_create(ddc_ctx** out, int32_t device);
ddc_status ddc_destroy(ddc_ctx* ctx);
/* Enqueue later calls on `hip_stream` (a hipStream_t on the context's device; NULL = null stream). */
ddc_status ddc_set_stream(ddc_ctx* ctx, void* hip_stream);
/* Text of the last failure on ctx (valid until the next call on ctx). */
const char* ddc_last_error(const ddc_ctx* ctx);
/* Bytes of workspace currently held by the context. */
int64_t ddc_workspace_bytes(const ddc_ctx* ctx);

/* Model coherencies of every cluster (the predict of the measurement equation above).
 * coh: [K][8][T][F][B] of the precision's element type.  The phase argument is always
 * evaluated in FP64 and reduced to its fractional part, [0, 1) turns; DDC_MIXED takes FP32 sin/cos
 * and accumulates in FP32, DDC_FP64 stays in double.  Paper Section 2 (clusters) and
 * Section 3 (baselines). */
ddc_status ddc_predict(ddc_ctx* ctx, const ddc_obs* obs, const ddc_sky* sky,
                       int32_t precision, void* coh);

/* The same coherencies as ddc_predict, with station-factorised phasors: when the baseline
 * coordinates are differences of station coordinates (uvw_pq = uvw_p - uvw_q, as for the
 * canonical baselines), the phase splits as phi_pq = phi_p - phi_q and each cluster's
 * coherency is the rank-S product C(p,q) = sum_s B_s E_p,s conj(E_q,s) with
 * E_p,s = exp(-2 pi i phi_p,s) (measurement equation of ddc_predict; paper Section 2
 * clusters, Section 3 baselines).  su, sv, sw: station coordinates in metres, DEVICE
 * [T][N] FP64, caller-owned; obs supplies N, T, F and the frequencies (its baseline uvw are
 * not read).  Phases are FP64, reduced to [-1/2, 1/2) turns per station; DDC_MIXED takes
 * FP32 sin/cos and FP32 accumulation, DDC_FP64 stays in double.  The library holds
 * T*F*S*ceil(N/64)*64 complex phasors of workspace.  Errors: DDC_EINVAL for NULL arrays,
 * bad offsets or more than 65535 clusters. */
ddc_status ddc_predict_factored(ddc_ctx* ctx, const ddc_obs* obs, const double* su,
                                const double* sv, const double* sw, const ddc_sky* sky,
                                int32_t precision, void* coh);

/* Residual of the measurement equation over all clusters (paper Section 2: the sky is the
 * sum of its clusters, each seen through its own Jones matrices; Section 3: every one of the
 * N(N-1)/2 baselines): res = vis - sum_{k<K} J_k C_k J_k^H and (optionally) the cost
 * f = ||res||^2, accumulated in FP64 in a fixed order.
 * vis, res: 8 planes [T][F][B]; coh: [K][8][T][F][B]; jones: [K][N][8].
 * res may be NULL (cost only); cost (HOST) may be NULL (no sync); res may alias vis.
 * With K >= 2 the workspace also holds a copy of the Jones matrices as K*8 component planes
 * (K*8*N elements, same values) that the kernel reads coalesced; the first call that needs
 * more workspace grows it, which synchronises the stream.
 * DDC_ENONFINITE if the cost is requested and is NaN/Inf (res is still written). */
ddc_status ddc_residual(ddc_ctx* ctx, const ddc_obs* obs, int32_t n_clusters, const void* vis,
                        const void* coh, const double* jones, int32_t precision,
                        void* res, double* cost);

/* ddc_residual for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * arithmetic and results, bit for bit (the Jones matrices are read in place, not from
 * component planes), with the call's scratch (canonical baseline table and
 * per-workgroup cost partials, 1.5 MiB) in a fixed device array that each GPU holds for the
 * life of the process, instead of the context workspace.  The call allocates nothing
 * (no hipMalloc/hipFree, no workspace growth).  Limits: n_stations <= 512 and
 * n_times * n_chans * N(N-1)/2 <= 16777216; beyond them DDC_EINVAL.  Every call on one GPU
 * shares that array (each call rebuilds what it reads from it first), so calls that overlap
 * on one GPU race: serialise them on one stream.  With cost (HOST) non-NULL the call
 * synchronises the stream; DDC_ENONFINITE as for ddc_residual. */
ddc_status ddc_residual_noalloc(ddc_ctx* ctx, const ddc_obs* obs, int32_t n_clusters,
                                const void* vis, const void* coh, const double* jones,
                                int32_t precision, void* res, double* cost);

/* out = in + alpha * sum_{k<K} J_k C_k J_k^H (alpha = +1 or -1); out may alias in: the
 * model of clusters 0..K-1 (paper Section 2, one Jones solution per cluster) added to or
 * taken from visibility planes.  Used to form synthetic data (in = noise) and the
 * per-cluster data of a SAGE sweep.  Workspace as for ddc_residual (Jones planes, K >= 2). */
ddc_status ddc_add_model(ddc_ctx* ctx, const ddc_obs* obs, int32_t n_clusters, const void* in,
                         const void* coh, const double* jones, double alpha,
                         int32_t precision, void* out);

/* Gauss-Newton normal equations of one cluster (the per-cluster solve of paper Section 2;
 * each of the N(N-1)/2 baselines of Section 3 couples its two stations' Jones) at jones_k
 * ([N][8]): with y the cluster's data and coh_k its coherencies ([8][T][F][B]),
 * r = y - J_p C J_q^H and A = d(J_p C J_q^H)/dx, JtJ = A^T A ([8N][8N] row-major, both
 * triangles written; nullable) and Jtr = A^T r ([8N]; nullable), in the precision's element
 * type; cost (HOST, nullable) = ||r||^2 in FP64 (synchronises).  DDC_ENONFINITE if the cost
 * is requested and is NaN/Inf. */
ddc_status ddc_build_normal_eq(ddc_ctx* ctx, const ddc_obs* obs, const void* y,
                               const void* coh_k, const double* jones_k, int32_t precision,
                               void* JtJ, void* Jtr, double* cost);

/* The damped linear solve of one LM step (Madsen, Nielsen & Tingleff 2004, Algorithm 3.16;
 * the 8N x 8N system of the paper's per-cluster solve, N stations of Section 2):
 * (H + mu I) d = g for symmetric H ([n][n] row-major; only the lower triangle is read) with
 * the library's blocked Cholesky; DDC_MIXED factors in FP32 and refines d in FP64
 * (refine_tol / refine_max as in ddc_lm_opts).  H, g: element type of the precision;
 * d: double [n].  refine_steps (HOST, nullable) receives the steps taken.  Synchronises.
 * DDC_ENOTPD if a pivot is not positive (d is then undefined); DDC_ETIMEOUT as for
 * ddc_lm_solve. */
ddc_status ddc_damped_solve(ddc_ctx* ctx, int32_t n, const void* H, const void* g, double mu,
                            int32_t precision, double refine_tol, int32_t refine_max,
                            double* d, int32_t* refine_steps);

/* Levenberg-Marquardt on one cluster (the per-cluster solve of the paper's Section 2: one
 * calibration solution per cluster, over all N(N-1)/2 baselines of Section 3), with the
 * damping schedule of Madsen, Nielsen & Tingleff (2004), Algorithm 3.16.
 * y ([8][T][F][B]) is that cluster's data, coh_k its coherencies; jones_k ([N][8], double)
 * is the start and receives the result.  state (HOST, nullable = fresh start) is read and
 * updated, so that calling again with it continues the iteration exactly; info (HOST,
 * nullable) receives the report; trace (HOST, nullable, [opts->n_iter]) receives one
 * ddc_lm_step per iteration.  The whole iteration runs on the device (no host round trip per
 * step); the call synchronises the stream once at the end to read the solve's status.
 * Errors: DDC_ENONFINITE if the cost at a built point is NaN/Inf (NaN/Inf in y, coh_k or
 * jones_k; the Jones are then left as they were), DDC_ETIMEOUT if an inter-workgroup wait
 * of the factorisation or the solves exceeded its bound (every later step of the call is
 * rejected, so the Jones hold the last accepted point).  A factorisation that finds a
 * non-positive pivot is not an error: the step is rejected (counted in n_notpd). */
ddc_status ddc_lm_solve(ddc_ctx* ctx, const ddc_obs* obs, const void* y, const void* coh_k,
                        double* jones_k, const ddc_lm_opts* opts, ddc_lm_state* state,
                        ddc_lm_info* info, ddc_lm_step* trace);

/* Full calibration (paper Section 2: a sky grouped into clusters, one solution per cluster,
 * solved for one cluster at a time): predict all clusters, then n_sweeps SAGE sweeps; in
 * each sweep every cluster k in index order gets Y_k = R + J_k C_k J_k^H, n_iter LM
 * iterations on Y_k (ddc_lm_solve's method, mu restarted from tau), and
 * R = Y_k - J_k C_k J_k^H.  vis: data; jones: [K][N][8] start and result; res (nullable)
 * receives the final residual R; info (HOST, nullable) receives [n_sweeps][K] reports;
 * trace (HOST, nullable) receives [n_sweeps][K][n_iter] iteration records.  The call
 * synchronises the stream once at the end to read the solves' status; errors as for
 * ddc_lm_solve (DDC_ENONFINITE, DDC_ETIMEOUT), reported for the whole calibration. */
ddc_status ddc_calibrate(ddc_ctx* ctx, const ddc_obs* obs, const ddc_sky* sky, const void* vis,
                         double* jones, const ddc_cal_opts* opts, void* res,
                         ddc_lm_info* info, ddc_lm_step* trace);

/* Gradient of the calibration cost (the per-cluster solves of paper Section 2 minimise it
 * cluster by cluster; this is its derivative for all clusters at once)
 * f = ||vis - sum_{k<K} J_k C_k J_k^H||^2 with respect to every cluster's Jones
 * in the real-pair layout of `jones`: grad[k][p][2e+c] = df/d(Re or Im of (J_{p,k})_e)
 * (double, [K][N][8]).  A hand-written adjoint kernel: df/dx_k = -2 (sum R G^H + sum R^H Hm)
 * per station with G = C J_q^H, Hm = J_p C.  cost (HOST, nullable) receives f and makes the
 * call synchronise.  DDC_MIXED computes the residual and the sums in FP32. */
ddc_status ddc_cost_gradient(ddc_ctx* ctx, const ddc_obs* obs, int32_t n_clusters,
                             const void* vis, const void* coh, const double* jones,
                             int32_t precision, double* grad, double* cost);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of whole calibrations (one request = one ddc_calibrate, e.g.
 * one frequency band; the paper's setting of many more bands than nodes, abstract and
 * Section 1).  Requests are admitted in arrival order when a slot (a context with its own
 * stream) is free and the request's workspace footprint fits in a free range of the server's
 * HBM arena; admitted requests run concurrently, and the predict work of requests admitted
 * together is fused into one persistent batched launch.  Every reduction in the path has a
 * fixed order, so a request's result is bitwise the same alone and in the mix.
 * ------------------------------------------------------------------------------------- */
typedef struct ddc_server ddc_server;

/* Bytes of workspace ddc_calibrate (and the server) needs for this problem; -1 if invalid. */
int64_t ddc_calibrate_footprint(const ddc_obs* obs, int32_t n_clusters, int32_t n_sweeps,
                                int32_t n_iter,
                                int32_t precision);
/* Server on `device` with n_slots concurrent solves (1..64) and an HBM arena of
 * hbm_budget_bytes (>= 64 KiB) allocated up front (DDC_ENOMEM if that fails). */
ddc_status ddc_server_create(ddc_server** out, int32_t device, int32_t n_slots,
                             int64_t hbm_budget_bytes);
/* Finishes every submitted request, then releases everything. */
ddc_status ddc_server_destroy(ddc_server* server);
/* Queue one calibration.  All device arrays of obs, sky, vis and jones must stay valid and
 * unmodified until ddc_server_wait returns for it; the host cluster offsets and the options
 * are copied.  DDC_ENOMEM if the request can never fit the arena. */
ddc_status ddc_server_submit(ddc_server* server, const ddc_obs* obs, const ddc_sky* sky,
                             const void* vis, double* jones, const ddc_cal_opts* opts,
                             int64_t* request_id);
/* Block until the request is done; info (HOST, nullable) receives [n_sweeps][K] reports,
 * latency_s the time from submit to completion, queue_s the time from submit to admission.
 * Returns the request's own status (its message via ddc_server_last_error). */
ddc_status ddc_server_wait(ddc_server* server, int64_t request_id, ddc_lm_info* info,
                           double* latency_s, double* queue_s);
ddc_status ddc_server_stats(ddc_server* server, int64_t* completed, int32_t* max_running,
                            int64_t* peak_arena_bytes);
const char* ddc_server_last_error(const ddc_server* server);

/* Kernel timing for measurement.  When enabled, the library brackets each launch of the
 * kernels below with HIP events on the context stream and accumulates, per kernel class,
 * the launch count, the summed durations and the summed algorithmic work of the launches.
 * Enabling or disabling resets the totals; ddc_get_timing synchronises the stream. */
typedef enum {
  DDC_TIMER_CHOLESKY = 0,   /* blocked Cholesky; work = n^3/3 flop per factorisation */
  DDC_TIMER_PREDICT = 1,    /* predict; work = source-visibility terms */
  DDC_TIMER_BUILD = 2,      /* normal-equation build; work = algorithmic HBM bytes */
  DDC_TIMER_TRSV = 3,       /* triangular solves; work = bytes of the factor read */
  DDC_TIMER_TRIAL = 4,      /* trial cost; work = bytes */
  DDC_TIMER_MODEL = 5,      /* model add/subtract and residual; work = bytes */
  DDC_TIMER_REFINE = 6,     /* refinement residual; work = bytes */
  DDC_TIMER_ADJOINT = 7,    /* cost adjoint; work = bytes */
  DDC_TIMER_PREDICT_FACTORED = 8  /* station-factorised predict; work = coherencies (K*T*F*B) */
} ddc_timer;
ddc_status ddc_enable_timing(ddc_ctx* ctx, int32_t on);
/* Bound every inter-workgroup wait of the context's factorisations and solves at `polls`
 * polls (0 restores the default, 2^22 polls, about a second).  Every such wait is bounded;
 * this makes the bound small so that the timeout path can be exercised: the factorisation or
 * solve that exceeds it aborts (all its workgroups leave), the LM step is rejected, and
 * ddc_lm_solve / ddc_calibrate / ddc_damped_solve report DDC_ETIMEOUT.  Synchronises. */
ddc_status ddc_set_wait_limit(ddc_ctx* ctx, uint32_t polls);
/* Time only the kernel classes whose bit (1 << ddc_timer) is set in mask (0: none).  Each
 * bracketing event pair adds a stream marker that waits for the launch before it, so a
 * throughput measurement times only the kernels it reports.  Resets the totals like
 * ddc_enable_timing. */
ddc_status ddc_enable_timers(ddc_ctx* ctx, uint32_t mask);
ddc_status ddc_get_timing(ddc_ctx* ctx, int32_t which, int64_t* launches, double* total_ms,
                          double* total_work);

#ifdef __cplusplus
}
#endif
#endif /* DDCAL_H */
