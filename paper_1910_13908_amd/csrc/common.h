// Internal declarations shared by the HIP sources of libddcal (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddcal.h"

namespace ddc {

constexpr double kCLight = 299792458.0;

// Tile edge of the blocked Cholesky and of the triangular solves.
constexpr int NB = 64;

// Number of per-baseline partial sums written by the normal-equation build:
// P (4: P00, P11, Re P01, Im P01), zl (8), Q (4), zr (8).
constexpr int kPartials = 24;

// Device-side state of one Levenberg-Marquardt solve (FP64 throughout).
struct LMState {
  double mu, nu;          // damping and its growth factor
  double mu_eff;          // damping used in the current iteration
  double f;               // cost at the current Jones
  double f0;              // cost at the starting Jones
  double f_trial;         // cost at the trial Jones
  double g_norm2;         // ||g||^2 of the current right-hand side (refinement stop test)
  double maxdiag;         // max diag of the current normal matrix
  int32_t need_build;     // 1: rebuild H, g, f at the current Jones
  int32_t fresh;          // 1: initialise mu from tau at the next build
  int32_t notpd;          // factorisation of the current iteration failed
  int32_t refine_done;    // refinement converged (or not requested) this iteration
  int32_t refine_steps;   // refinement steps taken this iteration
  int32_t max_refine;     // max over iterations
  int32_t n_accept, n_reject, n_notpd;
  int32_t timeout;        // an inter-workgroup wait exceeded its bound
  int32_t iter;           // iterations done
  int32_t nonfinite;      // the cost at a built point was NaN/Inf
};

// Scratch for the persistent kernels: ticket counters, exit counter and per-tile flags.
struct SyncArea {
  uint32_t ticket;
  uint32_t exited;
  uint32_t abort;
  uint32_t pad;
};

}  // namespace ddc

// ---------------------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files; all enqueue on `st`).
// ---------------------------------------------------------------------------------------
namespace ddc {

struct ObsDev {
  int N, T, F;
  int64_t B;
  const double* u;
  const double* v;
  const double* w;
  const double* freq;
  const int32_t* ant_p;   // canonical baseline table, owned by the context
  const int32_t* ant_q;
};

// One solve's predict, as a self-contained descriptor (also the unit of the batched launch).
struct PredictJob {
  const double *u, *v, *w, *freq, *l, *m, *I, *Q, *U, *V;
  const int32_t* offs;      // device [K+1]
  int64_t B, plane;         // plane = T*F*B
  int T, F, K, pad;
  void* coh;                // [K][8][T][F][B] of the element type
  int64_t first_block;      // offset of this job in the batch's flattened block list
};

inline PredictJob make_predict_job(const ObsDev& o, int K, const int32_t* offs_dev,
                                   const double* l, const double* m, const double* I,
                                   const double* Q, const double* U, const double* V,
                                   void* coh) {
  PredictJob j;
  j.u = o.u; j.v = o.v; j.w = o.w; j.freq = o.freq;
  j.l = l; j.m = m; j.I = I; j.Q = Q; j.U = U; j.V = V;
  j.offs = offs_dev;
  j.B = o.B;
  j.plane = (int64_t)o.T * o.F * o.B;
  j.T = o.T; j.F = o.F; j.K = K; j.pad = 0;
  j.coh = coh;
  j.first_block = 0;
  return j;
}

// Work items of one job in the batched predict: 256-baseline tiles x (timeslot, channel);
// each item covers every cluster.
inline int64_t predict_blocks(const PredictJob& j) {
  return (j.B + 255) / 256 * (int64_t)j.T * j.F;
}

// k_predict.hip
// Station-factorised predict: phasors into `phasors` (phasor_bytes of scratch), then the
// coherencies of all K clusters, same layout as launch_predict.
size_t phasor_bytes(int N, int S, int T, int F, size_t es);
template <typename R>
hipError_t launch_predict_factored(const ObsDev& o, const double* su, const double* sv,
                                   const double* sw, int K, int S, const int32_t* offs_dev,
                                   const double* l, const double* m, const double* I,
                                   const double* Q, const double* U, const double* V,
                                   void* phasors, R* coh, hipStream_t st);
template <typename R>
hipError_t launch_predict_batch(const PredictJob* jobs_dev, int njobs, int64_t total_blocks,
                                int grid, hipStream_t st);
template <typename R>
hipError_t launch_predict(const ObsDev& o, int K, const int32_t* offs_dev, const int32_t* offs_host,
                          const double* l, const double* m, const double* I, const double* Q,
                          const double* U, const double* V, R* coh, hipStream_t st);

// One solve's initial residual R = V - sum_k J_k C_k J_k^H, as a self-contained descriptor
// (the unit of the batched launch).
struct ResidualJob {
  const void* vis;          // [8][T][F][B] of the element type
  const void* coh;          // [K][8][T][F][B]
  const double* jones;      // [K][N][8]
  const int32_t* ant_p;     // canonical baseline table
  const int32_t* ant_q;
  void* out;                // [8][T][F][B]
  int64_t B, plane;         // plane = T*F*B
  int N, K;
  int64_t first_block;      // offset of this job in the batch's flattened block list
};

inline int64_t residual_blocks(const ResidualJob& j) { return (j.plane + 255) / 256; }

// k_vis.hip
template <typename R>
hipError_t launch_residual_batch(const ResidualJob* jobs_dev, int njobs, int64_t total_blocks,
                                 int grid, hipStream_t st);
// jplanes (optional, 8 (k1 - k0) N elements): workspace for the Jones matrices as component
// planes when k1 - k0 >= 2 (same results, coalesced reads)
template <typename R>
hipError_t launch_add_model(const ObsDev& o, int k0, int k1, const R* in, const R* coh,
                            const double* jones, double alpha, R* out, double* cost_part,
                            int* nblk, hipStream_t st, R* jplanes = nullptr);
hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t st);
template <typename R>
hipError_t launch_build_neq(const ObsDev& o, const R* y, const R* coh, const double* jones,
                            R* Hc, int ld, R* part, double* cost_part, int* nblk,
                            const LMState* lm, hipStream_t st);
template <typename R>
hipError_t launch_neq_station(const ObsDev& o, const R* part, R* Hc, int ld, double* g,
                              double* diag, const LMState* lm, hipStream_t st);
template <typename R>
hipError_t launch_trial_cost(const ObsDev& o, const R* y, const R* coh, const double* jones,
                             const double* d, double* cost_part, int* nblk, const LMState* lm,
                             hipStream_t st);

// grad[k][s][8] = df/dx of every cluster from the residual res (per-baseline partials in
// part, [K][16][B]).
template <typename R>
hipError_t launch_cost_adjoint(const ObsDev& o, int K, const R* res, const R* coh,
                               const double* jones, R* part, double* grad, hipStream_t st);

// k_chol.hip
// Factor H + mu I (mu from mu_dev if non-null); with g != null also y = L^{-1} g.
// part: scratch of T * 2 * 4096 + T(T+1)/2 * 4096 + 64 T 64-bit slots: the worker's two
// look-ahead tiles per step (FP64 raw; FP32 tagged with seq), the tagged copies of the
// handed-over tiles and
// the forward solve's block messages (FP32 only; kEmpty before the launch, and again after).
// seq must differ from every earlier launch's on the same scratch and be nonzero, the tagged
// part zeroed when the scratch is first used.  flags: T(T+1)/2 + 2T, zero between launches.
template <typename R>
hipError_t launch_cholesky(const R* Hc, int ld, int n_pad, const double* mu_dev, double mu_host,
                           const double* g, double* y, R* Lt, R* Linv, void* part,
                           uint32_t seq, SyncArea* sync, uint32_t* flags, uint32_t* yflags,
                           int32_t* status, hipStream_t st, int n_wg);
// dst tile t = transpose of src tile t for ntiles packed 64x64 tiles, and likewise dst2/src2
// for ntiles2 tiles, in one launch (the backward solve reads the transposed factor and
// inverses); both the transposed copies and, in place, the source tiles are left in the
// solves' tile layout; skipped when lm reports a failed factorisation.
template <typename R>
hipError_t launch_transpose_tiles(R* src, R* dst, int ntiles, R* src2, R* dst2,
                                  int ntiles2, const LMState* lm, hipStream_t st);
// x = L^{-1} b (forward: Lt, Linv) or L^{-T} b (backward: pass the transposed copies LtT,
// LinvT); acc_out (nullable) += x.  psum and xpub: 64 T
// message slots each, holding kEmpty before the launch (they hold it again after it).
template <typename R>
hipError_t launch_trsv(bool forward, const R* Lt, const R* Linv, int n_pad, const double* b,
                       double* x, double* acc_out, uint64_t* psum, uint64_t* xpub,
                       SyncArea* sync, int32_t* status, const LMState* lm, int gate,
                       hipStream_t st);
// Fill n message slots with kEmpty.
hipError_t launch_fill_empty(uint64_t* p, int n, hipStream_t st);
// s = g - (H + mu I) d (FP64) via per-tile partials prow/pcol ([T(T+1)/2][64] each); the
// same launch closes the refinement step (refine_done once ||s||^2 <= tol2 ||g||^2, else
// refine_steps + 1), with sync->exited as its zeroed counter and T message slots in norms
// that hold kEmpty before the launch (and again after it).
template <typename R>
hipError_t launch_refine_resid(const R* Hc, int ld, int n_pad, const double* mu_dev,
                               const double* g, const double* d, double* s, uint64_t* norms,
                               double* prow, double* pcol, LMState* lm, int gate,
                               SyncArea* sync, double tol2, hipStream_t st);
hipError_t set_chol_smem_attr();

// noalloc.hip: the fixed device scratch of the entry point that allocates nothing.
constexpr int kNoAllocMaxStations = 512;
constexpr int64_t kNoAllocMaxBaselines = (int64_t)kNoAllocMaxStations * (kNoAllocMaxStations - 1) / 2;
constexpr int64_t kNoAllocMaxBlocks = 65536;   // cost partials: T*F*B <= 65536 * 256
struct NoAllocScratch {
  int32_t* ant;     // [2][B] canonical baseline table (rebuilt by every call)
  double* parts;    // [kNoAllocMaxBlocks] per-workgroup cost partials
  double* total;    // the cost
};
// Looks up the scratch array's address on `device` (which must be current), once per device.
hipError_t noalloc_setup(int device);
// The looked-up scratch of `device` (all null before noalloc_setup succeeded on it).
NoAllocScratch noalloc_scratch(int device);
hipError_t launch_baseline_table(int N, int64_t B, int32_t* ant_p, int32_t* ant_q,
                                 hipStream_t st);

// k_lm.hip
hipError_t launch_lm_init(LMState* st, int fresh, double mu, double nu, hipStream_t s);
hipError_t launch_lm_pre(LMState* st, const double* cost_part, int nblk, const double* diag,
                         int n8, const double* g, double tau, double mu_floor, int refine_max,
                         hipStream_t s);
// trace (nullable): the iteration's record goes to trace[iter].
hipError_t launch_lm_post(LMState* st, const double* cost_part, int nblk, const double* d,
                          const double* g, int n8, double* jones, ddc_lm_step* trace,
                          hipStream_t s);
hipError_t launch_solve_setup(LMState* st, const double* g, int n, double mu, int refine_max,
                              hipStream_t s);
hipError_t launch_copy_state(const LMState* st, LMState* dst, hipStream_t s);
template <typename R>
hipError_t launch_init_matrix(R* Hc, int ld, int n_real, hipStream_t s);
template <typename R>
hipError_t launch_expand_sym(const R* Hc, int ld, int n, R* out, hipStream_t s);
template <typename Rin, typename Rout>
hipError_t launch_convert(const Rin* in, int64_t n, int64_t n_out, Rout* out, hipStream_t s);

}  // namespace ddc
