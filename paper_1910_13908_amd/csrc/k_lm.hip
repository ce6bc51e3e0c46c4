// Device-side Levenberg-Marquardt control and small utility kernels.
//
// The LM iteration (Madsen, Nielsen & Tingleff 2004, Algorithm 3.16, Levenberg damping mu I)
// runs entirely on the device so a whole solve is enqueued without a host round trip:
//   pre:  after a (re)build, f = ||r||^2, max diag H and ||g||^2 from fixed-order sums;
//         a fresh start sets mu = tau * max diag H, nu = 2; then
//         mu_eff = max(mu, mu_floor * max diag H)  (floor against the gauge null space)
//   post: f' = ||r(x + d)||^2, rho = (f - f') / (d . (mu_eff d + g));
//         rho > 0: x += d, f = f', mu *= max(1/3, 1 - (2 rho - 1)^3), nu = 2, rebuild;
//         else (also when the factorisation failed, an inter-workgroup wait of the solve
//         timed out, or the denominator is not positive): mu *= nu, nu *= 2.
// A non-finite cost at a built point (NaN/Inf in the data, coherencies or Jones) is flagged
// for the host; its steps are all rejected since no trial cost compares below it.
// The denominator is the decrease predicted by the Gauss-Newton model of f = ||r||^2.
#include "common.h"

namespace ddc {
namespace {

constexpr int kThreads = 256;

__device__ double wg_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double wg_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Fixed-order sum of parts[0..n): thread i takes i, i+256, ...; then a fixed tree.  The
// per-thread loops here are unrolled so that a thread's loads are in flight together; the
// order of each thread's additions is unchanged.
__device__ double fixed_sum(const double* parts, int n, double* sh) {
  double v = 0.0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += kThreads) v += parts[i];
  return wg_sum(v, sh);
}

__global__ void k_lm_init(LMState* st, int fresh, double mu, double nu) {
  if (threadIdx.x == 0) {
    LMState s = {};
    s.mu = mu;
    s.nu = nu;
    s.fresh = fresh;
    s.need_build = 1;
    *st = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_lm_pre(LMState* st, const double* cost_part,
                                                     int nblk, const double* diag, int n8,
                                                     const double* g, double tau,
                                                     double mu_floor, int refine_max) {
  __shared__ double sh[kThreads];
  const int need = st->need_build;
  if (need) {
    const double f = fixed_sum(cost_part, nblk, sh);
    double mx = 0.0, gg = 0.0;
#pragma unroll 8
    for (int i = threadIdx.x; i < n8; i += kThreads) {
      mx = fmax(mx, diag[i]);
      gg = fma(g[i], g[i], gg);
    }
    mx = wg_max(mx, sh);
    gg = wg_sum(gg, sh);
    if (threadIdx.x == 0) {
      st->f = f;
      if (!isfinite(f)) st->nonfinite = 1;
      st->maxdiag = mx;
      st->g_norm2 = gg;
      if (st->iter == 0) st->f0 = f;
      if (st->fresh) {
        st->mu = tau * mx;
        st->nu = 2.0;
        st->fresh = 0;
      }
      st->need_build = 0;
    }
  }
  if (threadIdx.x == 0) {
    st->mu_eff = fmax(st->mu, mu_floor * st->maxdiag);
    st->notpd = 0;
    st->refine_done = refine_max > 0 ? 0 : 1;
    st->refine_steps = 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_lm_post(LMState* st, const double* cost_part,
                                                      int nblk, const double* d,
                                                      const double* g, int n8,
                                                      double* jones, ddc_lm_step* trace) {
  __shared__ double sh[kThreads];
  __shared__ int s_acc;
  // bit 0: not positive definite; bit 1: a wait of the factorisation timed out; a timed-out
  // wait of a triangular solve or refinement step leaves d unfinished, so it fails as well
  const int fail = st->notpd | (st->timeout ? 2 : 0);
  double fnew = 0.0, den = 0.0;
  if (!fail) {
    fnew = fixed_sum(cost_part, nblk, sh);
    const double mu = st->mu_eff;
    double v = 0.0;
#pragma unroll 8
    for (int i = threadIdx.x; i < n8; i += kThreads) v = fma(d[i], fma(mu, d[i], g[i]), v);
    den = wg_sum(v, sh);
  }
  if (threadIdx.x == 0) {
    int acc = 0;
    double rho = 0.0;
    if (!fail && den > 0.0 && isfinite(den) && isfinite(fnew)) {
      rho = (st->f - fnew) / den;
      acc = rho > 0.0;
    }
    if (fail & 2) st->timeout = 1;
    const double mu_eff = st->mu_eff;
    if (acc) {
      st->f = fnew;
      const double t = 2.0 * rho - 1.0;
      st->mu *= fmax(1.0 / 3.0, 1.0 - t * t * t);
      st->nu = 2.0;
      st->need_build = 1;
      st->n_accept += 1;
    } else {
      st->mu *= st->nu;
      st->nu *= 2.0;
      st->n_reject += 1;
      if (fail & 1) st->n_notpd += 1;
    }
    if (st->refine_steps > st->max_refine) st->max_refine = st->refine_steps;
    if (trace) {
      ddc_lm_step r;
      r.cost = st->f;
      r.mu_eff = mu_eff;
      r.mu = st->mu;
      r.nu = st->nu;
      r.accepted = acc;
      r.refine_steps = st->refine_steps;
      trace[st->iter] = r;
    }
    st->iter += 1;
    s_acc = acc;
  }
  __syncthreads();
  if (s_acc) {
#pragma unroll 8
    for (int i = threadIdx.x; i < n8; i += kThreads) jones[i] += d[i];
  }
}

// Stand-alone damped solve: mu_eff = mu, ||g||^2, refinement bookkeeping.
__global__ __launch_bounds__(kThreads) void k_solve_setup(LMState* st, const double* g, int n,
                                                          double mu, int refine_max) {
  __shared__ double sh[kThreads];
  double gg = 0.0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += kThreads) gg = fma(g[i], g[i], gg);
  gg = wg_sum(gg, sh);
  if (threadIdx.x == 0) {
    LMState s = {};
    s.mu_eff = mu;
    s.g_norm2 = gg;
    s.refine_done = refine_max > 0 ? 0 : 1;
    *st = s;
  }
}

// Zero the whole column-major matrix storage and put 1 on the diagonal of the padding.
template <typename R>
__global__ void k_init_matrix(R* Hc, int64_t ld, int n_real) {
  const int64_t total = ld * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / ld, r = i % ld;
    Hc[i] = (r == c && r >= n_real) ? (R)1 : (R)0;
  }
}

// Column-major lower (ld) -> full symmetric row-major n x n.
template <typename R>
__global__ void k_expand_sym(const R* __restrict__ Hc, int64_t ld, int n, R* __restrict__ out) {
  const int64_t total = (int64_t)n * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, c = i % n;
    out[i] = (r >= c) ? Hc[c * ld + r] : Hc[r * ld + c];
  }
}

template <typename Rin, typename Rout>
__global__ void k_convert(const Rin* __restrict__ in, int64_t n, int64_t n_out, Rout* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = i < n ? (Rout)in[i] : (Rout)0;
}

__global__ void k_copy_state(const LMState* st, LMState* dst) {
  if (threadIdx.x == 0) *dst = *st;
}

}  // namespace

hipError_t launch_lm_init(LMState* st, int fresh, double mu, double nu, hipStream_t s) {
  hipLaunchKernelGGL(k_lm_init, dim3(1), dim3(64), 0, s, st, fresh, mu, nu);
  return hipGetLastError();
}
hipError_t launch_lm_pre(LMState* st, const double* cost_part, int nblk, const double* diag,
                         int n8, const double* g, double tau, double mu_floor, int refine_max,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_lm_pre, dim3(1), dim3(kThreads), 0, s, st, cost_part, nblk, diag, n8, g,
                     tau, mu_floor, refine_max);
  return hipGetLastError();
}
hipError_t launch_lm_post(LMState* st, const double* cost_part, int nblk, const double* d,
                          const double* g, int n8, double* jones, ddc_lm_step* trace,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_lm_post, dim3(1), dim3(kThreads), 0, s, st, cost_part, nblk, d, g, n8,
                     jones, trace);
  return hipGetLastError();
}
hipError_t launch_solve_setup(LMState* st, const double* g, int n, double mu, int refine_max,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_solve_setup, dim3(1), dim3(kThreads), 0, s, st, g, n, mu, refine_max);
  return hipGetLastError();
}
hipError_t launch_copy_state(const LMState* st, LMState* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_state, dim3(1), dim3(64), 0, s, st, dst);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_init_matrix(R* Hc, int ld, int n_real, hipStream_t s) {
  hipLaunchKernelGGL(k_init_matrix<R>, dim3(1024), dim3(kThreads), 0, s, Hc, (int64_t)ld, n_real);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_expand_sym(const R* Hc, int ld, int n, R* out, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_sym<R>, dim3(1024), dim3(kThreads), 0, s, Hc, (int64_t)ld, n, out);
  return hipGetLastError();
}
template <typename Rin, typename Rout>
hipError_t launch_convert(const Rin* in, int64_t n, int64_t n_out, Rout* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Rin, Rout>), dim3(256), dim3(kThreads), 0, s, in, n, n_out, out);
  return hipGetLastError();
}

template hipError_t launch_init_matrix<float>(float*, int, int, hipStream_t);
template hipError_t launch_init_matrix<double>(double*, int, int, hipStream_t);
template hipError_t launch_expand_sym<float>(const float*, int, int, float*, hipStream_t);
template hipError_t launch_expand_sym<double>(const double*, int, int, double*, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_convert<double, float>(const double*, int64_t, int64_t, float*, hipStream_t);

}  // namespace ddc
