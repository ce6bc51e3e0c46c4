// Per-visibility passes of the calibration hot path: model application / residual, the
// normal-equation build of one cluster, the per-station assembly and the trial cost.
//
// Model of baseline (p, q) for cluster k: M = J_p C J_q^H (measurement equation; paper
// Section 2: one Jones solution per station per cluster, Section 3: N(N-1)/2 baselines).
//
// Normal equations (Gauss-Newton for f = sum ||Y - M||^2 with real parameters
// x[8p + 2e + {0,1}] = (Re, Im) of (J_p)_e, e = 00, 01, 10, 11).  With G = C J_q^H,
// Hm = J_p C, residual Rr = Y - M and E_i = c_i e_a e_b^T (c_i = 1 or i):
//   cross block  (p,q)[i][j] = Re(conj(c_i c_j) S_abcd),  S_abcd = sum conj(G_bc) Hm_ad
//   diagonal     (p,p)[i][j] = [a==c] (Re(conj(c_i) c_j P_db) + Re(c_i conj(c_j) Q_bd))
//                P = sum_{p left} G G^H,  Q = sum_{p right} Hm^H Hm
//   right side   g_p = (Re, Im) of sum_{p left} Rr G^H + sum_{p right} Rr^H Hm
// One thread owns one baseline and reduces over all timeslots and channels; cross blocks
// go straight to the column-major lower normal matrix (row 8q+j > column 8p+i: the eight
// entries of one column are contiguous and neighbouring threads own neighbouring q, so the
// stores coalesce).  Per-station sums use per-baseline partials (structure of arrays) and a
// fixed-order reduction, so results do not depend on scheduling.
#include "common.h"

namespace ddc {
namespace {

constexpr int kThreads = 256;

template <typename R>
struct Cx {
  R r, i;
};

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return {fma(a.r, b.r, a.i * b.i), fma(a.i, b.r, -a.r * b.i)};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc) {
  return {fma(a.r, b.r, fma(-a.i, b.i, acc.r)), fma(a.r, b.i, fma(a.i, b.r, acc.i))};
}
// acc + a * conj(b)
template <typename R>
__device__ __forceinline__ Cx<R> cfmac(Cx<R> a, Cx<R> b, Cx<R> acc) {
  return {fma(a.r, b.r, fma(a.i, b.i, acc.r)), fma(a.i, b.r, fma(-a.r, b.i, acc.i))};
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cfmaca(Cx<R> a, Cx<R> b, Cx<R> acc) {
  return {fma(a.r, b.r, fma(a.i, b.i, acc.r)), fma(a.r, b.i, fma(-a.i, b.r, acc.i))};
}

// 2x2 complex, row-major entries 00, 01, 10, 11.
template <typename R>
struct M2 {
  Cx<R> e[4];
};

template <typename R>
__device__ __forceinline__ M2<R> mmul(const M2<R>& A, const M2<R>& B) {
  M2<R> o;
  o.e[0] = cfma(A.e[1], B.e[2], cmul(A.e[0], B.e[0]));
  o.e[1] = cfma(A.e[1], B.e[3], cmul(A.e[0], B.e[1]));
  o.e[2] = cfma(A.e[3], B.e[2], cmul(A.e[2], B.e[0]));
  o.e[3] = cfma(A.e[3], B.e[3], cmul(A.e[2], B.e[1]));
  return o;
}
// A B^H: [ij] = sum_k A_ik conj(B_jk)
template <typename R>
__device__ __forceinline__ M2<R> mmul_bh(const M2<R>& A, const M2<R>& B) {
  M2<R> o;
  o.e[0] = cfmac(A.e[1], B.e[1], cmulc(A.e[0], B.e[0]));
  o.e[1] = cfmac(A.e[1], B.e[3], cmulc(A.e[0], B.e[2]));
  o.e[2] = cfmac(A.e[3], B.e[1], cmulc(A.e[2], B.e[0]));
  o.e[3] = cfmac(A.e[3], B.e[3], cmulc(A.e[2], B.e[2]));
  return o;
}

template <typename R>
__device__ __forceinline__ M2<R> load_jones(const double* __restrict__ J, int st) {
  M2<R> o;
  const double* p = J + 8 * (int64_t)st;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.e[e] = {(R)p[2 * e], (R)p[2 * e + 1]};
  return o;
}

// The same Jones matrix from component planes (plane c holds component c of every station,
// already rounded to R): equal values, one coalesced load per component across a wave.
template <typename R>
__device__ __forceinline__ M2<R> load_jones_planes(const R* __restrict__ P, int64_t N, int st) {
  M2<R> o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.e[e] = {P[(2 * e) * N + st], P[(2 * e + 1) * N + st]};
  return o;
}

// (J + d) for the trial step, summed in FP64 before rounding to R.
template <typename R>
__device__ __forceinline__ M2<R> load_jones_step(const double* __restrict__ J,
                                                 const double* __restrict__ d, int st) {
  M2<R> o;
  const double* p = J + 8 * (int64_t)st;
  const double* q = d + 8 * (int64_t)st;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.e[e] = {(R)(p[2 * e] + q[2 * e]), (R)(p[2 * e + 1] + q[2 * e + 1])};
  return o;
}

template <typename R>
__device__ __forceinline__ M2<R> load_vis(const R* __restrict__ base, int64_t plane, int64_t idx) {
  M2<R> o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.e[e] = {base[(2 * e) * plane + idx], base[(2 * e + 1) * plane + idx]};
  return o;
}

template <typename R>
__device__ __forceinline__ double norm2(const M2<R>& A) {
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double a = (double)A.e[e].r, b = (double)A.e[e].i;
    s = fma(a, a, fma(b, b, s));
  }
  return s;
}

// Deterministic block sum of one double per thread (fixed tree order); result in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------------------
// out = in + alpha * sum_{k in [k0,k1)} J_k C_k J_k^H; optional cost partials of ||out||^2.
// ---------------------------------------------------------------------------------------
// One element i of out = in + alpha * sum_k J_k C_k J_k^H; returns ||out_i||^2.  Shared by
// the single-problem kernel and the batched one, so both round identically.  With PL the
// Jones matrices come from jpl, the component planes of clusters k0.. (the same values).
template <typename R, bool PL = false>
__device__ __forceinline__ double add_model_elem(
    const R* __restrict__ in, const R* __restrict__ coh, const double* __restrict__ jones,
    const R* __restrict__ jpl, const int32_t* __restrict__ ant_p,
    const int32_t* __restrict__ ant_q, int64_t B, int64_t plane, int N, int k0, int k1,
    R alpha, R* __restrict__ out, int64_t i) {
  const int64_t b = i % B;
  const int p = ant_p[b], q = ant_q[b];
  M2<R> acc = load_vis(in, plane, i);
  for (int k = k0; k < k1; ++k) {
    M2<R> Jp, Jq;
    if constexpr (PL) {
      const R* P = jpl + (int64_t)(k - k0) * 8 * N;
      Jp = load_jones_planes<R>(P, N, p);
      Jq = load_jones_planes<R>(P, N, q);
    } else {
      Jp = load_jones<R>(jones + (int64_t)k * 8 * N, p);
      Jq = load_jones<R>(jones + (int64_t)k * 8 * N, q);
    }
    const M2<R> C = load_vis(coh + (int64_t)k * 8 * plane, plane, i);
    const M2<R> M = mmul_bh(mmul(Jp, C), Jq);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc.e[e].r = fma(alpha, M.e[e].r, acc.e[e].r);
      acc.e[e].i = fma(alpha, M.e[e].i, acc.e[e].i);
    }
  }
  if (out) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      out[(2 * e) * plane + i] = acc.e[e].r;
      out[(2 * e + 1) * plane + i] = acc.e[e].i;
    }
  }
  return norm2(acc);
}

template <typename R, bool PL>
__global__ __launch_bounds__(kThreads) void k_add_model(
    const R* __restrict__ in, const R* __restrict__ coh, const double* __restrict__ jones,
    const R* __restrict__ jpl, const int32_t* __restrict__ ant_p,
    const int32_t* __restrict__ ant_q, int64_t B, int64_t plane, int N, int k0, int k1,
    R alpha, R* __restrict__ out, double* __restrict__ cost_part) {
  __shared__ double sh[kThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double cst = 0.0;
  if (i < plane)
    cst = add_model_elem<R, PL>(in, coh, jones, jpl, ant_p, ant_q, B, plane, N, k0, k1, alpha,
                                out, i);
  if (cost_part) {
    const double s = block_sum(cst, sh);
    if (threadIdx.x == 0) cost_part[blockIdx.x] = s;
  }
}

// Jones matrices of nk clusters (station-major, 8 doubles per station) as component planes
// rounded to R: planes[(k * 8 + c) * N + n] = J_k[n][c].  A wave's gather of 64 stations'
// 64-byte records touches 32 cache lines per 16-byte load; from the planes each component
// is one coalesced load.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_jones_planes(const double* __restrict__ jones,
                                                           int N, int nk, R* __restrict__ planes) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)nk * 8 * N) return;
  const int64_t kc = t / N;
  const int64_t n = t - kc * N;
  planes[t] = (R)jones[((kc >> 3) * N + n) * 8 + (kc & 7)];
}

// Initial residuals of several solves in one persistent launch: the workgroups walk the
// flattened list of (job, 256-element block) items with a grid stride; each element runs
// add_model_elem with every cluster and alpha = -1, as k_add_model does for one solve.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_residual_batch(const ResidualJob* __restrict__ jobs,
                                                            int njobs, int64_t total) {
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    int jj = 0;
    while (jj + 1 < njobs && jobs[jj + 1].first_block <= vb) ++jj;
    const ResidualJob& j = jobs[jj];
    const int64_t i = (vb - j.first_block) * kThreads + threadIdx.x;
    if (i < j.plane)
      (void)add_model_elem<R>(reinterpret_cast<const R*>(j.vis), reinterpret_cast<const R*>(j.coh),
                              j.jones, nullptr, j.ant_p, j.ant_q, j.B, j.plane, j.N, 0, j.K, (R)-1,
                              reinterpret_cast<R*>(j.out), i);
  }
}

// ---------------------------------------------------------------------------------------
// Normal equations of one cluster: cross blocks, per-baseline partials, cost partials.
// ---------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_build_neq(
    const R* __restrict__ y, const R* __restrict__ coh, const double* __restrict__ jones,
    const int32_t* __restrict__ ant_p, const int32_t* __restrict__ ant_q, int64_t B, int TF,
    R* __restrict__ Hc, int64_t ld, R* __restrict__ part, double* __restrict__ cost_part,
    const LMState* __restrict__ lm) {
  if (lm && !lm->need_build) return;
  __shared__ double sh[kThreads / 64];
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t plane = (int64_t)TF * B;
  double cst = 0.0;
  if (b < B) {
    const int p = ant_p[b], q = ant_q[b];
    const M2<R> Jp = load_jones<R>(jones, p);
    const M2<R> Jq = load_jones<R>(jones, q);
    Cx<R> S[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) S[i] = {0, 0};
    R P00 = 0, P11 = 0, Q00 = 0, Q11 = 0;
    Cx<R> P01 = {0, 0}, Q01 = {0, 0};
    M2<R> zl, zr;
#pragma unroll
    for (int e = 0; e < 4; ++e) zl.e[e] = zr.e[e] = {0, 0};
    for (int tf = 0; tf < TF; ++tf) {
      const int64_t idx = (int64_t)tf * B + b;
      const M2<R> C = load_vis(coh, plane, idx);
      const M2<R> Y = load_vis(y, plane, idx);
      const M2<R> G = mmul_bh(C, Jq);     // C J_q^H
      const M2<R> Hm = mmul(Jp, C);       // J_p C
      const M2<R> M = mmul_bh(Hm, Jq);
      M2<R> Rr;
#pragma unroll
      for (int e = 0; e < 4; ++e) Rr.e[e] = {Y.e[e].r - M.e[e].r, Y.e[e].i - M.e[e].i};
      cst += norm2(Rr);
      // S_abcd += conj(G_bc) Hm_ad
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
              const int s = a * 8 + bb * 4 + c * 2 + d;
              S[s] = cfmaca(G.e[bb * 2 + c], Hm.e[a * 2 + d], S[s]);
            }
      // P += G G^H (Hermitian), Q += Hm^H Hm
      P00 += G.e[0].r * G.e[0].r + G.e[0].i * G.e[0].i + G.e[1].r * G.e[1].r + G.e[1].i * G.e[1].i;
      P11 += G.e[2].r * G.e[2].r + G.e[2].i * G.e[2].i + G.e[3].r * G.e[3].r + G.e[3].i * G.e[3].i;
      P01 = cfmac(G.e[1], G.e[3], cfmac(G.e[0], G.e[2], P01));
      Q00 += Hm.e[0].r * Hm.e[0].r + Hm.e[0].i * Hm.e[0].i + Hm.e[2].r * Hm.e[2].r + Hm.e[2].i * Hm.e[2].i;
      Q11 += Hm.e[1].r * Hm.e[1].r + Hm.e[1].i * Hm.e[1].i + Hm.e[3].r * Hm.e[3].r + Hm.e[3].i * Hm.e[3].i;
      Q01 = cfmaca(Hm.e[2], Hm.e[3], cfmaca(Hm.e[0], Hm.e[1], Q01));
      // zl += Rr G^H, zr += Rr^H Hm
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          zl.e[i * 2 + k] = cfmac(Rr.e[i * 2 + 1], G.e[k * 2 + 1], cfmac(Rr.e[i * 2 + 0], G.e[k * 2 + 0], zl.e[i * 2 + k]));
          zr.e[i * 2 + k] = cfmaca(Rr.e[1 * 2 + i], Hm.e[1 * 2 + k], cfmaca(Rr.e[0 * 2 + i], Hm.e[0 * 2 + k], zr.e[i * 2 + k]));
        }
    }
    // cross block: column 8p+i, rows 8q..8q+7
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int a = i >> 2, bb = (i >> 1) & 1, ci = i & 1;
      R vals[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = j >> 2, d = (j >> 1) & 1, cj = j & 1;
        const Cx<R> s = S[a * 8 + bb * 4 + c * 2 + d];
        vals[j] = (ci == 0 && cj == 0) ? s.r : ((ci == 1 && cj == 1) ? -s.r : s.i);
      }
      R* dst = Hc + (int64_t)(8 * p + i) * ld + 8 * (int64_t)q;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j] = vals[j];
    }
    R pv[kPartials] = {P00, P11, P01.r, P01.i,
                       zl.e[0].r, zl.e[0].i, zl.e[1].r, zl.e[1].i, zl.e[2].r, zl.e[2].i, zl.e[3].r, zl.e[3].i,
                       Q00, Q11, Q01.r, Q01.i,
                       zr.e[0].r, zr.e[0].i, zr.e[1].r, zr.e[1].i, zr.e[2].r, zr.e[2].i, zr.e[3].r, zr.e[3].i};
#pragma unroll
    for (int k = 0; k < kPartials; ++k) part[(int64_t)k * B + b] = pv[k];
  }
  const double s = block_sum(cst, sh);
  if (threadIdx.x == 0) cost_part[blockIdx.x] = s;
}

// Re(coef * z) for coef in {1, i, -i}: 0 -> 1, 1 -> i, 2 -> -i
template <typename R>
__device__ __forceinline__ R re_coef(int coef, R zr, R zi) {
  return coef == 0 ? zr : (coef == 1 ? -zi : zi);
}

// One workgroup per station: fixed-order sums of the per-baseline partials, then the 8x8
// diagonal block, g and the diagonal.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_neq_station(
    const R* __restrict__ part, int N, int64_t B, R* __restrict__ Hc, int64_t ld,
    double* __restrict__ g, double* __restrict__ diag, const LMState* __restrict__ lm) {
  if (lm && !lm->need_build) return;
  __shared__ R red[kPartials][kThreads];
  __shared__ R tot[kPartials];
  const int s = blockIdx.x;
  const int tid = threadIdx.x;
  R acc[kPartials];
#pragma unroll
  for (int k = 0; k < kPartials; ++k) acc[k] = 0;
  // left: baselines (s, q), q > s, contiguous from b0
  const int64_t b0 = (int64_t)s * (2 * (int64_t)N - s - 1) / 2;
  for (int j = tid; j < N - 1 - s; j += kThreads) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += part[(int64_t)k * B + b0 + j];
  }
  // right: baselines (p, s), p < s
  for (int p = tid; p < s; p += kThreads) {
    const int64_t b = (int64_t)p * (2 * (int64_t)N - p - 1) / 2 + (s - p - 1);
#pragma unroll
    for (int k = 12; k < kPartials; ++k) acc[k] += part[(int64_t)k * B + b];
  }
#pragma unroll
  for (int k = 0; k < kPartials; ++k) red[k][tid] = acc[k];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int k = 0; k < kPartials; ++k) red[k][tid] += red[k][tid + w];
    }
    __syncthreads();
  }
  if (tid < kPartials) tot[tid] = red[tid][0];
  __syncthreads();
  if (tid < 64) {
    const int i = tid >> 3, j = tid & 7;
    const int a = i >> 2, bb = (i >> 1) & 1, ci = i & 1;
    const int c = j >> 2, d = (j >> 1) & 1, cj = j & 1;
    R val = 0;
    if (a == c) {
      // P_db and Q_bd from the Hermitian partials (P00, P11, P01)
      auto herm = [&](int base, int r, int cc, R& zr_, R& zi_) {
        if (r == cc) {
          zr_ = tot[base + (r == 0 ? 0 : 1)];
          zi_ = 0;
        } else if (r == 0) {
          zr_ = tot[base + 2];
          zi_ = tot[base + 3];
        } else {
          zr_ = tot[base + 2];
          zi_ = -tot[base + 3];
        }
      };
      R pr, pi, qr, qi;
      herm(0, d, bb, pr, pi);     // P_db
      herm(12, bb, d, qr, qi);    // Q_bd
      // conj(c_i) c_j: (0,0)->1 (0,1)->i (1,0)->-i (1,1)->1
      const int cl = (ci == cj) ? 0 : (ci == 0 ? 1 : 2);
      // c_i conj(c_j): (0,0)->1 (0,1)->-i (1,0)->i (1,1)->1
      const int cr = (ci == cj) ? 0 : (ci == 0 ? 2 : 1);
      val = re_coef(cl, pr, pi) + re_coef(cr, qr, qi);
    }
    Hc[(int64_t)(8 * s + j) * ld + 8 * (int64_t)s + i] = val;
    if (i == j) diag[8 * s + i] = (double)val;
  }
  if (tid < 8) {
    const int e = tid >> 1, im = tid & 1;
    g[8 * s + tid] = (double)tot[4 + 2 * e + im] + (double)tot[16 + 2 * e + im];
  }
}

// Trial cost ||y - (J+d)_p C (J+d)_q^H||^2: same per-thread decomposition as the build.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_trial_cost(
    const R* __restrict__ y, const R* __restrict__ coh, const double* __restrict__ jones,
    const double* __restrict__ d, const int32_t* __restrict__ ant_p,
    const int32_t* __restrict__ ant_q, int64_t B, int TF, double* __restrict__ cost_part,
    const LMState* __restrict__ lm) {
  if (lm && (lm->notpd || lm->timeout)) return;
  __shared__ double sh[kThreads / 64];
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t plane = (int64_t)TF * B;
  double cst = 0.0;
  if (b < B) {
    const int p = ant_p[b], q = ant_q[b];
    const M2<R> Jp = load_jones_step<R>(jones, d, p);
    const M2<R> Jq = load_jones_step<R>(jones, d, q);
    for (int tf = 0; tf < TF; ++tf) {
      const int64_t idx = (int64_t)tf * B + b;
      const M2<R> C = load_vis(coh, plane, idx);
      const M2<R> Y = load_vis(y, plane, idx);
      const M2<R> M = mmul_bh(mmul(Jp, C), Jq);
      M2<R> Rr;
#pragma unroll
      for (int e = 0; e < 4; ++e) Rr.e[e] = {Y.e[e].r - M.e[e].r, Y.e[e].i - M.e[e].i};
      cst += norm2(Rr);
    }
  }
  const double s = block_sum(cst, sh);
  if (threadIdx.x == 0) cost_part[blockIdx.x] = s;
}


// ---------------------------------------------------------------------------------------
// Adjoint of the cost f = ||R||^2, R = V - sum_k J_{p,k} C_k J_{q,k}^H, with respect to every
// cluster's Jones in the real-pair view: df/dx_k = -2 (Re, Im) of
//   sum_{p left} R G_k^H + sum_{p right} R^H Hm_k,   G_k = C_k J_{q,k}^H, Hm_k = J_{p,k} C_k.
// Pass 1: one thread per (baseline, cluster) reduces over T*F into per-baseline partials
// (the clusters of one baseline tile are neighbouring workgroups, so R is re-read from L2).
// Pass 2: one workgroup per (station, cluster) sums the partials in a fixed order.
// ---------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_cost_adjoint(
    const R* __restrict__ res, const R* __restrict__ coh, const double* __restrict__ jones,
    const int32_t* __restrict__ ant_p, const int32_t* __restrict__ ant_q, int64_t B, int TF,
    int N, int K, R* __restrict__ part) {
  const int k = blockIdx.x % K;
  const int64_t b = (int64_t)(blockIdx.x / K) * kThreads + threadIdx.x;
  if (b >= B) return;
  const int64_t plane = (int64_t)TF * B;
  const int p = ant_p[b], q = ant_q[b];
  const double* Jk = jones + (int64_t)k * 8 * N;
  const M2<R> Jp = load_jones<R>(Jk, p);
  const M2<R> Jq = load_jones<R>(Jk, q);
  const R* ck = coh + (int64_t)k * 8 * plane;
  M2<R> zl, zr;
#pragma unroll
  for (int e = 0; e < 4; ++e) zl.e[e] = zr.e[e] = {0, 0};
  for (int tf = 0; tf < TF; ++tf) {
    const int64_t idx = (int64_t)tf * B + b;
    const M2<R> C = load_vis(ck, plane, idx);
    const M2<R> Rr = load_vis(res, plane, idx);
    const M2<R> G = mmul_bh(C, Jq);
    const M2<R> Hm = mmul(Jp, C);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        zl.e[i * 2 + kk] = cfmac(Rr.e[i * 2 + 1], G.e[kk * 2 + 1], cfmac(Rr.e[i * 2 + 0], G.e[kk * 2 + 0], zl.e[i * 2 + kk]));
        zr.e[i * 2 + kk] = cfmaca(Rr.e[1 * 2 + i], Hm.e[1 * 2 + kk], cfmaca(Rr.e[0 * 2 + i], Hm.e[0 * 2 + kk], zr.e[i * 2 + kk]));
      }
  }
  R* out = part + (int64_t)k * 16 * B + b;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    out[(2 * e) * B] = zl.e[e].r;
    out[(2 * e + 1) * B] = zl.e[e].i;
    out[(8 + 2 * e) * B] = zr.e[e].r;
    out[(8 + 2 * e + 1) * B] = zr.e[e].i;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_adjoint_station(const R* __restrict__ part, int N,
                                                             int64_t B, double* __restrict__ grad) {
  __shared__ R red[8][kThreads];
  const int s = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const R* pk = part + (int64_t)k * 16 * B;
  R acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0;
  const int64_t b0 = (int64_t)s * (2 * (int64_t)N - s - 1) / 2;
  for (int j = tid; j < N - 1 - s; j += kThreads) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += pk[(int64_t)i * B + b0 + j];
  }
  for (int p = tid; p < s; p += kThreads) {
    const int64_t b = (int64_t)p * (2 * (int64_t)N - p - 1) / 2 + (s - p - 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += pk[(int64_t)(8 + i) * B + b];
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) red[i][tid] = acc[i];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int i = 0; i < 8; ++i) red[i][tid] += red[i][tid + w];
    }
    __syncthreads();
  }
  if (tid < 8) grad[((int64_t)k * N + s) * 8 + tid] = -2.0 * (double)red[tid][0];
}

__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ parts, int n,
                                                  double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += parts[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) *out = s;
}

}  // namespace

template <typename R>
hipError_t launch_add_model(const ObsDev& o, int k0, int k1, const R* in, const R* coh,
                            const double* jones, double alpha, R* out, double* cost_part,
                            int* nblk, hipStream_t st, R* jplanes) {
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  const unsigned g = (unsigned)((plane + kThreads - 1) / kThreads);
  if (nblk) *nblk = (int)g;
  // several clusters: their Jones matrices are read from component planes
  const R* jpl = nullptr;
  if (jplanes && k1 - k0 >= 2) {
    const int64_t n = (int64_t)(k1 - k0) * 8 * o.N;
    hipLaunchKernelGGL(k_jones_planes<R>, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, jones + (int64_t)k0 * 8 * o.N, o.N, k1 - k0,
                       jplanes);
    jpl = jplanes;
  }
  if (jpl)
    hipLaunchKernelGGL((k_add_model<R, true>), dim3(g), dim3(kThreads), 0, st, in, coh, jones,
                       jpl, o.ant_p, o.ant_q, o.B, plane, o.N, k0, k1, (R)alpha, out, cost_part);
  else
    hipLaunchKernelGGL((k_add_model<R, false>), dim3(g), dim3(kThreads), 0, st, in, coh, jones,
                       jpl, o.ant_p, o.ant_q, o.B, plane, o.N, k0, k1, (R)alpha, out, cost_part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_residual_batch(const ResidualJob* jobs_dev, int njobs, int64_t total_blocks,
                                 int grid, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  const int g = (int)(total_blocks < grid ? total_blocks : grid);
  hipLaunchKernelGGL(k_residual_batch<R>, dim3(g), dim3(kThreads), 0, st, jobs_dev, njobs,
                     total_blocks);
  return hipGetLastError();
}

hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, st, parts, n, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_build_neq(const ObsDev& o, const R* y, const R* coh, const double* jones,
                            R* Hc, int ld, R* part, double* cost_part, int* nblk,
                            const LMState* lm, hipStream_t st) {
  const unsigned g = (unsigned)((o.B + kThreads - 1) / kThreads);
  if (nblk) *nblk = (int)g;
  hipLaunchKernelGGL(k_build_neq<R>, dim3(g), dim3(kThreads), 0, st, y, coh, jones, o.ant_p,
                     o.ant_q, o.B, o.T * o.F, Hc, (int64_t)ld, part, cost_part, lm);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_neq_station(const ObsDev& o, const R* part, R* Hc, int ld, double* g,
                              double* diag, const LMState* lm, hipStream_t st) {
  hipLaunchKernelGGL(k_neq_station<R>, dim3(o.N), dim3(kThreads), 0, st, part, o.N, o.B, Hc,
                     (int64_t)ld, g, diag, lm);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_trial_cost(const ObsDev& o, const R* y, const R* coh, const double* jones,
                             const double* d, double* cost_part, int* nblk, const LMState* lm,
                             hipStream_t st) {
  const unsigned g = (unsigned)((o.B + kThreads - 1) / kThreads);
  if (nblk) *nblk = (int)g;
  hipLaunchKernelGGL(k_trial_cost<R>, dim3(g), dim3(kThreads), 0, st, y, coh, jones, d, o.ant_p,
                     o.ant_q, o.B, o.T * o.F, cost_part, lm);
  return hipGetLastError();
}


template <typename R>
hipError_t launch_cost_adjoint(const ObsDev& o, int K, const R* res, const R* coh,
                               const double* jones, R* part, double* grad, hipStream_t st) {
  const unsigned tiles = (unsigned)((o.B + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_cost_adjoint<R>, dim3(tiles * (unsigned)K), dim3(kThreads), 0, st, res, coh,
                     jones, o.ant_p, o.ant_q, o.B, o.T * o.F, o.N, K, part);
  hipLaunchKernelGGL(k_adjoint_station<R>, dim3(o.N, K), dim3(kThreads), 0, st, part, o.N, o.B, grad);
  return hipGetLastError();
}

#define DDC_INST(R)                                                                          \
  template hipError_t launch_residual_batch<R>(const ResidualJob*, int, int64_t, int,          \
                                               hipStream_t);                                   \
  template hipError_t launch_add_model<R>(const ObsDev&, int, int, const R*, const R*,        \
                                          const double*, double, R*, double*, int*,           \
                                          hipStream_t, R*);                                   \
  template hipError_t launch_build_neq<R>(const ObsDev&, const R*, const R*, const double*,   \
                                          R*, int, R*, double*, int*, const LMState*,          \
                                          hipStream_t);                                       \
  template hipError_t launch_neq_station<R>(const ObsDev&, const R*, R*, int, double*,        \
                                            double*, const LMState*, hipStream_t);            \
  template hipError_t launch_trial_cost<R>(const ObsDev&, const R*, const R*, const double*,  \
                                           const double*, double*, int*, const LMState*,      \
                                           hipStream_t);                                       \
  template hipError_t launch_cost_adjoint<R>(const ObsDev&, int, const R*, const R*,          \
                                             const double*, R*, double*, hipStream_t);
DDC_INST(float)
DDC_INST(double)
#undef DDC_INST

}  // namespace ddc
