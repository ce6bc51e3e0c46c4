// Model-coherency predict (measurement equation; paper Section 2 groups sources into
// clusters, Section 3 fixes the N(N-1)/2 baselines):
//
//   C_k(b, t, f) = sum_{s in k} B_s exp(-2 pi i phi),  phi = (u l_s + v m_s + w (n_s - 1)) f / c
//   B_s = [[I+Q, U+iV], [U-iV, I-Q]]
//
// One thread owns one baseline at one (timeslot, channel) of one cluster; the cluster's
// sources are staged through LDS in chunks shared by the 256 threads of a workgroup, so the
// inner loop reads only LDS broadcasts and registers.  The phase argument is always FP64
// (it reaches thousands of turns on long baselines); it is reduced to [-1/2, 1/2) turns in
// FP64 before the trigonometry.  The FP32 path then takes the hardware sin/cos, whose
// input is in turns; the FP64 path uses sincospi.  Clusters whose chunk has Q = U = V = 0
// take the Stokes-I-only inner loop (two FMAs per term instead of eight).
#include "common.h"

#include <algorithm>

namespace ddc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void sincos_turns(double frac, float& s, float& c) {
  const float x = (float)frac;                // |x| <= 1/2 turn
  s = __builtin_amdgcn_sinf(x);               // sin(2 pi x)
  c = __builtin_amdgcn_cosf(x);
}

__device__ __forceinline__ void sincos_turns(double frac, double& s, double& c) {
  sincospi(2.0 * frac, &s, &c);
}

struct PredictShared {
  double l[kThreads], m[kThreads], n[kThreads];
  double I[kThreads], Q[kThreads], U[kThreads], V[kThreads];
};

// One 256-baseline tile at one (timeslot, channel) of one cluster.
template <typename R>
__device__ __forceinline__ void predict_tile(const PredictJob& j, int64_t btile, int tf, int k,
                                             PredictShared& sh) {
  const int tid = threadIdx.x;
  const int64_t b = btile * kThreads + tid;
  const int t = tf / j.F, f = tf % j.F;
  const int s0 = j.offs[k], s1 = j.offs[k + 1];

  const double scale = j.freq[f] / kCLight;
  double uu = 0.0, vv = 0.0, ww = 0.0;
  if (b < j.B) {
    const int64_t i = (int64_t)t * j.B + b;
    uu = j.u[i] * scale;
    vv = j.v[i] * scale;
    ww = j.w[i] * scale;
  }
  // accumulators: sum I e, sum Q e, sum U e, sum V e with e = exp(-2 pi i phi)
  R iR = 0, iI = 0, qR = 0, qI = 0, uR = 0, uI = 0, vR = 0, vI = 0;

  for (int c0 = s0; c0 < s1; c0 += kThreads) {
    const int n = min(kThreads, s1 - c0);
    __syncthreads();
    int pol = 0;
    if (tid < n) {
      const double l = j.l[c0 + tid], m = j.m[c0 + tid];
      const double r2 = l * l + m * m;
      sh.l[tid] = l;
      sh.m[tid] = m;
      sh.n[tid] = -r2 / (1.0 + sqrt(1.0 - r2));       // n - 1 without cancellation
      sh.I[tid] = j.I[c0 + tid];
      const double q = j.Q[c0 + tid], uu_ = j.U[c0 + tid], vv_ = j.V[c0 + tid];
      sh.Q[tid] = q;
      sh.U[tid] = uu_;
      sh.V[tid] = vv_;
      pol = (q != 0.0) | (uu_ != 0.0) | (vv_ != 0.0);
    }
    pol = __syncthreads_or(pol);
    if (b < j.B) {
      if (!pol) {
        for (int s = 0; s < n; ++s) {
          const double ph = fma(uu, sh.l[s], fma(vv, sh.m[s], ww * sh.n[s]));
          const double fr = ph - rint(ph);
          R sn, cs;
          sincos_turns(fr, sn, cs);
          const R I = (R)sh.I[s];
          iR = fma(I, cs, iR);
          iI = fma(-I, sn, iI);
        }
      } else {
        for (int s = 0; s < n; ++s) {
          const double ph = fma(uu, sh.l[s], fma(vv, sh.m[s], ww * sh.n[s]));
          const double fr = ph - rint(ph);
          R sn, cs;
          sincos_turns(fr, sn, cs);
          const R I = (R)sh.I[s], Q = (R)sh.Q[s], U = (R)sh.U[s], V = (R)sh.V[s];
          iR = fma(I, cs, iR);
          iI = fma(-I, sn, iI);
          qR = fma(Q, cs, qR);
          qI = fma(-Q, sn, qI);
          uR = fma(U, cs, uR);
          uI = fma(-U, sn, uI);
          vR = fma(V, cs, vR);
          vI = fma(-V, sn, vI);
        }
      }
    }
  }
  if (b < j.B) {
    // XX = SI + SQ, XY = SU + i SV, YX = SU - i SV, YY = SI - SQ
    const int64_t plane = j.plane;
    R* out = reinterpret_cast<R*>(j.coh) + (int64_t)k * 8 * plane + (int64_t)tf * j.B + b;
    out[0 * plane] = iR + qR;
    out[1 * plane] = iI + qI;
    out[2 * plane] = uR - vI;
    out[3 * plane] = uI + vR;
    out[4 * plane] = uR + vI;
    out[5 * plane] = uI - vR;
    out[6 * plane] = iR - qR;
    out[7 * plane] = iI - qI;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict(PredictJob j) {
  __shared__ PredictShared sh;
  predict_tile<R>(j, blockIdx.x, blockIdx.y, blockIdx.z, sh);
}

// Persistent batched predict over several solves: the workgroups walk the flattened list of
// (job, cluster, timeslot-channel, baseline tile) items with a grid stride.  Each item runs
// exactly the per-thread arithmetic of k_predict, so a solve predicted in a batch is bitwise
// identical to the same solve predicted alone.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict_batch(const PredictJob* __restrict__ jobs,
                                                           int njobs, int64_t total) {
  __shared__ PredictShared sh;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    int jj = 0;
    while (jj + 1 < njobs && jobs[jj + 1].first_block <= vb) ++jj;
    const PredictJob& j = jobs[jj];
    const int64_t local = vb - j.first_block;
    const int64_t nbt = (j.B + kThreads - 1) / kThreads;
    const int TF = j.T * j.F;
    const int64_t btile = local % nbt;
    const int64_t rest = local / nbt;
    predict_tile<R>(j, btile, (int)(rest % TF), (int)(rest / TF), sh);
    __syncthreads();
  }
}

}  // namespace

template <typename R>
hipError_t launch_predict(const ObsDev& o, int K, const int32_t* offs_dev, const int32_t*,
                          const double* l, const double* m, const double* I, const double* Q,
                          const double* U, const double* V, R* coh, hipStream_t st) {
  PredictJob j = make_predict_job(o, K, offs_dev, l, m, I, Q, U, V, coh);
  dim3 grid((unsigned)((o.B + kThreads - 1) / kThreads), (unsigned)(o.T * o.F), (unsigned)K);
  hipLaunchKernelGGL(k_predict<R>, grid, dim3(kThreads), 0, st, j);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_predict_batch(const PredictJob* jobs_dev, int njobs, int64_t total_blocks,
                                int grid, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  const int g = (int)std::min<int64_t>(total_blocks, (int64_t)grid);
  hipLaunchKernelGGL(k_predict_batch<R>, dim3(g), dim3(kThreads), 0, st, jobs_dev, njobs, total_blocks);
  return hipGetLastError();
}

template hipError_t launch_predict<float>(const ObsDev&, int, const int32_t*, const int32_t*,
                                          const double*, const double*, const double*,
                                          const double*, const double*, const double*, float*,
                                          hipStream_t);
template hipError_t launch_predict<double>(const ObsDev&, int, const int32_t*, const int32_t*,
                                           const double*, const double*, const double*,
                                           const double*, const double*, const double*, double*,
                                           hipStream_t);
template hipError_t launch_predict_batch<float>(const PredictJob*, int, int64_t, int, hipStream_t);
template hipError_t launch_predict_batch<double>(const PredictJob*, int, int64_t, int, hipStream_t);

}  // namespace ddc
