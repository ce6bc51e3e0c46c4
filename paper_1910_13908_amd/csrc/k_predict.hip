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

template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    const double* __restrict__ freq, const double* __restrict__ sl, const double* __restrict__ sm,
    const double* __restrict__ sI, const double* __restrict__ sQ, const double* __restrict__ sU,
    const double* __restrict__ sV, const int32_t* __restrict__ offs, int64_t B, int F,
    int64_t plane, R* __restrict__ coh) {
  __shared__ double s_l[kThreads], s_m[kThreads], s_n[kThreads];
  __shared__ double s_I[kThreads], s_Q[kThreads], s_U[kThreads], s_V[kThreads];

  const int tid = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kThreads + tid;
  const int tf = blockIdx.y;
  const int t = tf / F, f = tf % F;
  const int k = blockIdx.z;
  const int s0 = offs[k], s1 = offs[k + 1];

  const double scale = freq[f] / kCLight;
  double uu = 0.0, vv = 0.0, ww = 0.0;
  if (b < B) {
    const int64_t i = (int64_t)t * B + b;
    uu = u[i] * scale;
    vv = v[i] * scale;
    ww = w[i] * scale;
  }
  // accumulators: sum I e, sum Q e, sum U e, sum V e with e = exp(-2 pi i phi)
  R iR = 0, iI = 0, qR = 0, qI = 0, uR = 0, uI = 0, vR = 0, vI = 0;

  for (int c0 = s0; c0 < s1; c0 += kThreads) {
    const int n = min(kThreads, s1 - c0);
    __syncthreads();
    int pol = 0;
    if (tid < n) {
      const double l = sl[c0 + tid], m = sm[c0 + tid];
      const double r2 = l * l + m * m;
      s_l[tid] = l;
      s_m[tid] = m;
      s_n[tid] = -r2 / (1.0 + sqrt(1.0 - r2));       // n - 1 without cancellation
      s_I[tid] = sI[c0 + tid];
      const double q = sQ[c0 + tid], uu_ = sU[c0 + tid], vv_ = sV[c0 + tid];
      s_Q[tid] = q;
      s_U[tid] = uu_;
      s_V[tid] = vv_;
      pol = (q != 0.0) | (uu_ != 0.0) | (vv_ != 0.0);
    }
    pol = __syncthreads_or(pol);
    if (b < B) {
      if (!pol) {
        for (int j = 0; j < n; ++j) {
          const double ph = fma(uu, s_l[j], fma(vv, s_m[j], ww * s_n[j]));
          const double fr = ph - rint(ph);
          R sn, cs;
          sincos_turns(fr, sn, cs);
          const R I = (R)s_I[j];
          iR = fma(I, cs, iR);
          iI = fma(-I, sn, iI);
        }
      } else {
        for (int j = 0; j < n; ++j) {
          const double ph = fma(uu, s_l[j], fma(vv, s_m[j], ww * s_n[j]));
          const double fr = ph - rint(ph);
          R sn, cs;
          sincos_turns(fr, sn, cs);
          const R I = (R)s_I[j], Q = (R)s_Q[j], U = (R)s_U[j], V = (R)s_V[j];
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
  if (b < B) {
    // XX = SI + SQ, XY = SU + i SV, YX = SU - i SV, YY = SI - SQ
    R* out = coh + (int64_t)k * 8 * plane + (int64_t)tf * B + b;
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

}  // namespace

template <typename R>
hipError_t launch_predict(const ObsDev& o, int K, const int32_t* offs_dev, const int32_t*,
                          const double* l, const double* m, const double* I, const double* Q,
                          const double* U, const double* V, R* coh, hipStream_t st) {
  const int64_t plane = (int64_t)o.T * o.F * o.B;
  dim3 grid((unsigned)((o.B + kThreads - 1) / kThreads), (unsigned)(o.T * o.F), (unsigned)K);
  hipLaunchKernelGGL(k_predict<R>, grid, dim3(kThreads), 0, st, o.u, o.v, o.w, o.freq, l, m, I, Q,
                     U, V, offs_dev, o.B, o.F, plane, coh);
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

}  // namespace ddc
