// Model-coherency predict (measurement equation; paper Section 2 groups sources into
// clusters, Section 3 fixes the N(N-1)/2 baselines):
//
//   C_k(b, t, f) = sum_{s in k} B_s exp(-2 pi i phi),  phi = (u l_s + v m_s + w (n_s - 1)) f / c
//   B_s = [[I+Q, U+iV], [U-iV, I-Q]]
//
// One thread owns one baseline at one (timeslot, channel) of one cluster; the cluster's
// sources are staged through LDS in chunks shared by the 256 threads of a workgroup, so the
// inner loop reads only LDS broadcasts and registers.  The phase argument is always FP64
// (it reaches thousands of turns on long baselines); it is reduced to its fractional part,
// [0, 1) turns, in FP64 before the trigonometry.  The FP32 path then takes the hardware sin/cos, whose
// input is in turns; the FP64 path uses sincospi.  Clusters whose chunk has Q = U = V = 0
// take the Stokes-I-only inner loop (two FMAs per term instead of eight).
#include "common.h"

#include <algorithm>

// Evaluated exactly as written: no multiply-add contraction beyond the explicit fma() calls
// (the phase argument is the FP64 path whose rounding the reference arithmetic fixes).
#pragma clang fp contract(off)

namespace ddc {
namespace {

constexpr int kThreads = 256;

// Range reduction of the phase (in turns) in FP64: its fractional part, in [0, 1), with the
// hardware fract (one instruction); sin and cos have period one turn.
__device__ __forceinline__ double turns_fraction(double ph) {
  return __builtin_amdgcn_fract(ph);
}

__device__ __forceinline__ void sincos_turns(double frac, float& s, float& c) {
  const float x = (float)frac;                // 0 <= x <= 1 turn
  s = __builtin_amdgcn_sinf(x);               // sin(2 pi x)
  c = __builtin_amdgcn_cosf(x);
}

__device__ __forceinline__ void sincos_turns(double frac, double& s, double& c) {
  sincospi(2.0 * frac, &s, &c);
}

// Sources of the chunk being summed: positions in FP64 (they enter the FP64 phase), fluxes
// in the accumulation type.  What the Stokes-I loop reads of one source (l, m, n - 1, I)
// sits in one 32-byte record, so an unrolled group of sources is read with 16-byte LDS loads
// at immediate offsets from one address.
template <typename R>
struct alignas(16) SrcTerm {
  double l, m, n;
  R I;
};

template <typename R>
struct PredictShared {
  SrcTerm<R> src[kThreads];
  R Q[kThreads], U[kThreads], V[kThreads];
};

// One 256-baseline tile at one (timeslot, channel), every cluster in turn: the tile's uvw are
// read once and kept in registers for all clusters.
template <typename R>
__device__ __forceinline__ void predict_tile(const PredictJob& j, int64_t btile, int tf,
                                             PredictShared<R>& sh) {
  const int tid = threadIdx.x;
  const int64_t b = btile * kThreads + tid;
  const int t = tf / j.F, f = tf % j.F;

  const double scale = j.freq[f] / kCLight;
  double uu = 0.0, vv = 0.0, ww = 0.0;
  if (b < j.B) {
    const int64_t i = (int64_t)t * j.B + b;
    uu = j.u[i] * scale;
    vv = j.v[i] * scale;
    ww = j.w[i] * scale;
  }
  for (int k = 0; k < j.K; ++k) {
    const int s0 = j.offs[k], s1 = j.offs[k + 1];
    // accumulators: sum I e, sum Q e, sum U e, sum V e with e = exp(-2 pi i phi)
    R iR = 0, iI = 0, qR = 0, qI = 0, uR = 0, uI = 0, vR = 0, vI = 0;
    for (int c0 = s0; c0 < s1; c0 += kThreads) {
      const int n = min(kThreads, s1 - c0);
      __syncthreads();
      int pol = 0;
      if (tid < n) {
        const double l = j.l[c0 + tid], m = j.m[c0 + tid];
        const double r2 = l * l + m * m;
        SrcTerm<R> st;
        st.l = l;
        st.m = m;
        st.n = -r2 / (1.0 + sqrt(1.0 - r2));       // n - 1 without cancellation
        st.I = (R)j.I[c0 + tid];
        sh.src[tid] = st;
        const double q = j.Q[c0 + tid], uu_ = j.U[c0 + tid], vv_ = j.V[c0 + tid];
        sh.Q[tid] = (R)q;
        sh.U[tid] = (R)uu_;
        sh.V[tid] = (R)vv_;
        pol = (q != 0.0) | (uu_ != 0.0) | (vv_ != 0.0);
      }
      pol = __syncthreads_or(pol);
      if (b < j.B) {
        if (!pol) {
#pragma unroll 4
          for (int s = 0; s < n; ++s) {
            const SrcTerm<R> st = sh.src[s];
            const double ph = fma(uu, st.l, fma(vv, st.m, ww * st.n));
            const double fr = turns_fraction(ph);
            R sn, cs;
            sincos_turns(fr, sn, cs);
            iR = fma(st.I, cs, iR);
            iI = fma(-st.I, sn, iI);
          }
        } else {
#pragma unroll 4
          for (int s = 0; s < n; ++s) {
            const SrcTerm<R> st = sh.src[s];
            const double ph = fma(uu, st.l, fma(vv, st.m, ww * st.n));
            const double fr = turns_fraction(ph);
            R sn, cs;
            sincos_turns(fr, sn, cs);
            const R I = st.I, Q = sh.Q[s], U = sh.U[s], V = sh.V[s];
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
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict(PredictJob j) {
  __shared__ PredictShared<R> sh;
  predict_tile<R>(j, blockIdx.x, blockIdx.y, sh);
}

// Persistent batched predict over several solves: the workgroups walk the flattened list of
// (job, timeslot-channel, baseline tile) items with a grid stride.  Each item runs
// exactly the per-thread arithmetic of k_predict, so a solve predicted in a batch is bitwise
// identical to the same solve predicted alone.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict_batch(const PredictJob* __restrict__ jobs,
                                                           int njobs, int64_t total) {
  __shared__ PredictShared<R> sh;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    int jj = 0;
    while (jj + 1 < njobs && jobs[jj + 1].first_block <= vb) ++jj;
    const PredictJob& j = jobs[jj];
    const int64_t local = vb - j.first_block;
    const int64_t nbt = (j.B + kThreads - 1) / kThreads;
    const int TF = j.T * j.F;
    const int64_t btile = local % nbt;
    const int64_t rest = local / nbt;
    (void)TF;
    predict_tile<R>(j, btile, (int)rest, sh);
    __syncthreads();
  }
}

}  // namespace

template <typename R>
hipError_t launch_predict(const ObsDev& o, int K, const int32_t* offs_dev, const int32_t*,
                          const double* l, const double* m, const double* I, const double* Q,
                          const double* U, const double* V, R* coh, hipStream_t st) {
  PredictJob j = make_predict_job(o, K, offs_dev, l, m, I, Q, U, V, coh);
  dim3 grid((unsigned)((o.B + kThreads - 1) / kThreads), (unsigned)(o.T * o.F));
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
