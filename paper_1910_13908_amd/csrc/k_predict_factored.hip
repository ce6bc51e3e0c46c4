// Model-coherency predict with station-factorised phasors (same quantity and layout as the
// direct predict; measurement equation, paper Section 2 clusters, Section 3 baselines).
//
// With the baseline coordinates the difference of two stations' coordinates, the phase of a
// baseline splits:  phi_pq = phi_p - phi_q,  phi_p = (u_p l + v_p m + w_p (n-1)) f / c, so
//
//   exp(-2 pi i phi_pq) = E_p conj(E_q),   E_p = exp(-2 pi i phi_p),
//   C_k(p, q) = sum_{s in k} B_s E_p,s conj(E_q,s).
//
// Two kernels.  k_phasors evaluates E for every (timeslot-channel, source, station): FP64
// phase reduced to [-1/2, 1/2) turns, then FP32 hardware sin/cos (mixed) or FP64 sincospi;
// N*S*T*F phasors instead of B*S*T*F terms.  k_predict_factored then forms, for one cluster
// and one timeslot-channel, a 64 x 64 block of station pairs (p block <= q block) as a rank-S
// Hermitian product: sources are staged through LDS in chunks (p-side phasors already
// multiplied by the correlation's brightness weight), and each of the 256 threads keeps a
// 4 x 4 block of pairs in registers.  The correlations are
//   XX: (I+Q),  XY: (U+iV),  YX: (U-iV),  YY: (I-Q)   times E_p conj(E_q),
// one pass each; a cluster whose Q, U, V are all zero needs only the XX pass (YY = XX,
// XY = YX = 0).  The work is bound by its VALU arithmetic and the coherency writes, not by
// transcendentals.
#include "common.h"

#include <algorithm>

namespace ddc {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 32;        // sources staged per pass through LDS

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
  using T = float2;
};
template <>
struct Cplx<double> {
  using T = double2;
};

__device__ __forceinline__ void sincos_turns_f(double frac, float& s, float& c) {
  const float x = (float)frac;               // |x| <= 1/2 turn
  s = __builtin_amdgcn_sinf(x);              // sin(2 pi x)
  c = __builtin_amdgcn_cosf(x);
}
__device__ __forceinline__ void sincos_turns_f(double frac, double& s, double& c) {
  sincospi(2.0 * frac, &s, &c);
}

// E[(tf * S + s) * Np + p] = exp(-2 pi i phi_p,s(t, f)) for p < N; zero for N <= p < Np.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_phasors(const double* __restrict__ su,
                                                      const double* __restrict__ sv,
                                                      const double* __restrict__ sw,
                                                      const double* __restrict__ freq,
                                                      const double* __restrict__ l,
                                                      const double* __restrict__ m, int N,
                                                      int Np, int S, int T, int F,
                                                      typename Cplx<R>::T* __restrict__ E) {
  using C2 = typename Cplx<R>::T;
  const int64_t total = (int64_t)T * F * S * Np;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const int p = (int)(i % Np);
    const int64_t r = i / Np;
    const int s = (int)(r % S);
    const int tf = (int)(r / S);
    C2 e;
    e.x = (R)0;
    e.y = (R)0;
    if (p < N) {
      const int t = tf / F, f = tf % F;
      const double scale = freq[f] / kCLight;
      const double ls = l[s], ms = m[s];
      const double r2 = ls * ls + ms * ms;
      const double n1 = -r2 / (1.0 + sqrt(1.0 - r2));      // n - 1 without cancellation
      const int64_t st = (int64_t)t * N + p;
      const double ph = fma(su[st] * scale, ls, fma(sv[st] * scale, ms, sw[st] * scale * n1));
      R sn, cs;
      sincos_turns_f(ph - rint(ph), sn, cs);
      e.x = cs;
      e.y = -sn;
    }
    E[i] = e;
  }
}

// Four consecutive elements with only element alignment (the store address is a baseline
// index, 4-byte aligned for float).
template <typename R>
using V4 = R __attribute__((ext_vector_type(4), aligned(sizeof(R))));
template <typename R>
__device__ __forceinline__ void store4(R* p, const V4<R>& v) {
  *reinterpret_cast<V4<R>*>(p) = v;
}

struct FactoredJob {
  const void* E;                    // [T*F][S][Np] complex phasors
  const double *I, *Q, *U, *V;
  const int32_t* offs;              // device [K+1]
  void* coh;                        // [K][8][T*F][B]
  int64_t B, plane;                 // plane = T*F*B
  int N, Np, S, TF, nb, npairs;
};

// Brightness weight of correlation c for source s: XX I+Q, XY U+iV, YX U-iV, YY I-Q.
template <typename R>
__device__ __forceinline__ void corr_weight(const FactoredJob& j, int s, int c, R& wr, R& wi) {
  const double I = j.I[s], Q = j.Q[s], U = j.U[s], V = j.V[s];
  switch (c) {
    case 0: wr = (R)(I + Q); wi = (R)0; break;
    case 1: wr = (R)U; wi = (R)V; break;
    case 2: wr = (R)U; wi = (R)(-V); break;
    default: wr = (R)(I - Q); wi = (R)0; break;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict_factored(FactoredJob j) {
  using C2 = typename Cplx<R>::T;
  __shared__ C2 sp[kChunk][64];     // weighted p-side phasors of the chunk
  __shared__ C2 sq[kChunk][64];     // q-side phasors of the chunk
  __shared__ R swr[kChunk], swi[kChunk];   // the chunk's brightness weights for this pass
  const C2* __restrict__ E = reinterpret_cast<const C2*>(j.E);
  const int k = blockIdx.y;
  const int pair = (int)(blockIdx.x % j.npairs);
  const int tf = (int)(blockIdx.x / j.npairs);
  // pair -> (pb, qb), pb <= qb, row by row over the upper triangle of station blocks
  int pb = 0, rem = pair;
  while (rem >= j.nb - pb) {
    rem -= j.nb - pb;
    ++pb;
  }
  const int qb = pb + rem;
  const int tid = threadIdx.x, pg = tid >> 4, qg = tid & 15;
  const int s0 = j.offs[k], s1 = j.offs[k + 1];

  // polarised cluster? (uniform decision for the workgroup)
  int pol = 0;
  for (int s = s0 + tid; s < s1; s += kThreads)
    pol |= (j.Q[s] != 0.0) | (j.U[s] != 0.0) | (j.V[s] != 0.0);
  pol = __syncthreads_or(pol);

  R* out = reinterpret_cast<R*>(j.coh) + (int64_t)k * 8 * j.plane + (int64_t)tf * j.B;
  const C2* Etf = E + (int64_t)tf * j.S * j.Np;
  R ar[4][4], ai[4][4];

  // One pass: ar + i ai = sum_s w_c,s E_p,s conj(E_q,s) over the cluster's sources.
  auto pass = [&](int c) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        ar[a][b] = (R)0;
        ai[a][b] = (R)0;
      }
    for (int c0 = s0; c0 < s1; c0 += kChunk) {
      const int n = min(kChunk, s1 - c0);
      __syncthreads();
      if (tid < kChunk) {
        R wr = (R)0, wi = (R)0;
        if (tid < n) corr_weight<R>(j, c0 + tid, c, wr, wi);
        swr[tid] = wr;
        swi[tid] = wi;
      }
      __syncthreads();
      for (int e = tid; e < kChunk * 64; e += kThreads) {
        const int sl = e >> 6, pl = e & 63;
        C2 xp, xq;
        xp.x = xp.y = xq.x = xq.y = (R)0;
        if (sl < n) {
          const C2* row = Etf + (int64_t)(c0 + sl) * j.Np;
          const C2 ep = row[64 * pb + pl];
          xq = row[64 * qb + pl];
          const R wr = swr[sl], wi = swi[sl];
          xp.x = wr * ep.x - wi * ep.y;
          xp.y = wr * ep.y + wi * ep.x;
        }
        sp[sl][pl] = xp;
        sq[sl][pl] = xq;
      }
      __syncthreads();
      for (int s = 0; s < n; ++s) {
        C2 a[4], e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = sp[s][4 * pg + u];
          e[u] = sq[s][4 * qg + u];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            // (a) conj(e)
            ar[x][y] = fma(a[x].x, e[y].x, fma(a[x].y, e[y].y, ar[x][y]));
            ai[x][y] = fma(a[x].y, e[y].x, fma(-a[x].x, e[y].y, ai[x][y]));
          }
      }
    }
  };

  // Stores of the pairs p < q < N into the planes listed (re, im) with their values.  A
  // thread's four pairs of one row are four consecutive baselines: one 16-byte store per
  // plane when all four exist (baseline indices are only element-aligned, which global
  // vector stores accept), element stores on the diagonal block and the ragged edge.  The
  // stores sit outside any loop so that their addresses are not hoisted across the sources.
  auto store_rows = [&](int plane_re, int plane_im, bool stokes_i) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int p = 64 * pb + 4 * pg + x;
      if (p >= j.N) continue;
      const int64_t base = (int64_t)p * (2 * j.N - p - 1) / 2 - p - 1;
      const int q0 = 64 * qb + 4 * qg;
      R* o0 = out + base + q0;
      if (q0 > p && q0 + 3 < j.N) {
        const V4<R> re = {ar[x][0], ar[x][1], ar[x][2], ar[x][3]};
        const V4<R> im = {ai[x][0], ai[x][1], ai[x][2], ai[x][3]};
        store4<R>(o0 + plane_re * j.plane, re);
        store4<R>(o0 + plane_im * j.plane, im);
        if (stokes_i) {
          const V4<R> z = {(R)0, (R)0, (R)0, (R)0};
          store4<R>(o0 + 2 * j.plane, z);
          store4<R>(o0 + 3 * j.plane, z);
          store4<R>(o0 + 4 * j.plane, z);
          store4<R>(o0 + 5 * j.plane, z);
          store4<R>(o0 + 6 * j.plane, re);
          store4<R>(o0 + 7 * j.plane, im);
        }
        continue;
      }
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int q = q0 + y;
        if (q <= p || q >= j.N) continue;
        R* o = out + base + q;
        o[plane_re * j.plane] = ar[x][y];
        o[plane_im * j.plane] = ai[x][y];
        if (stokes_i) {
          o[2 * j.plane] = (R)0;
          o[3 * j.plane] = (R)0;
          o[4 * j.plane] = (R)0;
          o[5 * j.plane] = (R)0;
          o[6 * j.plane] = ar[x][y];
          o[7 * j.plane] = ai[x][y];
        }
      }
    }
  };

  if (!pol) {
    pass(0);                        // XX; YY = XX, XY = YX = 0
    store_rows(0, 1, true);
  } else {
    for (int c = 0; c < 4; ++c) {   // XX, XY, YX, YY
      pass(c);
      store_rows(2 * c, 2 * c + 1, false);
    }
  }
}

}  // namespace

size_t phasor_bytes(int N, int S, int T, int F, size_t es) {
  const int Np = (N + 63) / 64 * 64;
  return (size_t)T * F * S * Np * 2 * es;
}

template <typename R>
hipError_t launch_predict_factored(const ObsDev& o, const double* su, const double* sv,
                                   const double* sw, int K, int S, const int32_t* offs_dev,
                                   const double* l, const double* m, const double* I,
                                   const double* Q, const double* U, const double* V,
                                   void* phasors, R* coh, hipStream_t st) {
  using C2 = typename Cplx<R>::T;
  const int Np = (o.N + 63) / 64 * 64;
  const int TF = o.T * o.F;
  if (S > 0) {
    const int64_t total = (int64_t)TF * S * Np;
    const int64_t blocks = std::min<int64_t>((total + kThreads - 1) / kThreads, 65536);
    hipLaunchKernelGGL(k_phasors<R>, dim3((unsigned)blocks), dim3(kThreads), 0, st, su, sv, sw,
                       o.freq, l, m, o.N, Np, S, o.T, o.F, reinterpret_cast<C2*>(phasors));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  FactoredJob j;
  j.E = phasors;
  j.I = I; j.Q = Q; j.U = U; j.V = V;
  j.offs = offs_dev;
  j.coh = coh;
  j.B = o.B;
  j.plane = (int64_t)TF * o.B;
  j.N = o.N;
  j.Np = Np;
  j.S = S;
  j.TF = TF;
  j.nb = Np / 64;
  j.npairs = j.nb * (j.nb + 1) / 2;
  const int64_t gx = (int64_t)j.npairs * TF;
  if (gx > 0x7fffffff || K > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_predict_factored<R>, dim3((unsigned)gx, (unsigned)K), dim3(kThreads), 0, st,
                     j);
  return hipGetLastError();
}

template hipError_t launch_predict_factored<float>(const ObsDev&, const double*, const double*,
                                                   const double*, int, int, const int32_t*,
                                                   const double*, const double*, const double*,
                                                   const double*, const double*, const double*,
                                                   void*, float*, hipStream_t);
template hipError_t launch_predict_factored<double>(const ObsDev&, const double*, const double*,
                                                    const double*, int, int, const int32_t*,
                                                    const double*, const double*, const double*,
                                                    const double*, const double*, const double*,
                                                    void*, double*, hipStream_t);

}  // namespace ddc
