// Dense damped Cholesky of the 8N x 8N normal matrix and the triangular solves of the LM step.
//
// The matrix is symmetric positive definite after damping (H + mu I, mu > 0).  It is
// factored as L L^T in 64 x 64 tiles by ONE persistent kernel: workgroups take tiles of the
// lower triangle from an atomic ticket in column-major tile order, and each tile is owned by
// one workgroup from its first update to its final value (left-looking):
//
//   A_IJ <- H_IJ + mu [I==J] - sum_{K<J} L_IK L_JK^T      (MFMA, operands staged in LDS)
//   I == J:  L_JJ = chol(A_JJ), and its inverse;          (one wave, registers + LDS)
//   I >  J:  L_IJ = A_IJ L_JJ^{-T}                        (MFMA with the stored inverse)
//
// A tile publishes a ready flag when it is final; a consumer waits only on flags of tiles
// with a smaller ticket.  Tickets are claimed only by running workgroups, so the smallest
// unfinished ticket never waits on unfinished work and the schedule cannot deadlock without
// any co-residency guarantee.  Every wait is bounded; on expiry the kernel raises an abort
// flag, every other wait returns at once, and the status word reports DDC_ETIMEOUT.  The
// last workgroup to leave resets the tickets and flags, so the kernel needs no host-side
// clearing between launches.
//
// The factor is stored tile-packed (column-major over the tiles of the lower triangle,
// row-major inside a tile) next to the inverses of the diagonal tiles, which the
// triangular solves use as small dense products.  Forward and backward substitution follow
// the same ticket-and-flag scheme over 64-row blocks.  In mixed precision the factor and
// the products run in FP32 (FP32 MFMA); right-hand sides, solutions and the refinement
// residual g - (H + mu I) d are FP64.
#include "common.h"

namespace ddc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kSpinLimit = 1u << 22;   // polls (with s_sleep) before a wait gives up

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R>
struct Mfma;

// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16]; result element
// v of lane l is D[4(l/16)+v][l%16].
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  static constexpr int STR = 68;   // LDS row stride (elements): 16-byte aligned, spreads banks
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// v_mfma_f64_16x16x4f64: same operand layout; result element v of lane l is D[l/16+4v][l%16].
template <>
struct Mfma<double> {
  using acc_t = f64x4;
  static constexpr int STR = 66;
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Result-element coordinates inside a 16x16 block: v_mfma_f32_16x16x4f32 puts element v of
// lane l at row 4(l/16)+v, v_mfma_f64_16x16x4f64 at row l/16 + 4v; both at column l%16.
template <typename R>
__device__ __forceinline__ int out_row(int lane, int v) {
  return sizeof(R) == 4 ? 4 * (lane >> 4) + v : (lane >> 4) + 4 * v;
}
__device__ __forceinline__ int out_col(int lane, int) { return lane & 15; }

__device__ __forceinline__ uint32_t tile_index(int I, int J, int T) {
  // column-major over the lower triangle: column J starts at J*T - J(J-1)/2
  return (uint32_t)(J * T - (J * (J - 1)) / 2 + (I - J));
}

__device__ __forceinline__ void decode_ticket(uint32_t t, int T, int& I, int& J) {
  int j = 0;
  uint32_t start = 0;
  while (start + (uint32_t)(T - j) <= t) {
    start += (uint32_t)(T - j);
    ++j;
  }
  J = j;
  I = j + (int)(t - start);
}

// Wait until *flag != 0 (thread 0 polls; the workgroup then acquires).  Returns false on
// abort or timeout.
__device__ bool wait_flag(const uint32_t* flag, SyncArea* sync, int32_t* status) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    uint32_t spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if (++spins > kSpinLimit) {
        __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (status) atomicOr(status, 2);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ void publish(uint32_t* flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Leave the persistent loop; the last workgroup out clears the flags and the counters.
__device__ void exit_and_reset(SyncArea* sync, uint32_t* flags, int nflags) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&sync->exited, 1u) == gridDim.x - 1);
  __syncthreads();
  if (s_last) {
    __threadfence();
    for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0u;
    if (threadIdx.x == 0) {
      sync->ticket = 0u;
      sync->exited = 0u;
      sync->abort = 0u;
    }
    __threadfence();
  }
}

__device__ __forceinline__ uint32_t claim(SyncArea* sync) {
  __shared__ uint32_t s_t;
  if (threadIdx.x == 0) s_t = atomicAdd(&sync->ticket, 1u);
  __syncthreads();
  const uint32_t t = s_t;
  __syncthreads();
  return t;
}

// Copy one packed 64x64 row-major tile from global memory into LDS (row stride STR).
template <typename R>
__device__ __forceinline__ void tile_to_lds(const R* __restrict__ src, R* dst) {
  constexpr int STR = Mfma<R>::STR;
  if constexpr (sizeof(R) == 4) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * kThreads;       // 1024 float4
      const int r = idx >> 4, c = (idx & 15) * 4;
      *reinterpret_cast<float4*>(dst + r * STR + c) = s4[idx];
    }
  } else {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = threadIdx.x + it * kThreads;       // 2048 double2
      const int r = idx >> 5, c = (idx & 31) * 2;
      *reinterpret_cast<double2*>(dst + r * STR + c) = s2[idx];
    }
  }
}

// acc[r][c] += sgn * sum_k A[r][k] * B[c][k] over this wave's 32x32 quadrant; A and B are
// row-major LDS tiles.  The K index is split so that lane group g = l/16 walks k = 16g + s,
// s = 0..15, which makes each lane's operands 16 consecutive LDS elements.
template <typename R, bool NEG>
__device__ __forceinline__ void tile_mma(typename Mfma<R>::acc_t (&acc)[2][2], const R* A,
                                         const R* B, int qr, int qc) {
  constexpr int STR = Mfma<R>::STR;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, rr = lane & 15;
  const R* a0 = A + (qr * 32 + rr) * STR + 16 * g;
  const R* a1 = a0 + 16 * STR;
  const R* b0 = B + (qc * 32 + rr) * STR + 16 * g;
  const R* b1 = b0 + 16 * STR;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const R x0 = NEG ? -a0[s] : a0[s];
    const R x1 = NEG ? -a1[s] : a1[s];
    const R y0 = b0[s], y1 = b1[s];
    acc[0][0] = Mfma<R>::mma(x0, y0, acc[0][0]);
    acc[0][1] = Mfma<R>::mma(x0, y1, acc[0][1]);
    acc[1][0] = Mfma<R>::mma(x1, y0, acc[1][0]);
    acc[1][1] = Mfma<R>::mma(x1, y1, acc[1][1]);
  }
}

template <typename R>
__device__ __forceinline__ void acc_to_lds(const typename Mfma<R>::acc_t (&acc)[2][2], R* dst,
                                           int qr, int qc) {
  constexpr int STR = Mfma<R>::STR;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = qr * 32 + bi * 16 + out_row<R>(lane, v);
        const int c = qc * 32 + bj * 16 + out_col(lane, v);
        dst[r * STR + c] = acc[bi][bj][v];
      }
}

template <typename R>
__device__ __forceinline__ void acc_to_global(const typename Mfma<R>::acc_t (&acc)[2][2],
                                              R* __restrict__ dst, int qr, int qc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = qr * 32 + bi * 16 + out_row<R>(lane, v);
        const int c = qc * 32 + bj * 16 + out_col(lane, v);
        dst[r * 64 + c] = acc[bi][bj][v];
      }
}

// Cholesky of the lower triangle of a 64x64 LDS tile in place (wave 0; lane i owns row i).
// Crout order: column j needs row j of L (k < j) from LDS and the lane's own row from
// registers.  Returns nonzero in lane 0 if a pivot was not positive (it is then set to 1 so
// that the factorisation still finishes with finite values).
template <typename R>
__device__ int potrf_wave(R* A) {
  constexpr int STR = Mfma<R>::STR;
  const int i = threadIdx.x & 63;
  R a[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) a[k] = A[i * STR + k];
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    R dot = 0;
    const R* rowj = A + j * STR;
#pragma unroll
    for (int k = 0; k < j; ++k) dot = fma(a[k], rowj[k], dot);
    const R x = a[j] - dot;
    R d = __shfl(x, j, 64);
    if (!(d > (R)0) || !(d < (R)INFINITY)) {
      bad = 1;
      d = (R)1;
    }
    const R ljj = sqrt(d);
    const R lij = (i == j) ? ljj : x / ljj;
    a[j] = lij;
    if (i >= j) A[i * STR + j] = lij;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  return bad;
}

// X = L^{-1} for the lower-triangular 64x64 L in LDS tile A (wave 0; lane c owns column c
// of X).  Row-oriented substitution: X[i][c] = ([i==c] - sum_{k<i} L[i][k] X[k][c]) / L[i][i].
template <typename R>
__device__ void trinv_wave(const R* A, R* X) {
  constexpr int STR = Mfma<R>::STR;
  const int c = threadIdx.x & 63;
  R x[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    const R* rowi = A + i * STR;
    R dot = 0;
#pragma unroll
    for (int k = 0; k < i; ++k) dot = fma(rowi[k], x[k], dot);
    x[i] = ((i == c ? (R)1 : (R)0) - dot) / rowi[i];
  }
#pragma unroll
  for (int i = 0; i < 64; ++i) X[i * STR + c] = x[i];
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_cholesky(
    const R* __restrict__ Hc, int64_t ld, int T, const double* __restrict__ mu_dev, double mu_host,
    R* __restrict__ Lt, R* __restrict__ Linv, SyncArea* sync, uint32_t* flags,
    int32_t* status) {
  constexpr int STR = Mfma<R>::STR;
  using acc_t = typename Mfma<R>::acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* As = reinterpret_cast<R*>(smem_raw);
  R* Bs = As + 64 * STR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int qr = wv >> 1, qc = wv & 1;
  const double mu = mu_dev ? *mu_dev : mu_host;
  const uint32_t ntasks = (uint32_t)(T * (T + 1) / 2);

  for (;;) {
    const uint32_t t = claim(sync);
    if (t >= ntasks) break;
    int I, J;
    decode_ticket(t, T, I, J);

    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = qr * 32 + bi * 16 + out_row<R>(lane, v);
          const int c = qc * 32 + bj * 16 + out_col(lane, v);
          R h = Hc[(int64_t)(64 * J + c) * ld + 64 * I + r];
          if (I == J && r == c) h = (R)((double)h + mu);
          acc[bi][bj][v] = h;
        }

    bool ok = true;
    for (int K = 0; K < J && ok; ++K) {
      ok = wait_flag(flags + tile_index(I, K, T), sync, status);
      if (ok && I != J) ok = wait_flag(flags + tile_index(J, K, T), sync, status);
      if (!ok) break;
      tile_to_lds<R>(Lt + (int64_t)tile_index(I, K, T) * 4096, As);
      if (I != J) tile_to_lds<R>(Lt + (int64_t)tile_index(J, K, T) * 4096, Bs);
      __syncthreads();
      tile_mma<R, true>(acc, As, I != J ? Bs : As, qr, qc);
      __syncthreads();
    }

    if (I == J) {
      acc_to_lds<R>(acc, As, qr, qc);
      __syncthreads();
      __shared__ int s_bad;
      if (wv == 0) {
        const int bad = potrf_wave<R>(As);
        if (lane == 0) s_bad = bad;
      }
      __syncthreads();
      if (s_bad && tid == 0 && status) atomicOr(status, 1);
      if (wv == 0) trinv_wave<R>(As, Bs);
      __syncthreads();
      R* dstL = Lt + (int64_t)tile_index(J, J, T) * 4096;
      R* dstI = Linv + (int64_t)J * 4096;
      for (int e = tid; e < 4096; e += kThreads) {
        const int r = e >> 6, c = e & 63;
        dstL[e] = (c <= r) ? As[r * STR + c] : (R)0;
        dstI[e] = (c <= r) ? Bs[r * STR + c] : (R)0;
      }
    } else {
      if (ok) ok = wait_flag(flags + tile_index(J, J, T), sync, status);
      acc_to_lds<R>(acc, As, qr, qc);
      if (ok) tile_to_lds<R>(Linv + (int64_t)J * 4096, Bs);
      __syncthreads();
      acc_t out[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) out[bi][bj] = acc_t{0, 0, 0, 0};
      tile_mma<R, false>(out, As, Bs, qr, qc);
      acc_to_global<R>(out, Lt + (int64_t)tile_index(I, J, T) * 4096, qr, qc);
    }
    publish(flags + tile_index(I, J, T));
    __syncthreads();
  }
  exit_and_reset(sync, flags, (int)ntasks);
}

// ---------------------------------------------------------------------------------------
// Triangular solves on the tile-packed factor.  Thread layout inside a 64-row block:
// r = tid & 63 (row or column of the tile), part = tid >> 6 (a quarter of the other index).
// ---------------------------------------------------------------------------------------

// Gate: 0 = always run, 1 = skip if the factorisation failed, 2 = also skip once the
// refinement has converged.
__device__ __forceinline__ bool gated(const LMState* lm, int gate) {
  if (!lm || gate == 0) return false;
  if (lm->notpd) return true;
  return gate == 2 && lm->refine_done;
}

__device__ __forceinline__ double reduce4(double v, double* sh) {
  // sum the four parts (tid>>6) of row tid&63 in fixed order; result valid for tid < 64
  sh[threadIdx.x] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < 64)
    r = ((sh[threadIdx.x] + sh[threadIdx.x + 64]) + sh[threadIdx.x + 128]) + sh[threadIdx.x + 192];
  __syncthreads();
  return r;
}

// Forward: x = L^{-1} b.  Task I (in ticket order): s = b_I - sum_{K<I} L_IK x_K; x_I = Linv_II s.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_trsv_fwd(
    const R* __restrict__ Lt, const R* __restrict__ Linv, int T, const double* __restrict__ b,
    double* __restrict__ x, SyncArea* sync, uint32_t* flags, int32_t* status,
    const LMState* __restrict__ lm, int gate) {
  __shared__ double sh[kThreads];
  __shared__ double s_vec[64];
  if (gated(lm, gate)) {
    exit_and_reset(sync, flags, T);
    return;
  }
  const int tid = threadIdx.x, r = tid & 63, part = tid >> 6;
  for (;;) {
    const uint32_t t = claim(sync);
    if (t >= (uint32_t)T) break;
    const int I = (int)t;
    double acc = 0.0;
    bool ok = true;
    for (int K = 0; K < I; ++K) {
      ok = wait_flag(flags + K, sync, status);
      if (!ok) break;
      const R* tile = Lt + (int64_t)tile_index(I, K, T) * 4096 + r * 64 + part * 16;
      const double* xv = x + 64 * K + part * 16;
#pragma unroll
      for (int c = 0; c < 16; ++c) acc = fma((double)tile[c], xv[c], acc);
    }
    const double sum = reduce4(acc, sh);
    if (tid < 64) s_vec[tid] = b[64 * I + tid] - sum;
    __syncthreads();
    const R* inv = Linv + (int64_t)I * 4096 + r * 64 + part * 16;
    double y = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) y = fma((double)inv[c], s_vec[part * 16 + c], y);
    const double xi = reduce4(y, sh);
    if (tid < 64) x[64 * I + tid] = xi;
    publish(flags + I);
    __syncthreads();
  }
  exit_and_reset(sync, flags, T);
}

// Backward: x = L^{-T} b.  Task t solves block I = T-1-t: s = b_I - sum_{K>I} L_KI^T x_K;
// x_I = Linv_II^T s.  With acc_out != null the result is also added into acc_out (d += e).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_trsv_bwd(
    const R* __restrict__ Lt, const R* __restrict__ Linv, int T, const double* __restrict__ b,
    double* __restrict__ x, double* __restrict__ acc_out, SyncArea* sync, uint32_t* flags,
    int32_t* status, const LMState* __restrict__ lm, int gate) {
  __shared__ double sh[kThreads];
  __shared__ double s_vec[64];
  if (gated(lm, gate)) {
    exit_and_reset(sync, flags, T);
    return;
  }
  const int tid = threadIdx.x, c = tid & 63, part = tid >> 6;
  for (;;) {
    const uint32_t t = claim(sync);
    if (t >= (uint32_t)T) break;
    const int I = T - 1 - (int)t;
    double acc = 0.0;
    bool ok = true;
    for (int K = T - 1; K > I; --K) {
      ok = wait_flag(flags + K, sync, status);
      if (!ok) break;
      // (L_KI^T x_K)[c] = sum_r L_KI[r][c] x_K[r]
      const R* tile = Lt + (int64_t)tile_index(K, I, T) * 4096 + (part * 16) * 64 + c;
      const double* xv = x + 64 * K + part * 16;
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) acc = fma((double)tile[rr * 64], xv[rr], acc);
    }
    const double sum = reduce4(acc, sh);
    if (tid < 64) s_vec[tid] = b[64 * I + tid] - sum;
    __syncthreads();
    // x_I[c] = sum_r Linv[r][c] s[r]
    const R* inv = Linv + (int64_t)I * 4096 + (part * 16) * 64 + c;
    double y = 0.0;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) y = fma((double)inv[rr * 64], s_vec[part * 16 + rr], y);
    const double xi = reduce4(y, sh);
    if (tid < 64) {
      x[64 * I + tid] = xi;
      if (acc_out) acc_out[64 * I + tid] += xi;
    }
    publish(flags + I);
    __syncthreads();
  }
  exit_and_reset(sync, flags, T);
}

// Refinement residual s = g - (H + mu I) d in FP64 (H column-major lower, element type R),
// one workgroup per 64-row block; per-block ||s||^2 into s_part.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_refine_resid(
    const R* __restrict__ Hc, int64_t ld, int T, const double* __restrict__ mu_dev,
    const double* __restrict__ g, const double* __restrict__ d, double* __restrict__ s,
    double* __restrict__ s_part, const LMState* __restrict__ lm, int gate) {
  if (gated(lm, gate)) return;
  __shared__ double sh[kThreads];
  const int I = blockIdx.x;
  const int tid = threadIdx.x, r = tid & 63, part = tid >> 6;
  const int64_t row = 64 * (int64_t)I + r;
  double acc = 0.0;
  // columns left of the diagonal tile and the diagonal tile: H[row][col] at col*ld + row
  for (int J = 0; J < I; ++J) {
    for (int cc = 0; cc < 16; ++cc) {
      const int64_t col = 64 * (int64_t)J + part * 16 + cc;
      acc = fma((double)Hc[col * ld + row], d[col], acc);
    }
  }
  for (int cc = 0; cc < 16; ++cc) {
    const int cl = part * 16 + cc;
    const int64_t col = 64 * (int64_t)I + cl;
    const R h = (cl <= r) ? Hc[col * ld + row] : Hc[row * ld + col];
    acc = fma((double)h, d[col], acc);
  }
  // below the diagonal tile: H[row][col] = H[col][row] stored at row*ld + col
  for (int J = I + 1; J < T; ++J) {
    const R* src = Hc + row * ld + 64 * (int64_t)J + part * 16;
    const double* dv = d + 64 * (int64_t)J + part * 16;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc = fma((double)src[cc], dv[cc], acc);
  }
  const double hd = reduce4(acc, sh);
  double sq = 0.0;
  if (tid < 64) {
    const double mu = *mu_dev;
    const double si = g[row] - mu * d[row] - hd;
    s[row] = si;
    sq = si * si;
  }
  // fixed-order block sum of sq over the first wave
  if (tid < 64) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if (tid == 0) s_part[I] = sq;
  }
}

}  // namespace

template <typename R>
size_t chol_smem_bytes() {
  return 2 * 64 * Mfma<R>::STR * sizeof(R);
}

template <typename R>
hipError_t launch_cholesky(const R* Hc, int ld, int n_pad, const double* mu_dev, double mu_host,
                           R* Lt, R* Linv, SyncArea* sync, uint32_t* flags, int32_t* status,
                           const LMState*, hipStream_t st, int n_wg) {
  const int T = n_pad / 64;
  const int ntasks = T * (T + 1) / 2;
  const int grid = n_wg < ntasks ? n_wg : ntasks;
  hipLaunchKernelGGL(k_cholesky<R>, dim3(grid), dim3(kThreads), chol_smem_bytes<R>(), st, Hc,
                     (int64_t)ld, T, mu_dev, mu_host, Lt, Linv, sync, flags, status);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_trsv(bool forward, const R* Lt, const R* Linv, int n_pad, const double* b,
                       double* x, double* acc_out, SyncArea* sync, uint32_t* flags,
                       int32_t* status, const LMState* lm, int gate, hipStream_t st) {
  const int T = n_pad / 64;
  const int grid = T < 256 ? T : 256;
  if (forward)
    hipLaunchKernelGGL(k_trsv_fwd<R>, dim3(grid), dim3(kThreads), 0, st, Lt, Linv, T, b, x, sync,
                       flags, status, lm, gate);
  else
    hipLaunchKernelGGL(k_trsv_bwd<R>, dim3(grid), dim3(kThreads), 0, st, Lt, Linv, T, b, x,
                       acc_out, sync, flags, status, lm, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_refine_resid(const R* Hc, int ld, int n_pad, const double* mu_dev,
                               const double* g, const double* d, double* s, double* s_part,
                               const LMState* lm, int gate, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_resid<R>, dim3(n_pad / 64), dim3(kThreads), 0, st, Hc, (int64_t)ld,
                     n_pad / 64, mu_dev, g, d, s, s_part, lm, gate);
  return hipGetLastError();
}

hipError_t set_chol_smem_attr() {
  hipError_t e = hipFuncSetAttribute((const void*)k_cholesky<float>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)chol_smem_bytes<float>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_cholesky<double>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)chol_smem_bytes<double>());
}

#define DDC_INST(R)                                                                           \
  template hipError_t launch_cholesky<R>(const R*, int, int, const double*, double, R*, R*,    \
                                         SyncArea*, uint32_t*, int32_t*, const LMState*,       \
                                         hipStream_t, int);                                    \
  template hipError_t launch_trsv<R>(bool, const R*, const R*, int, const double*, double*,    \
                                     double*, SyncArea*, uint32_t*, int32_t*, const LMState*,  \
                                     int, hipStream_t);                                        \
  template hipError_t launch_refine_resid<R>(const R*, int, int, const double*, const double*, \
                                             const double*, double*, double*, const LMState*,  \
                                             int, hipStream_t);
DDC_INST(float)
DDC_INST(double)
#undef DDC_INST

}  // namespace ddc
