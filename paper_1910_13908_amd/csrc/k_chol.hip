// Dense damped Cholesky of the 8N x 8N normal matrix and the triangular solves of the LM step.
//
// The matrix is symmetric positive definite after damping (H + mu I, mu > 0).  It is
// factored as L L^T in 64 x 64 tiles by ONE persistent kernel: workgroups take tiles of the
// lower triangle from an atomic ticket in column-major tile order, and each tile is owned by
// one workgroup from its first update to its final value (left-looking):
//
//   A_IJ <- H_IJ + mu [I==J] - sum_{K<J} L_IK L_JK^T      (MFMA, double-buffered LDS operands)
//   I == J:  L_JJ = chol(A_JJ) and X_JJ = L_JJ^{-1}       (blocked 16-column panels + MFMA)
//   I >  J:  L_IJ = A_IJ X_JJ^T                           (MFMA with the stored inverse)
//
// One workgroup walks the diagonal (subdiagonal tile, update, factor and inverse of every
// diagonal tile in turn) with its operands in LDS, so the dependent chain along the
// diagonal never waits on another workgroup; the others pre-accumulate what it needs and
// fill in the rest of the factor.  With a right-hand side g the same kernel also runs the
// forward substitution y = L^{-1} g block by block as the factor appears.  Every wait is on
// work that is finished or held by a running workgroup: tickets are claimed only by running
// workgroups, so the smallest unfinished ticket never waits on unfinished work and the
// schedule cannot deadlock without any co-residency guarantee.  Every wait is bounded; on
// expiry the kernel raises an abort flag, every other wait returns at once, and the status
// word reports DDC_ETIMEOUT.
//
// Hand-offs between workgroups.  An agent-scope release/acquire pair writes back and
// invalidates the L2 of the XCDs involved, which dominated the kernel's time, so the FP32
// factorisation has none: every tile a task hands over is also written as a tagged copy (each
// 64-bit slot holds the value and the launch's sequence number) that consumers poll until
// every tag they read matches, and the forward solve passes its blocks as messages that hold
// an "empty" pattern until written.  FP64 values leave no room for a tag: there results
// publish ready flags with release/acquire.  The last workgroup to leave resets the tickets,
// flags and messages, so the kernel needs no host-side clearing between launches.
//
// The factor is stored tile-packed (column-major over the tiles of the lower triangle,
// row-major inside a tile while it is built; after the factorisation k_transpose_tiles
// rewrites every tile in the solves' layout and writes their transposed copies) next to the
// inverses of the diagonal tiles, which the triangular solves use as small dense products.
// Forward and backward substitution use the same ticket scheme over 64-row blocks, with
// message hand-offs.  In mixed precision the factor and the products run in FP32 (FP32
// MFMA); right-hand sides, solutions and the refinement residual g - (H + mu I) d are FP64.
#include "common.h"

#include <type_traits>

namespace ddc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kSpinLimit = 1u << 22;   // polls (with s_sleep) before a wait gives up

// The bound of every wait of a launch: the host may lower it through the sync area's spare
// word (ddc_set_wait_limit, to exercise the timeout path); zero keeps kSpinLimit.
__device__ __forceinline__ uint32_t spin_limit(const SyncArea* sync) {
  const uint32_t v = sync->pad;
  return v ? v : kSpinLimit;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

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
      if (++spins > spin_limit(sync)) {
        __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (status) atomicOr(status, 2);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Number of leading K in [0, nK) whose flags (I_a, K) and (I_b, K) are already set, found
// with one relaxed load per flag in parallel and one agent-scope acquire for the whole
// prefix, so the common case (operands finished long ago) pays a single fence.
__device__ int ready_prefix(const uint32_t* flags, int T, int IA, int IB, int nK) {
  __shared__ int s_first_missing;
  if (threadIdx.x == 0) s_first_missing = nK;
  __syncthreads();
  for (int K = threadIdx.x; K < nK; K += blockDim.x) {
    const uint32_t ti_a = (uint32_t)(K * T - (K * (K - 1)) / 2 + (IA - K));
    const uint32_t ti_b = (uint32_t)(K * T - (K * (K - 1)) / 2 + (IB - K));
    const bool ready = __hip_atomic_load(flags + ti_a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u &&
                       __hip_atomic_load(flags + ti_b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (!ready) atomicMin(&s_first_missing, K);
  }
  __syncthreads();
  const int n = s_first_missing;
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return n;
}

__device__ __forceinline__ void publish(uint32_t* flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Leave the persistent loop; the last workgroup out clears the flags and the counters.
__device__ void exit_and_reset(SyncArea* sync, uint32_t* flags, int nflags,
                               uint32_t* flags2 = nullptr, int nflags2 = 0,
                               uint64_t* msgs = nullptr, int nmsgs = 0) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&sync->exited, 1u) == gridDim.x - 1);
  __syncthreads();
  if (s_last) {
    __threadfence();
    for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0u;
    for (int i = threadIdx.x; i < nflags2; i += blockDim.x) flags2[i] = 0u;
    for (int i = threadIdx.x; i < nmsgs; i += blockDim.x)   // the "empty" message pattern
      __hip_atomic_store(msgs + i, 0x7FF4DD0000000001ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const f32x4* s4 = reinterpret_cast<const f32x4*>(src);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * kThreads;       // 1024 x 4 floats
      const int r = idx >> 4, c = (idx & 15) * 4;
      *reinterpret_cast<f32x4*>(dst + r * STR + c) = s4[idx];
    }
  } else {
    const f64x2* s2 = reinterpret_cast<const f64x2*>(src);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = threadIdx.x + it * kThreads;       // 2048 x 2 doubles
      const int r = idx >> 5, c = (idx & 31) * 2;
      *reinterpret_cast<f64x2*>(dst + r * STR + c) = s2[idx];
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
  // four chunks of four consecutive k per lane keep only 16 operand values live
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    R x0[4], x1[4], y0[4], y1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x0[u] = a0[4 * ch + u];
      x1[u] = a1[4 * ch + u];
      y0[u] = b0[4 * ch + u];
      y1[u] = b1[4 * ch + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const R p0 = NEG ? -x0[u] : x0[u];
      const R p1 = NEG ? -x1[u] : x1[u];
      acc[0][0] = Mfma<R>::mma(p0, y0[u], acc[0][0]);
      acc[0][1] = Mfma<R>::mma(p0, y1[u], acc[0][1]);
      acc[1][0] = Mfma<R>::mma(p1, y0[u], acc[1][0]);
      acc[1][1] = Mfma<R>::mma(p1, y1[u], acc[1][1]);
    }
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

// ---------------------------------------------------------------------------------------
// Diagonal tile: Cholesky factor and inverse of a 64x64 LDS tile (row-major, stride STR).
// Blocked right-looking with 16-column panels: wave 0 factors a panel (lane i owns row i,
// Crout order inside the panel, pivots broadcast with readlane, 1/sqrt via rsq), then all
// four waves apply the rank-16 trailing update with MFMA.  The inverse X = L^{-1} is built
// from the four 16x16 diagonal inverses (one wave each, forward substitution) and, block
// row by block row, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj with MFMA.
// ---------------------------------------------------------------------------------------

// Index inside a 16-wide reduction walked by lane group g at step s, chosen so that an
// MFMA result element v = s of lane l is exactly the B operand that lane needs.
template <typename R>
__device__ __forceinline__ int kwalk16(int g, int s) {
  return sizeof(R) == 4 ? 4 * g + s : g + 4 * s;
}

__device__ __forceinline__ float bcast_lane(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double bcast_lane(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float rsq_full(float d) { return __builtin_amdgcn_rsqf(d); }
__device__ __forceinline__ double rsq_full(double d) {
  double r = __builtin_amdgcn_rsq(d);
  // two Newton steps r <- r (3 - d r^2) / 2 take the hardware estimate to full precision
  r = r * fma(-0.5 * d, r * r, 1.5);
  r = r * fma(-0.5 * d, r * r, 1.5);
  return r;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave 0: factor columns 16P..16P+15 (rows >= 16P) in place; returns nonzero on a bad pivot.
// Lane i keeps its panel row in registers.  Right-looking inside the panel: once column j is
// scaled, each later column jj takes its rank-1 update with the multiplier L[16P+jj][j] of
// lane 16P+jj: the next column's by readlane, so that only the pivot broadcast, the rsq and
// one update sit on the serial chain, the others read back from LDS as broadcast vectors
// (readlanes would occupy the VALU).  The pivot lane holds d itself, so scaling every lane by
// rsq(d) leaves sqrt(d) on the diagonal.  The whole panel is written back: entries above the
// diagonal of the tile are never read.
template <typename R, int P>
__device__ int panel_factor(R* A, R* rdiag, R* colbuf) {
  constexpr int STR = Mfma<R>::STR;
  constexpr int c0 = 16 * P;
  const int i = threadIdx.x & 63;
  R a[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = A[i * STR + c0 + j];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const R r = rsq_full(bcast_lane(a[j], c0 + j));
    a[j] *= r;
    if (i == 0) rdiag[c0 + j] = r;
    if (j + 1 < 16) {
      // the next column's multiplier by readlane (it is on the chain); the later ones
      // through LDS: every lane stores its a[j], and all read the 16 of the panel's rows back
      // as broadcast vectors, off the chain and off the VALU
      a[j + 1] = fma(-a[j], bcast_lane(a[j], c0 + j + 1), a[j + 1]);
      if (j + 2 < 16) {
        colbuf[j * 64 + i] = a[j];
        R m[16];
        if constexpr (sizeof(R) == 4) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 t = *reinterpret_cast<const f32x4*>(colbuf + j * 64 + c0 + 4 * q);
            m[4 * q] = t[0];
            m[4 * q + 1] = t[1];
            m[4 * q + 2] = t[2];
            m[4 * q + 3] = t[3];
          }
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const f64x2 t = *reinterpret_cast<const f64x2*>(colbuf + j * 64 + c0 + 2 * q);
            m[2 * q] = t[0];
            m[2 * q + 1] = t[1];
          }
        }
#pragma unroll
        for (int jj = j + 2; jj < 16; ++jj) a[jj] = fma(-a[j], m[jj], a[jj]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) A[i * STR + c0 + j] = a[j];
  // a pivot d <= 0, inf or nan leaves 1/sqrt(d) outside (0, inf): one check per column after
  // the panel instead of a lane mask per column inside it (the values are then garbage, and
  // the caller discards them on the flag)
  const R rc = rdiag[c0 + (i & 15)];
  return __any(!(rc > (R)0 && rc < (R)INFINITY)) ? 1 : 0;
}

// Zero the six 16x16 blocks above the block diagonal of a 64x64 LDS tile.
template <typename R>
__device__ __forceinline__ void zero_upper_blocks(R* X) {
  constexpr int STR = Mfma<R>::STR;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int e = threadIdx.x + k * kThreads;       // 6 x 256 elements
    const int blk = e >> 8, r = (e >> 4) & 15, c = e & 15;
    // blk 0..5 -> (row block, column block) = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    const int bi = blk < 3 ? 0 : (blk < 5 ? 1 : 2);
    const int bj = blk < 3 ? blk + 1 : (blk < 5 ? blk - 1 : 3);
    X[(16 * bi + r) * STR + 16 * bj + c] = (R)0;
  }
}

// One wave: A[br][bc] -= A[br][P] A[bc][P]^T for one 16x16 block (the rank-16 update of panel
// P), with MFMA.
template <typename R>
__device__ __forceinline__ void block_update(R* A, int br, int bc, int P) {
  constexpr int STR = Mfma<R>::STR;
  using acc_t = typename Mfma<R>::acc_t;
  const int lane = threadIdx.x & 63, g = lane >> 4, rr = lane & 15;
  acc_t acc;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    acc[v] = A[(16 * br + out_row<R>(lane, v)) * STR + 16 * bc + out_col(lane, v)];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 16 * P + 4 * g + s;
    acc = Mfma<R>::mma(-A[(16 * br + rr) * STR + k], A[(16 * bc + rr) * STR + k], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    A[(16 * br + out_row<R>(lane, v)) * STR + 16 * bc + out_col(lane, v)] = acc[v];
}

// One wave: X_bb = L_bb^{-1} of diagonal 16x16 block b by forward substitution, lane c < 16
// taking column c; the right-hand side e_c is formed arithmetically (no per-row lane masks).
// FP32: the block's lower triangle and the pivot reciprocals are read from LDS first, as
// 16-byte vectors, so the substitution waits for LDS once rather than once per row (in FP64
// the 120 values would take 240 registers, and the rows are read as they are needed).
template <typename R>
__device__ __forceinline__ void diag_inverse(const R* A, R* X, const R* rdiag, int b) {
  constexpr int STR = Mfma<R>::STR;
  const int lane = threadIdx.x & 63;
  if constexpr (sizeof(R) == 8) {
    // FP64: each row's part of the block and its pivot reciprocal are read one row ahead, as
    // 16-byte vectors, so that the substitution of a row does not wait for its own reads
    if (lane < 16) {
      const int b0 = 16 * b, c = lane;
      R x[16], cur[16], nxt[16], rcur, rnxt;
      rcur = rdiag[b0];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i + 1 < 16) {
#pragma unroll
          for (int k0 = 0; k0 < i + 1; k0 += 2) {
            const f64x2 t = *reinterpret_cast<const f64x2*>(A + (b0 + i + 1) * STR + b0 + k0);
            nxt[k0] = t[0];
            nxt[k0 + 1] = t[1];
          }
          rnxt = rdiag[b0 + i + 1];
        }
        R d0 = 0, d1 = 0;
#pragma unroll
        for (int k = 0; k < i; k += 2) {
          d0 = fma(cur[k], x[k], d0);
          if (k + 1 < i) d1 = fma(cur[k + 1], x[k + 1], d1);
        }
        const R e = (R)(1 - min(abs(i - c), 1));
        x[i] = (e - (d0 + d1)) * rcur;
#pragma unroll
        for (int k = 0; k < 16; ++k) cur[k] = nxt[k];
        rcur = rnxt;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) X[(b0 + i) * STR + b0 + c] = x[i];
    }
    return;
  }
  constexpr int V = 16 / (int)sizeof(R);            // elements per 16-byte vector
  if (lane < 16) {
    const int b0 = 16 * b, c = lane;
    R L[16][16];
#pragma unroll
    for (int i = 1; i < 16; ++i) {
#pragma unroll
      for (int k0 = 0; k0 < i; k0 += V) {
        const f32x4 t = *reinterpret_cast<const f32x4*>(A + (b0 + i) * STR + b0 + k0);
#pragma unroll
        for (int w = 0; w < V; ++w) L[i][k0 + w] = t[w];
      }
    }
    R rd[16];
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += V) {
      const f32x4 t = *reinterpret_cast<const f32x4*>(rdiag + b0 + k0);
#pragma unroll
      for (int w = 0; w < V; ++w) rd[k0 + w] = t[w];
    }
    R x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      R d0 = 0, d1 = 0;
#pragma unroll
      for (int k = 0; k < i; k += 2) {
        d0 = fma(L[i][k], x[k], d0);
        if (k + 1 < i) d1 = fma(L[i][k + 1], x[k + 1], d1);
      }
      const R e = (R)(1 - min(abs(i - c), 1));
      x[i] = (e - (d0 + d1)) * rd[i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) X[(b0 + i) * STR + b0 + c] = x[i];
  }
}

// One wave: X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj (i > j), with MFMA.
template <typename R>
__device__ __forceinline__ void offdiag_inverse(const R* A, R* X, int i, int j) {
  constexpr int STR = Mfma<R>::STR;
  using acc_t = typename Mfma<R>::acc_t;
  const int lane = threadIdx.x & 63, g = lane >> 4, rr = lane & 15;
  acc_t t = acc_t{0, 0, 0, 0};
  for (int k = j; k < i; ++k) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int m = kwalk16<R>(g, s);
      t = Mfma<R>::mma(A[(16 * i + rr) * STR + 16 * k + m], X[(16 * k + m) * STR + 16 * j + rr], t);
    }
  }
  acc_t o = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s)
    o = Mfma<R>::mma(-X[(16 * i + rr) * STR + 16 * i + kwalk16<R>(g, s)], t[s], o);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    X[(16 * i + out_row<R>(lane, v)) * STR + 16 * j + out_col(lane, v)] = o[v];
}

// Factor the tile in A (lower triangle) in place and write X = L^{-1} into X; the blocks of X
// above its block diagonal must already hold zeros (zero_upper_blocks).  Returns nonzero (in
// every thread) if a pivot was not positive.  Six phases, one workgroup barrier each: wave 0
// runs the chain (the part of the previous panel's update that the next panel needs, then that
// panel's factorisation), while waves 1-3 apply the rest of the update and form the inverse
// blocks whose operands are final:
//   1: w0 U0 on panel 1, P1 | w1 U0 on (2,2),(3,2) | w2 U0 on (3,3) | w3 X_00
//   2: w0 U1 on panel 2, P2 | w1 U1 on (3,3)       | w2 X_11
//   3: w0 U2 on panel 3, P3 | w1 X_22              | w2 X_10
//   4: w0 X_33              | w1 X_20              | w2 X_21
//   5: w0 X_30              | w1 X_31              | w2 X_32
template <typename R>
__device__ int cholinv_tile(R* A, R* X, R* rdiag) {
  __shared__ int s_bad;
  __shared__ __align__(16) R colbuf[14 * 64];     // panel columns 0..13 (multipliers)
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int bad = 0;
  if (wv == 0) bad |= panel_factor<R, 0>(A, rdiag, colbuf);
  __syncthreads();
  if (wv == 0) {
    block_update<R>(A, 1, 1, 0);
    block_update<R>(A, 2, 1, 0);
    block_update<R>(A, 3, 1, 0);
    wave_sync_lds();
    bad |= panel_factor<R, 1>(A, rdiag, colbuf);
  } else if (wv == 1) {
    block_update<R>(A, 2, 2, 0);
    block_update<R>(A, 3, 2, 0);
  } else if (wv == 2) {
    block_update<R>(A, 3, 3, 0);
  } else {
    diag_inverse<R>(A, X, rdiag, 0);
  }
  __syncthreads();
  if (wv == 0) {
    block_update<R>(A, 2, 2, 1);
    block_update<R>(A, 3, 2, 1);
    wave_sync_lds();
    bad |= panel_factor<R, 2>(A, rdiag, colbuf);
  } else if (wv == 1) {
    block_update<R>(A, 3, 3, 1);
  } else if (wv == 2) {
    diag_inverse<R>(A, X, rdiag, 1);
  }
  __syncthreads();
  if (wv == 0) {
    block_update<R>(A, 3, 3, 2);
    wave_sync_lds();
    bad |= panel_factor<R, 3>(A, rdiag, colbuf);
    if (lane == 0) s_bad = bad;
  } else if (wv == 1) {
    diag_inverse<R>(A, X, rdiag, 2);
  } else if (wv == 2) {
    offdiag_inverse<R>(A, X, 1, 0);
  }
  __syncthreads();
  if (wv == 0) diag_inverse<R>(A, X, rdiag, 3);
  else if (wv == 1) offdiag_inverse<R>(A, X, 2, 0);
  else if (wv == 2) offdiag_inverse<R>(A, X, 2, 1);
  __syncthreads();
  if (wv < 3) offdiag_inverse<R>(A, X, 3, wv);
  __syncthreads();
  return s_bad;
}

// ---------------------------------------------------------------------------------------
// Operand staging for the tile updates: one 64x64 packed tile is 16 elements per thread.
// ---------------------------------------------------------------------------------------
template <typename R>
struct TileRegs;
template <>
struct TileRegs<float> {
  f32x4 v[4];
};
template <>
struct TileRegs<double> {
  f64x2 v[8];
};

template <typename R>
__device__ __forceinline__ void tile_fetch(const R* __restrict__ src, TileRegs<R>& t) {
  if constexpr (sizeof(R) == 4) {
    const f32x4* s4 = reinterpret_cast<const f32x4*>(src);
#pragma unroll
    for (int it = 0; it < 4; ++it) t.v[it] = s4[threadIdx.x + it * kThreads];
  } else {
    const f64x2* s2 = reinterpret_cast<const f64x2*>(src);
#pragma unroll
    for (int it = 0; it < 8; ++it) t.v[it] = s2[threadIdx.x + it * kThreads];
  }
}

template <typename R>
__device__ __forceinline__ void tile_stash(const TileRegs<R>& t, R* dst) {
  constexpr int STR = Mfma<R>::STR;
  if constexpr (sizeof(R) == 4) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * kThreads;
      *reinterpret_cast<f32x4*>(dst + (idx >> 4) * STR + (idx & 15) * 4) = t.v[it];
    }
  } else {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = threadIdx.x + it * kThreads;
      *reinterpret_cast<f64x2*>(dst + (idx >> 5) * STR + (idx & 31) * 2) = t.v[it];
    }
  }
}

template <typename R>
__device__ __forceinline__ void acc_load_h(typename Mfma<R>::acc_t (&acc)[2][2],
                                           const R* __restrict__ Hc, int64_t ld, int I, int J,
                                           double mu, int qr, int qc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = qr * 32 + bi * 16 + out_row<R>(lane, v);
        const int c = qc * 32 + bj * 16 + out_col(lane, v);
        R h = Hc[(int64_t)(64 * J + c) * ld + 64 * I + r];
        if (I == J) {
          // mu on the diagonal only, selected arithmetically: a per-element lane mask here
          // would be hoisted out of the step loop and exhaust the scalar registers
          const double on = (double)(1 - min(abs(r - c), 1));
          h = (R)((double)h + mu * on);
        }
        acc[bi][bj][v] = h;
      }
}

// Messages: 64-bit slots written and read with agent-scope relaxed atomics; a slot holding
// kEmpty (a signalling-NaN payload that no arithmetic result carries) is not written yet.
constexpr uint64_t kEmpty = 0x7FF4DD0000000001ull;

__device__ __forceinline__ uint64_t msg_get(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void msg_put(uint64_t* p, double v) {
  __hip_atomic_store(p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Per-lane bounded poll of one message slot; on abort or time-out returns kEmpty (the caller
// carries on with garbage; the status word reports the failure).
__device__ uint64_t msg_wait(uint64_t* p, SyncArea* sync, int32_t* status) {
  uint32_t spins = 0;
  uint64_t m;
  while ((m = msg_get(p)) == kEmpty) {
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return m;
}

// v[j] = the doubles at p + off(j) once none holds kEmpty (bounded poll).
template <typename F>
__device__ bool msg_get16(const uint64_t* p, F off, double (&v)[16], SyncArea* sync,
                          int32_t* status) {
  uint32_t spins = 0;
  for (;;) {
    uint64_t m[16];
#pragma unroll
    for (int j = 0; j < 16; ++j)
      m[j] = __hip_atomic_load(p + off(j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool all = true;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      all &= m[j] != kEmpty;
      v[j] = __longlong_as_double((long long)m[j]);
    }
    if (all) return true;
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Look-ahead tiles in FP32 travel as tagged messages: each 64-bit slot holds a value and
// the launch's sequence number, so the diagonal worker reads them as soon as they exist, with
// no flag, no fence and no clearing between launches.  Slot (tile s, which, k, thread) sits at
// ((s * 2 + which) * 16 + k) * kThreads + thread, so a wave's accesses are contiguous.
__device__ __forceinline__ uint64_t* tagged_slots(void* base, int s, int which) {
  return reinterpret_cast<uint64_t*>(base) + (int64_t)(s * 2 + which) * 16 * kThreads;
}
__device__ __forceinline__ void tagged_put16(uint64_t* p, uint32_t seq,
                                             const Mfma<float>::acc_t (&acc)[2][2]) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = (bi * 2 + bj) * 4 + v;
        const uint64_t m = ((uint64_t)seq << 32) | (uint64_t)__float_as_uint(acc[bi][bj][v]);
        __hip_atomic_store(p + k * kThreads + threadIdx.x, m, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
}
// One look-ahead tile: its 16 loads per thread are issued without waiting (tagged_issue16) and
// the values taken once every tag matches (tagged_take16); tagged_poll16 is the bounded wait.
// Keeping issue and use apart lets the loads stay in flight over other work.
__device__ __forceinline__ void tagged_issue16(const uint64_t* p, uint64_t (&m)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k)
    m[k] = __hip_atomic_load(p + k * kThreads + threadIdx.x, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool tagged_take16(const uint64_t (&m)[16], uint32_t seq,
                                              Mfma<float>::acc_t (&acc)[2][2]) {
  bool all = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) all &= (uint32_t)(m[k] >> 32) == seq;
  if (!all) return false;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[bi][bj][v] = __uint_as_float((uint32_t)m[(bi * 2 + bj) * 4 + v]);
  return true;
}
// false on abort or time-out
__device__ bool tagged_poll16(const uint64_t* p, uint32_t seq, Mfma<float>::acc_t (&acc)[2][2],
                              SyncArea* sync, int32_t* status) {
  uint32_t spins = 0;
  for (;;) {
    uint64_t m[16];
    tagged_issue16(p, m);
    if (tagged_take16(m, seq, acc)) return true;
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// In FP32 every tile a task hands to another (L_IJ, and in the slot of the diagonal tile
// (s, s) the inverse X_s) is also written as a tagged copy and read from there, so no task
// publishes a flag or runs a fence.  The copy is laid out in the order its readers load it:
// a reader's thread t holds elements 4 (t + 256 i) + u (i, u = 0..3; the tile_fetch layout),
// and element e = 4 (t + 256 i) + u sits in slot (4 i + u) * 256 + t, so that every load
// instruction of a wave reads 512 contiguous bytes.  The copies sit after the look-ahead
// tiles' messages, tile t at t * 4096 (column-major tile order).
__device__ __forceinline__ uint64_t* tile_slots(void* base, int T, uint32_t ti) {
  return reinterpret_cast<uint64_t*>(base) + (int64_t)T * 2 * 16 * kThreads + (int64_t)ti * 4096;
}
__device__ __forceinline__ int slot_of(int e) {
  return ((e >> 10) * 4 + (e & 3)) * kThreads + ((e >> 2) & (kThreads - 1));
}
__device__ __forceinline__ int elem_of_slot(int q) {
  return 4 * ((q & (kThreads - 1)) + kThreads * (q >> 10)) + ((q >> 8) & 3);
}
// FP32: the forward-substitution blocks y_K as messages (T x 64 slots, kEmpty between launches)
__device__ __forceinline__ uint64_t* y_slots(void* base, int T) {
  return reinterpret_cast<uint64_t*>(base) + (int64_t)T * 2 * 16 * kThreads +
         (int64_t)T * (T + 1) / 2 * 4096;
}
__device__ __forceinline__ void tagged_put(uint64_t* p, uint32_t seq, float v) {
  __hip_atomic_store(p, ((uint64_t)seq << 32) | (uint64_t)__float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// The tagged copy of a 64x64 LDS tile (row stride STR): thread t stores slots k * 256 + t,
// k = 0..15, so each store instruction of a wave writes 512 contiguous bytes; slot 4095 (the
// one waiting tasks watch) is the last store of the last wave.
__device__ __forceinline__ void tagged_put_lds(uint64_t* t, uint32_t seq, const float* X) {
  constexpr int STR = Mfma<float>::STR;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int q = k * kThreads + threadIdx.x;
    const int e = elem_of_slot(q);
    tagged_put(t + q, seq, X[(e >> 6) * STR + (e & 63)]);
  }
}
// v[j] = element base_e[j] of a tagged tile once all 16 carry tag seq (bounded poll).
template <typename F>
__device__ bool tagged_get16(const uint64_t* t, uint32_t seq, F elem, float (&v)[16],
                             SyncArea* sync, int32_t* status) {
  uint32_t spins = 0;
  for (;;) {
    uint64_t m[16];
#pragma unroll
    for (int j = 0; j < 16; ++j)
      m[j] = __hip_atomic_load(t + elem(j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool all = true;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      all &= (uint32_t)(m[j] >> 32) == seq;
      v[j] = __uint_as_float((uint32_t)m[j]);
    }
    if (all) return true;
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}
// The tile_fetch layout (thread t holds elements 4 (t + 256 i) .. + 3, i = 0..3) from a
// tagged tile.
__device__ __forceinline__ bool tagged_tile_fetch(const uint64_t* t, uint32_t seq,
                                                  TileRegs<float>& r, SyncArea* sync,
                                                  int32_t* status) {
  float v[16];
  const int tid = threadIdx.x;
  const bool ok = tagged_get16(t, seq, [&](int j) { return j * kThreads + tid; }, v, sync, status);
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = f32x4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]};
  return ok;
}

// The same tile as tagged_tile_fetch in two halves: tagged_tile_issue starts the 16 loads and
// tagged_tile_take converts them once every tag matches (false if one does not yet), so the
// loads can stay in flight over other work.
__device__ __forceinline__ void tagged_tile_issue(const uint64_t* t, uint64_t (&m)[16]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    m[j] = __hip_atomic_load(t + j * kThreads + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool tagged_tile_take(const uint64_t (&m)[16], uint32_t seq,
                                                 TileRegs<float>& r) {
  bool all = true;
#pragma unroll
  for (int j = 0; j < 16; ++j) all &= (uint32_t)(m[j] >> 32) == seq;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    r.v[i] = f32x4{__uint_as_float((uint32_t)m[4 * i]), __uint_as_float((uint32_t)m[4 * i + 1]),
                   __uint_as_float((uint32_t)m[4 * i + 2]), __uint_as_float((uint32_t)m[4 * i + 3])};
  return all;
}

// Bounded wait until the last slot a tagged tile's writer stores (element 4095: the last
// store of its last wave) carries tag seq.  Every lane reads the same slot, so a poll is one
// request per wave; the whole tile is fetched (and every tag checked) only after it.  With
// dozens of tasks waiting on one tile, whole-tile polls would load the lines its writer is
// still storing to many times over.
__device__ bool tagged_watch(const uint64_t* t, uint32_t seq, SyncArea* sync, int32_t* status) {
  uint32_t spins = 0;
  while ((uint32_t)(__hip_atomic_load(t + 4095, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) != seq) {
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Both tiles of an accumulation step, polled together (bounded): one round trip per poll
// for the pair instead of one per tile.
__device__ bool tagged_tile_fetch2(const uint64_t* ta, const uint64_t* tb, uint32_t seq,
                                   TileRegs<float>& ra, TileRegs<float>& rb, SyncArea* sync,
                                   int32_t* status) {
  uint32_t spins = 0;
  for (;;) {
    uint64_t ma[16], mb[16];
    tagged_tile_issue(ta, ma);
    tagged_tile_issue(tb, mb);
    const bool ga = tagged_tile_take(ma, seq, ra);
    const bool gb = tagged_tile_take(mb, seq, rb);
    if (ga && gb) return true;
    if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (++spins > spin_limit(sync)) {
      __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (status) atomicOr(status, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Roles of the factorisation.  Ticket 0 makes its workgroup the diagonal worker (DW): it
// factors the diagonal tiles in order, s = 0..T-1, and keeps each inverse in LDS for the next
// step, so the chain of dependent diagonal factorisations has no inter-workgroup hand-off.
// At step s it computes the subdiagonal tile L_{s,s-1} = A_{s,s-1} X_{s-1}^T, applies its
// rank-64 update to the diagonal tile and factors/inverts it.  Every other workgroup takes
// tickets >= 1 in groups g = 0..T-1:
//   DA_{g+1}, DD_{g+1} (2 <= g+1 <= T-1): the tiles the DW starts step g+1 from, all but its
//            last product: A_{g+1,g} - sum_{K <= g-1} L_{g+1,K} L_{g,K}^T (DA) and
//            A_{g+1,g+1} + mu I - sum_{K <= g-1} L_{g+1,K} L_{g+1,K}^T (DD);
//   Y_g:     forward-substitution block y_g = X_gg (g_g - sum_{K<g} L_gK y_K);
//   R_g:     tiles (I, g), I >= g+2: A_Ig - sum_K L_IK L_gK^T, then times X_gg^T.
// A task waits only on tasks of earlier groups or on DW steps whose own inputs come from
// earlier groups, so the schedule cannot deadlock with any number (>= 2) of resident
// workgroups.
enum { TASK_DW = 0, TASK_DA = 1, TASK_Y = 2, TASK_R = 3, TASK_DD = 4, TASK_NONE = 5 };

__device__ __forceinline__ void decode_task(uint32_t t, int T, int& kind, int& I, int& J) {
  kind = TASK_NONE;
  I = J = 0;
  if (t == 0) { kind = TASK_DW; return; }
  t -= 1;
  for (int g = 0; g < T; ++g) {
    const uint32_t da = (g >= 1 && g + 1 <= T - 1) ? 2u : 0u;
    const uint32_t nr = (uint32_t)max(0, T - g - 2);
    if (t < da + 1 + nr) {
      if (da) {
        if (t == 0) { kind = TASK_DA; I = J = g + 1; return; }
        if (t == 1) { kind = TASK_DD; I = J = g + 1; return; }
        t -= 2;
      }
      if (t == 0) { kind = TASK_Y; I = J = g; return; }
      kind = TASK_R; J = g; I = g + 2 + (int)(t - 1);
      return;
    }
    t -= da + 1 + nr;
  }
}

__host__ __device__ inline uint32_t chol_tasks(int T) {
  const int da = T >= 2 ? 2 * (T - 2) : 0;
  const int nr = T >= 2 ? (T - 2) * (T - 1) / 2 : 0;
  return (uint32_t)(1 + T + da + nr);
}

// Accumulate acc1 -= A_K B_K^T (and acc2 -= A_K A_K^T when TWO) over K < nK, where
// A_K = L(IA, K), B_K = L(IB, K), with a double-buffered LDS pipeline: the next pair of
// tiles is fetched into registers while the current pair feeds the MFMAs.
// FP32 reads every operand from the tagged copies (no flags); FP64 waits on the tiles' flags
// (one acquire for the prefix already set, then one by one).
template <typename R, bool TWO>
__device__ __forceinline__ bool accumulate(typename Mfma<R>::acc_t (&acc1)[2][2],
                                           typename Mfma<R>::acc_t (&acc2)[2][2],
                           const R* __restrict__ Lt, int T, int IA, int IB, int nK, R* lds,
                           SyncArea* sync, uint32_t* flags, int32_t* status, int qr, int qc,
                           void* tagbase, uint32_t seq) {
  constexpr int STR = Mfma<R>::STR;
  constexpr int TILE = 64 * STR;
  constexpr bool TAG = sizeof(R) == 4;
  if (nK <= 0) return true;
  TileRegs<R> ra, rb;
  const int ready = TAG ? nK : ready_prefix(flags, T, IA, IB, nK);
  bool ok = true;
  auto wait_k = [&](int K) {
    if (TAG || K < ready || !ok) return;
    ok = wait_flag(flags + tile_index(IA, K, T), sync, status);
    if (ok && IB != IA) ok = wait_flag(flags + tile_index(IB, K, T), sync, status);
  };
  auto fetch_k = [&](int K) {
    if constexpr (TAG) {
      // per-thread polls; ok is made uniform once, at the end
      const bool ga = tagged_tile_fetch(tile_slots(tagbase, T, tile_index(IA, K, T)), seq, ra,
                                        sync, status);
      const bool gb = tagged_tile_fetch(tile_slots(tagbase, T, tile_index(IB, K, T)), seq, rb,
                                        sync, status);
      ok = ok && ga && gb;
    } else {
      tile_fetch<R>(Lt + (int64_t)tile_index(IA, K, T) * 4096, ra);
      tile_fetch<R>(Lt + (int64_t)tile_index(IB, K, T) * 4096, rb);
    }
  };
  wait_k(0);
  fetch_k(0);
  tile_stash<R>(ra, lds);
  tile_stash<R>(rb, lds + TILE);
  __syncthreads();
  int buf = 0;
  for (int K = 0; K < nK; ++K) {
    const bool more = K + 1 < nK;
    // FP32: the next pair's loads are issued before this pair's products and taken after
    // them, so a pair that is still being written is waited for behind the products
    uint64_t ma[16], mb[16];
    if constexpr (TAG) {
      const int Kn = more ? K + 1 : K;
      tagged_tile_issue(tile_slots(tagbase, T, tile_index(IA, Kn, T)), ma);
      tagged_tile_issue(tile_slots(tagbase, T, tile_index(IB, Kn, T)), mb);
    } else if (more && ok) {
      wait_k(K + 1);
      fetch_k(K + 1);
    }
    const R* As = lds + buf * 2 * TILE;
    tile_mma<R, true>(acc1, As, As + TILE, qr, qc);
    if constexpr (TWO) tile_mma<R, true>(acc2, As, As, qr, qc);
    if constexpr (TAG) {
      if (more) {
        const bool ga = tagged_tile_take(ma, seq, ra);
        const bool gb = tagged_tile_take(mb, seq, rb);
        if (!(ga && gb)) {
          const uint64_t* ta = tile_slots(tagbase, T, tile_index(IA, K + 1, T));
          const uint64_t* tb = tile_slots(tagbase, T, tile_index(IB, K + 1, T));
          bool w = ga || tagged_watch(ta, seq, sync, status);
          w = (gb || tagged_watch(tb, seq, sync, status)) && w;
          ok = w && tagged_tile_fetch2(ta, tb, seq, ra, rb, sync, status) && ok;
        }
      }
    }
    if (more) {
      R* nxt = lds + (buf ^ 1) * 2 * TILE;
      tile_stash<R>(ra, nxt);
      tile_stash<R>(rb, nxt + TILE);
    }
    __syncthreads();
    buf ^= 1;
  }
  if constexpr (TAG) ok = __syncthreads_and(ok) != 0;
  return ok;
}

template <typename R>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_cholesky(
    const R* __restrict__ Hc, int64_t ld, int T, const double* __restrict__ mu_dev, double mu_host,
    const double* __restrict__ gvec, double* __restrict__ yvec, R* __restrict__ Lt,
    R* __restrict__ Linv, void* part_raw, uint32_t seq, SyncArea* sync, uint32_t* flags,
    uint32_t* yflags, int32_t* status) {
  constexpr int STR = Mfma<R>::STR;
  constexpr int TILE = 64 * STR;
  using acc_t = typename Mfma<R>::acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);            // 4 tiles
  __shared__ __align__(16) R rdiag[64];
  __shared__ double s_vec[64];
  __shared__ double s_red[kThreads];
  const int tid = threadIdx.x, wv = tid >> 6;
  const int qr = wv >> 1, qc = wv & 1;
  const double mu = mu_dev ? *mu_dev : mu_host;
  const uint32_t ntasks = chol_tasks(T);
  const uint32_t ntile_flags = (uint32_t)(T * (T + 1) / 2);
  uint32_t* daflags = flags + ntile_flags;
  // FP64: raw per-thread layout of one accumulator tile, thread tid owns 16 values (published
  // with a flag); FP32: tagged messages
  R* part = reinterpret_cast<R*>(part_raw);
  auto part_ptr = [&](int s, int which) { return part + ((int64_t)s * 2 + which) * 4096 + tid * 16; };

  for (;;) {
    const uint32_t t = claim(sync);
    if (t >= ntasks) break;
    int kind, I, J;
    decode_task(t, T, kind, I, J);
    bool ok = true;

    if (kind == TASK_DW) {
      R* Abuf = lds;
      R* Xprev = lds + TILE;
      R* Xcur = lds + 2 * TILE;
      R* Lbuf = lds + 3 * TILE;
      zero_upper_blocks<R>(Xprev);
      zero_upper_blocks<R>(Xcur);
      uint64_t mda[16], mdd[16];
      if constexpr (sizeof(R) == 4) tagged_issue16(tagged_slots(part_raw, 0, 0), mda);
      for (int st = 0; st < T; ++st) {
        // Steps 0 and 1 start from H; later steps from the two look-ahead tiles (H already
        // added).  In FP32 the subdiagonal tile's loads were issued before the previous step's
        // stores; the diagonal tile's 16 loads are issued here on every step (the slots of
        // steps 0 and 1 exist and go unused), after any H loads, so that the in-order
        // memory-counter waits leave them in flight over the subdiagonal product and the
        // diagonal update, which need only the subdiagonal tile.
        acc_t accd[2][2], accs[2][2];
        if (st < 2) {
          acc_load_h<R>(accd, Hc, ld, st, st, mu, qr, qc);
          if (st == 1) acc_load_h<R>(accs, Hc, ld, st, st - 1, 0.0, qr, qc);
        }
        if constexpr (sizeof(R) == 4) tagged_issue16(tagged_slots(part_raw, st, 1), mdd);
        if (st >= 1) {
          if (st >= 2) {
            if constexpr (sizeof(R) == 4) {
              if (ok && !tagged_take16(mda, seq, accs))
                ok = tagged_poll16(tagged_slots(part_raw, st, 0), seq, accs, sync, status);
            } else {
              if (ok) ok = wait_flag(daflags + st, sync, status);
              if (ok) ok = wait_flag(daflags + T + st, sync, status);
              const R* ps = part_ptr(st, 0);
              const R* pd = part_ptr(st, 1);
#pragma unroll
              for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                  for (int v = 0; v < 4; ++v) {
                    accs[bi][bj][v] = ps[(bi * 2 + bj) * 4 + v];
                    accd[bi][bj][v] = pd[(bi * 2 + bj) * 4 + v];
                  }
            }
          }
          acc_to_lds<R>(accs, Abuf, qr, qc);
          __syncthreads();
          acc_t ls[2][2];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) ls[bi][bj] = acc_t{0, 0, 0, 0};
          tile_mma<R, false>(ls, Abuf, Xprev, qr, qc);      // L_{s,s-1} = A X_{s-1}^T
          // FP32: the tagged copy, which the waiting tasks read, is stored before the plain one
          if constexpr (sizeof(R) == 4) {
            acc_to_lds<R>(ls, Lbuf, qr, qc);
            __syncthreads();
            tagged_put_lds(tile_slots(part_raw, T, tile_index(st, st - 1, T)), seq, Lbuf);
            acc_to_global<R>(ls, Lt + (int64_t)tile_index(st, st - 1, T) * 4096, qr, qc);
          } else {
            acc_to_global<R>(ls, Lt + (int64_t)tile_index(st, st - 1, T) * 4096, qr, qc);
            acc_to_lds<R>(ls, Lbuf, qr, qc);
            publish(flags + tile_index(st, st - 1, T));
          }
          __syncthreads();
          if (sizeof(R) == 4 && st >= 2) {
            // the diagonal update runs from zero and the diagonal look-ahead tile is added
            // after it, so its loads are waited for only here
            acc_t upd[2][2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj) upd[bi][bj] = acc_t{0, 0, 0, 0};
            tile_mma<R, true>(upd, Lbuf, Lbuf, qr, qc);
            if constexpr (sizeof(R) == 4) {
              if (ok && !tagged_take16(mdd, seq, accd))
                ok = tagged_poll16(tagged_slots(part_raw, st, 1), seq, accd, sync, status);
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) accd[bi][bj][v] += upd[bi][bj][v];
          } else {
            tile_mma<R, true>(accd, Lbuf, Lbuf, qr, qc);
          }
          __syncthreads();
        }
        acc_to_lds<R>(accd, Abuf, qr, qc);
        __syncthreads();
        const int bad = cholinv_tile<R>(Abuf, Xcur, rdiag);
        if (bad && tid == 0 && status) atomicOr(status, 1);
        R* dstX = Linv + (int64_t)st * 4096;
        if constexpr (sizeof(R) == 4) {
          // The next step's subdiagonal look-ahead tile is normally published by now: its
          // loads go out before this step's stores, so the wait for them at the next step
          // does not cover the stores (the vector-memory counter is in order).  Then the
          // tagged copy of the inverse (slot 4095, which waiting tasks watch, is among the
          // last stores) and the plain one.
          tagged_issue16(tagged_slots(part_raw, st + 1 < T ? st + 1 : T - 1, 0), mda);
          tagged_put_lds(tile_slots(part_raw, T, tile_index(st, st, T)), seq, Xcur);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int e4 = 4 * (tid + kThreads * k);
            *reinterpret_cast<f32x4*>(dstX + e4) =
                *reinterpret_cast<const f32x4*>(Xcur + (e4 >> 6) * STR + (e4 & 63));
          }
          __syncthreads();
        } else {
          for (int e = tid; e < 4096; e += kThreads) dstX[e] = Xcur[(e >> 6) * STR + (e & 63)];
          publish(flags + tile_index(st, st, T));
        }
        __syncthreads();
        R* tmp = Xprev;
        Xprev = Xcur;
        Xcur = tmp;
      }
    } else if (kind == TASK_DA || kind == TASK_DD) {
      // one of the worker's two look-ahead tiles for step s: the subdiagonal one
      // (DA, -sum_{K<s-1} L_sK L_{s-1,K}^T + H_{s,s-1}) or the diagonal one
      // (DD, -sum_{K<s-1} L_sK L_sK^T + H_ss + mu I), each a task of its own so that each runs
      // one product per K
      const int s = I, which = kind == TASK_DA ? 0 : 1;
      acc_t accp[2][2], dummy[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) accp[bi][bj] = acc_t{0, 0, 0, 0};
      // the H tile (with the damping on the diagonal) is loaded before the products and added
      // after them, off the worker's path; the sum rounds as the worker's own
      // (H + mu I) + partial
      acc_t hp[2][2];
      acc_load_h<R>(hp, Hc, ld, s, which ? s : s - 1, which ? mu : 0.0, qr, qc);
      ok = accumulate<R, false>(accp, dummy, Lt, T, s, which ? s : s - 1, s - 1, lds, sync, flags,
                                status, qr, qc, part_raw, seq);
      {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) accp[bi][bj][v] += hp[bi][bj][v];
      }
      if constexpr (sizeof(R) == 4) {
        tagged_put16(tagged_slots(part_raw, s, which), seq, accp);
        __syncthreads();
      } else {
        R* pp = part_ptr(s, which);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) pp[(bi * 2 + bj) * 4 + v] = accp[bi][bj][v];
        publish(daflags + which * T + s);
        __syncthreads();
      }
    } else if (kind == TASK_R) {
      acc_t acc[2][2], dummy[2][2];
      acc_load_h<R>(acc, Hc, ld, I, J, 0.0, qr, qc);
      ok = accumulate<R, false>(acc, dummy, Lt, T, I, J, J, lds, sync, flags, status, qr, qc,
                                part_raw, seq);
      acc_to_lds<R>(acc, lds, qr, qc);
      if constexpr (sizeof(R) == 4) {
        TileRegs<R> xr;
        const uint64_t* tx = tile_slots(part_raw, T, tile_index(J, J, T));
        // the tile two below the diagonal feeds the next look-ahead tasks: it polls the inverse
        // whole (one round trip sooner); the others watch one slot first
        const bool g = (I == J + 2 || tagged_watch(tx, seq, sync, status)) &&
                       tagged_tile_fetch(tx, seq, xr, sync, status);
        ok = __syncthreads_and(ok && g) != 0;
        tile_stash<R>(xr, lds + TILE);
      } else {
        if (ok) ok = wait_flag(flags + tile_index(J, J, T), sync, status);
        tile_to_lds<R>(Linv + (int64_t)J * 4096, lds + TILE);
      }
      __syncthreads();
      acc_t out[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) out[bi][bj] = acc_t{0, 0, 0, 0};
      tile_mma<R, false>(out, lds, lds + TILE, qr, qc);
      if constexpr (sizeof(R) == 4) {
        acc_to_lds<R>(out, lds + 2 * TILE, qr, qc);      // tile 2 is free after the accumulation
        __syncthreads();
        tagged_put_lds(tile_slots(part_raw, T, tile_index(I, J, T)), seq, lds + 2 * TILE);
        acc_to_global<R>(out, Lt + (int64_t)tile_index(I, J, T) * 4096, qr, qc);
        __syncthreads();
      } else {
        acc_to_global<R>(out, Lt + (int64_t)tile_index(I, J, T) * 4096, qr, qc);
        publish(flags + tile_index(I, J, T));
      }
      __syncthreads();
    } else if (kind == TASK_Y && gvec) {
      // y_J = X_JJ (g_J - sum_{K<J} L_JK y_K), FP64 accumulation.  FP32: the blocks y_K come
      // as messages and L_{J,J-1}, X_J from the worker's tagged copies, so only the flags of
      // the other factor tiles are waited on (one acquire for the prefix already set)
      const int r = tid & 63, pt = tid >> 6;
      double acc = 0.0;
      float iv[16];
      if constexpr (sizeof(R) == 4) {
        uint64_t* ymsg = y_slots(part_raw, T);
        bool g = true;
        for (int K = 0; K < J; ++K) {
          float lv[16];
          double yk[16];
          g = tagged_get16(tile_slots(part_raw, T, tile_index(J, K, T)), seq,
                           [&](int c) { return slot_of(r * 64 + pt * 16 + c); }, lv, sync, status) && g;
          g = msg_get16(ymsg + 64 * K + pt * 16, [](int c) { return c; }, yk, sync, status) && g;
#pragma unroll
          for (int c = 0; c < 16; ++c) acc = fma((double)lv[c], yk[c], acc);
        }
        g = tagged_get16(tile_slots(part_raw, T, tile_index(J, J, T)), seq,
                         [&](int c) { return slot_of(r * 64 + pt * 16 + c); }, iv, sync, status) && g;
        ok = __syncthreads_and(g) != 0;
      } else {
        for (int K = 0; K < J && ok; ++K) {
          ok = wait_flag(flags + tile_index(J, K, T), sync, status);
          if (ok) ok = wait_flag(yflags + K, sync, status);
          const R* tile = Lt + (int64_t)tile_index(J, K, T) * 4096 + r * 64 + pt * 16;
          const double* yv = yvec + 64 * K + pt * 16;
#pragma unroll
          for (int c = 0; c < 16; ++c) acc = fma((double)tile[c], yv[c], acc);
        }
      }
      s_red[tid] = acc;
      __syncthreads();
      if (tid < 64)
        s_vec[tid] = gvec[64 * J + tid] - (((s_red[tid] + s_red[tid + 64]) + s_red[tid + 128]) + s_red[tid + 192]);
      double y = 0.0;
      if constexpr (sizeof(R) == 4) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) y = fma((double)iv[c], s_vec[pt * 16 + c], y);
      } else {
        if (ok) ok = wait_flag(flags + tile_index(J, J, T), sync, status);
        const R* inv = Linv + (int64_t)J * 4096 + r * 64 + pt * 16;
#pragma unroll
        for (int c = 0; c < 16; ++c) y = fma((double)inv[c], s_vec[pt * 16 + c], y);
      }
      s_red[tid] = y;
      __syncthreads();
      if (tid < 64) {
        const double yj = ((s_red[tid] + s_red[tid + 64]) + s_red[tid + 128]) + s_red[tid + 192];
        yvec[64 * J + tid] = yj;
        if constexpr (sizeof(R) == 4) msg_put(y_slots(part_raw, T) + 64 * J + tid, yj);
      }
      if constexpr (sizeof(R) != 4) publish(yflags + J);
      __syncthreads();
    }
  }
  // FP32: the last workgroup out also restores kEmpty in the y messages
  exit_and_reset(sync, flags, (int)(ntile_flags + 2u * (uint32_t)T), yflags, yflags ? T : 0,
                 sizeof(R) == 4 ? y_slots(part_raw, T) : nullptr, sizeof(R) == 4 ? 64 * T : 0);
}

// ---------------------------------------------------------------------------------------
// Triangular solves on the tile-packed factor.  Thread layout inside a 64-row block:
// r = tid & 63 (row or column of the tile), part = tid >> 6 (a quarter of the other index).
// ---------------------------------------------------------------------------------------

// Gate: 0 = always run, 1 = skip if the factorisation failed or an earlier wait of the
// solve timed out, 2 = also skip once the refinement has converged.
__device__ __forceinline__ bool gated(const LMState* lm, int gate) {
  if (!lm || gate == 0) return false;
  if (lm->notpd || lm->timeout) return true;
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

// Triangular solves x = L^{-1} b (forward) and x = L^{-T} b (backward) on the tile-packed
// factor, with the inverses X_II of the diagonal tiles:
//   forward:  x_I = X_II (b_I - sum_{K<I} L_IK x_K),        blocks I = 0, 1, ..., T-1
//   backward: x_I = X_II^T (b_I - sum_{K>I} L_KI^T x_K),    blocks I = T-1, ..., 0
// Ticket 0 makes its workgroup the chain worker: it walks the blocks in solve order and
// applies the D-1 nearest blocks itself, so it never waits on another workgroup for them.  It
// applies them by columns: in step q it reads x of the previous block once from LDS and adds
// its products with the D-1 tiles below it into per-lane partial sums of the next D-1 blocks,
// the first of which is then complete.  The other workgroups (helpers, one per block from
// solve position D on) accumulate the contributions of all blocks at distance >= D as their
// solutions appear and hand the 64-entry partial sum to the worker, which has D-1 steps of
// slack (D = chain_d<R> = 3: the worker streams D tiles per step through its one compute
// unit, so a larger D slows every step, and a smaller one leaves the hand-off too little
// slack).  In the worker the four 16-column parts of a row sit in adjacent lanes of one
// wave, so a row sum is two DPP exchanges in a fixed order and a step needs two workgroup
// barriers.
// Hand-offs carry the data itself: solution blocks and partial sums travel through two
// message arrays written and read with agent-scope relaxed 64-bit atomics, and a slot that
// still holds kEmpty (a signalling-NaN payload that no arithmetic result carries) is not
// ready yet.  So there is no fence or flag on the chain.  The worker fetches the partial sum
// of a block a step ahead; a helper polls the solution blocks it waits for with one wave, one
// entry per lane, which keeps the polling off most of the lines the worker writes.  The last
// workgroup out restores kEmpty in both arrays.
template <typename R>
constexpr int chain_d() { return 3; }
// Register slots of the chain worker's operands (prefetch depth + 1): three in FP32, two in
// FP64, where the operands take twice the registers.
template <typename R>
constexpr int trsv_slots() { return sizeof(R) == 4 ? 3 : 2; }

// Lane exchange inside quads of lanes by DPP quad permutes (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// (p0 + p1) + (p2 + p3) of the four lanes of a quad, bitwise equal in all four.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_quad<0xB1>(v);      // quad_perm [1,0,3,2]: partner lane ^ 1
  return v + dpp_quad<0x4E>(v);  // quad_perm [2,3,0,1]: partner lane ^ 2
}
template <bool FWD>
__device__ __forceinline__ int solve_block(int T, int q) { return FWD ? q : T - 1 - q; }

// Solve layout of the tiles the solves read (k_transpose_tiles writes it, for the factor and
// inverse tiles in place and for their transposed copies): the 16-byte chunk j of (row r,
// columns 16 p ..) sits at chunk j * 256 + tl(r, p), with tl(r, p) = 64 (r / 16) + 4 (r % 16)
// + p the thread of the solve's chain worker that reads it, so that each load instruction of
// the worker's waves reads 1 KB of contiguous memory.
__device__ __forceinline__ int solve_tl(int r, int p) { return 64 * (r >> 4) + 4 * (r & 15) + p; }
template <typename R>
__device__ __forceinline__ void load16_solve(const R* __restrict__ tile, int r, int p, R (&v)[16]) {
  constexpr int V = 16 / (int)sizeof(R);
  const int tl = solve_tl(r, p);
  if constexpr (sizeof(R) == 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 t = *reinterpret_cast<const f32x4*>(tile + (j * kThreads + tl) * V);
      v[4 * j] = t[0];
      v[4 * j + 1] = t[1];
      v[4 * j + 2] = t[2];
      v[4 * j + 3] = t[3];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const f64x2 t = *reinterpret_cast<const f64x2*>(tile + (j * kThreads + tl) * V);
      v[2 * j] = t[0];
      v[2 * j + 1] = t[1];
    }
  }
}

// Tile coupling block I to block K (K before I in solve order), row r, columns 16 part ..:
// forward, row r of L_IK from the factor; backward, column r of L_KI, which is row r of the
// transposed tile, from the transposed copy (L is then the transposed factor); both in the
// solve layout.
template <typename R, bool FWD>
__device__ __forceinline__ void load_coupling(const R* __restrict__ L, int T, int I, int K,
                                              int rc, int part, R (&v)[16]) {
  load16_solve<R>(L + (int64_t)(FWD ? tile_index(I, K, T) : tile_index(K, I, T)) * 4096, rc, part, v);
}

// Row r, columns 16 part .. of X_II (forward) or of X_II^T (backward; Linv is then the
// transposed copy of the inverses).
template <typename R>
__device__ __forceinline__ void load_inverse(const R* __restrict__ Linv, int I, int rc, int part,
                                             R (&v)[16]) {
  load16_solve<R>(Linv + (int64_t)I * 4096, rc, part, v);
}

// Leave the solve: the last workgroup out restores kEmpty in the message arrays and clears
// the counters.
__device__ void trsv_exit(SyncArea* sync, uint64_t* psum, uint64_t* xpub, int n) {
  __shared__ int s_last;
  __threadfence();      // this workgroup's message stores land before it is counted out
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&sync->exited, 1u) == gridDim.x - 1);
  __syncthreads();
  if (s_last) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      __hip_atomic_store(psum + i, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(xpub + i, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
      sync->ticket = 0u;
      sync->exited = 0u;
      sync->abort = 0u;
    }
    __threadfence();
  }
}

// One wave per SIMD: the worker's prefetched tiles then have registers of their own, so no
// register that a prefetch is still filling gets reused (which would stall the chain for a
// full memory latency).
template <typename R, bool FWD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trsv(
    const R* __restrict__ Lt, const R* __restrict__ Linv, int T, const double* __restrict__ b,
    double* __restrict__ x, double* __restrict__ acc_out, uint64_t* psum, uint64_t* xpub,
    SyncArea* sync, int32_t* status, const LMState* __restrict__ lm, int gate) {
  __shared__ double sh[kThreads];
  __shared__ double s_vec[64];
  constexpr int D = chain_d<R>();
  __shared__ double s_y[2][64];   // the last two solution blocks
  __shared__ double sxb[2][64];   // a helper's two polled solution blocks
  // a gated launch touches nothing (counters and message slots stay as the last solve left
  // them), so its workgroups just leave
  if (gated(lm, gate)) return;
  const int tid = threadIdx.x, rc = tid & 63, part = tid >> 6;
  const uint32_t ntasks = 1u + (uint32_t)(T > D ? T - D : 0);
  for (;;) {
    const uint32_t t = claim(sync);
    if (t >= ntasks) break;
    if (t == 0) {
      // Chain worker.  Operands of a position (the row parts of X_II and of the D-1 coupling
      // tiles, the right-hand side and the accumulation target) sit in one of NS register
      // slots, filled PF = NS-1 steps ahead at the start of a step, so a tile fetch has PF
      // whole steps to arrive.  In FP32 the partial-sum message of the next position is
      // fetched in the middle of a step, one step ahead (two ahead it was usually not yet
      // published and the step polled for it), and before the tile loads issued there, so
      // its wait covers none of them (the vector-memory counter is in order); FP64 keeps it
      // two steps ahead.  Fetches are unconditional with
      // positions clamped into range (values fetched for a position that does not exist are
      // never used): a conditional load would make the wave wait for it at the join.  The
      // step loop is unrolled by NS, so every slot is a fixed set of registers.
      // Lane layout: row wr = 16 * wave + lane / 4, part wp = lane % 4.
      constexpr int NS = trsv_slots<R>(), PF = NS - 1;
      const int wr = 16 * (tid >> 6) + ((tid & 63) >> 2), wp = tid & 3;
      R inv[NS][16], nb[NS][D - 1][16];
      double cacc[D - 1];
#pragma unroll
      for (int d = 0; d < D - 1; ++d) cacc[d] = 0.0;
      double bq[NS], aq[NS];
      uint64_t mq[NS];
      const double* ap = acc_out ? acc_out : b;
      // step p applies y_{p-1} to blocks p .. p+D-2: the column tiles C(p+j, p-1)
      auto fetch = [&](auto slot, int p) {
        constexpr int S = decltype(slot)::value;
        const int pc = p < T ? p : T - 1;
        const int In = solve_block<FWD>(T, pc);
        const int pk = pc >= 1 ? pc - 1 : 0;
#pragma unroll
        for (int d = 0; d < D - 1; ++d)
          load_coupling<R, FWD>(Lt, T, solve_block<FWD>(T, pc + d < T ? pc + d : T - 1),
                                solve_block<FWD>(T, pk), wr, wp, nb[S][d]);
        load_inverse<R>(Linv, In, wr, wp, inv[S]);
        bq[S] = b[64 * In + wr];
        aq[S] = ap[64 * In + wr];
      };
#pragma unroll
      for (int s = 0; s < NS; ++s) mq[s] = kEmpty;
      if constexpr (NS == 3) {
        fetch(std::integral_constant<int, 0>{}, 0);
        fetch(std::integral_constant<int, 1>{}, 1);
      } else {
        fetch(std::integral_constant<int, 0>{}, 0);
      }
      auto step = [&](auto slot, int q) {
        constexpr int S = decltype(slot)::value;
        // FP64 (two slots): the operands of the next step are fetched here, a whole step ahead
        if constexpr (NS == 2) fetch(std::integral_constant<int, (S + PF) % NS>{}, q + PF);
        const int I = solve_block<FWD>(T, q);
        double pv = 0.0;
        if (q >= D) {
          uint64_t mm = mq[S];
          if (mm == kEmpty) mm = msg_wait(psum + 64 * I + wr, sync, status);
          pv = __longlong_as_double((long long)mm);
        }
        // y_{q-1}, read once, goes into the per-lane partial sums of blocks q .. q+D-2; the
        // first of them is then complete
        if (q >= 1) {
          const double* ys = s_y[(q - 1) & 1] + wp * 16;
#pragma unroll
          for (int d = 0; d < D - 1; ++d) {
            double c2[2] = {0.0, 0.0};
#pragma unroll
            for (int u = 0; u < 16; ++u) c2[u & 1] = fma((double)nb[S][d][u], ys[u], c2[u & 1]);
            cacc[d] += c2[0] + c2[1];
          }
        }
        const double sv = bq[S] - pv - quad_sum(cacc[0]);
#pragma unroll
        for (int d = 0; d + 1 < D - 1; ++d) cacc[d] = cacc[d + 1];
        cacc[D - 2] = 0.0;
        if (wp == 0) s_vec[wr] = sv;
        __syncthreads();
        if constexpr (NS == 3) {
          // FP32 (three slots): the next block's partial sum is fetched here, one step ahead,
          // and then the operands of the step two ahead; the partial-sum load is older than
          // those tile loads, so the in-order memory-counter wait for it at the next step does
          // not cover them
          mq[(S + 1) % NS] = msg_get(psum + 64 * solve_block<FWD>(T, q + 1 < T ? q + 1 : T - 1) + wr);
          fetch(std::integral_constant<int, (S + PF) % NS>{}, q + PF);
        }
        double y4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 16; ++u) y4[u & 3] = fma((double)inv[S][u], s_vec[wp * 16 + u], y4[u & 3]);
        // FP64: the partial sum two steps ahead (one step ahead measured 1 % slower here)
        if constexpr (NS == 2)
          mq[(S + 2) % NS] = msg_get(psum + 64 * solve_block<FWD>(T, q + 2 < T ? q + 2 : T - 1) + wr);
        const double xi = quad_sum((y4[0] + y4[1]) + (y4[2] + y4[3]));
        if (wp == 0) {
          x[64 * I + wr] = xi;
          s_y[q & 1][wr] = xi;
          msg_put(xpub + 64 * I + wr, xi);
          if (acc_out) acc_out[64 * I + wr] = aq[S] + xi;
        }
        __syncthreads();
      };
      // whole groups of NS steps in the loop (no conditional step inside it, so no path
      // reaches the back-edge with a slot's fetch unconsumed), the remainder after it
      int q = 0;
      for (; q + NS <= T; q += NS) {
        step(std::integral_constant<int, 0>{}, q);
        step(std::integral_constant<int, 1>{}, q + 1);
        if constexpr (NS == 3) step(std::integral_constant<int, 2 % NS>{}, q + 2);
      }
      if (q < T) step(std::integral_constant<int, 0>{}, q);
      if constexpr (NS == 3) {
        if (q + 1 < T) step(std::integral_constant<int, 1>{}, q + 1);
      }
    } else {
      // helper for the block at solve position q = t + D - 1: contributions of positions
      // 0 .. q-D, two solution blocks polled at a time by one wave
      const int q = (int)t + D - 1;
      const int I = solve_block<FWD>(T, q);
      const int last = q - D;
      R c0[16], c1[16], n0[16], n1[16];
      // unconditional prefetches with clamped positions, as in the worker
      load_coupling<R, FWD>(Lt, T, I, solve_block<FWD>(T, 0), rc, part, n0);
      load_coupling<R, FWD>(Lt, T, I, solve_block<FWD>(T, last >= 1 ? 1 : 0), rc, part, n1);
      double acc = 0.0;
      bool live = true;
      for (int k0 = 0; k0 <= last; k0 += 2) {
        const bool two = k0 + 1 <= last;
        const int K0 = solve_block<FWD>(T, k0), K1 = solve_block<FWD>(T, two ? k0 + 1 : k0);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          c0[u] = n0[u];
          c1[u] = n1[u];
        }
        // next pair's tiles in flight while this pair's solutions are polled
        load_coupling<R, FWD>(Lt, T, I, solve_block<FWD>(T, k0 + 2 <= last ? k0 + 2 : last), rc, part, n0);
        load_coupling<R, FWD>(Lt, T, I, solve_block<FWD>(T, k0 + 3 <= last ? k0 + 3 : last), rc, part, n1);
        double x0[16], x1[16];
        uint32_t spins = 0;
        for (;;) {
          // wave 0 polls both blocks whole (one entry per lane and block, one round trip per
          // poll) and leaves them in LDS for the other waves
          bool miss = false;
          if (tid < 64) {
            const uint64_t m0 = msg_get(xpub + 64 * K0 + tid);
            const uint64_t m1 = msg_get(xpub + 64 * K1 + tid);
            miss = (m0 == kEmpty) | (m1 == kEmpty);
            sxb[0][tid] = __longlong_as_double((long long)m0);
            sxb[1][tid] = __longlong_as_double((long long)m1);
          }
          if (!__syncthreads_or(miss) || !live) break;
          if (tid == 0) {
            if (__hip_atomic_load(&sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
              live = false;
            } else if (++spins > spin_limit(sync)) {
              __hip_atomic_store(&sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (status) atomicOr(status, 2);
              live = false;
            }
            sh[0] = live ? 1.0 : 0.0;
          }
          __syncthreads();
          live = sh[0] != 0.0;
          __syncthreads();
          __builtin_amdgcn_s_sleep(2);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          x0[u] = sxb[0][part * 16 + u];
          x1[u] = sxb[1][part * 16 + u];
        }
        __syncthreads();     // the next poll rewrites sxb
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma((double)c0[u], x0[u], acc);
        if (two) {
#pragma unroll
          for (int u = 0; u < 16; ++u) acc = fma((double)c1[u], x1[u], acc);
        }
      }
      const double sum = reduce4(acc, sh);
      if (tid < 64) msg_put(psum + 64 * I + tid, sum);
    }
  }
  trsv_exit(sync, psum, xpub, 64 * T);
}

// Refinement residual s = g - (H + mu I) d in FP64 from the FP32/FP64 column-major lower
// storage.  Pass 1: one workgroup per lower tile (I, J) writes its two contributions,
// H_IJ d_J (to rows of block I) and, off the diagonal, H_IJ^T d_I (to rows of block J), into
// per-tile partials; the tile is read once, along the storage's contiguous columns, and the
// transposed product takes it from LDS.  Pass 2: one workgroup per block row sums the
// partials in a fixed order, so the result is deterministic.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_symv_tiles(
    const R* __restrict__ Hc, int64_t ld, int T, const double* __restrict__ d,
    double* __restrict__ prow, double* __restrict__ pcol, const LMState* __restrict__ lm,
    int gate) {
  if (gated(lm, gate)) return;
  __shared__ double sd_col[64];   // d_J
  __shared__ double sd_row[64];   // d_I
  __shared__ double sh[kThreads];
  __shared__ R tt[64][65];        // off-diagonal tile, tt[c][r] = H[r][c] (padded: no conflicts)
  int I = 0, J = 0;
  {
    // blockIdx.x enumerates the lower tiles column-major
    uint32_t t = blockIdx.x, start = 0;
    int j = 0;
    while (start + (uint32_t)(T - j) <= t) {
      start += (uint32_t)(T - j);
      ++j;
    }
    J = j;
    I = j + (int)(t - start);
  }
  const int tid = threadIdx.x, r = tid & 63, part = tid >> 6;
  const R* base = Hc + (int64_t)(64 * J) * ld + 64 * I;   // element (row r, col c) at c*ld + r
  R hv[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    // rows of block I: H[r][c] for the 16 columns of this part; on the diagonal tile the
    // lower part only (the upper element mirrored)
    const int cl = part * 16 + cc;
    hv[cc] = (I != J || cl <= r) ? base[(int64_t)cl * ld + r] : base[(int64_t)r * ld + cl];
  }
  if (tid < 64) {
    sd_col[tid] = d[64 * J + tid];
    sd_row[tid] = d[64 * I + tid];
  }
  // off the diagonal the same elements serve the rows of block J through LDS (read per lane
  // from global memory, each load touched 64 lines)
  if (I != J) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) tt[part * 16 + cc][r] = hv[cc];
  }
  __syncthreads();
  // rows of block I: sum_c H[r][c] d_J[c]
  double a = 0.0;
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) a = fma((double)hv[cc], sd_col[part * 16 + cc], a);
  const double rowsum = reduce4(a, sh);
  if (tid < 64) prow[((int64_t)blockIdx.x) * 64 + tid] = rowsum;
  if (I != J) {
    // rows of block J: sum_r H[r][c] d_I[r], c = tid & 63, over the 16 rows of this part
    double b2 = 0.0;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr)
      b2 = fma((double)tt[r][part * 16 + rr], sd_row[part * 16 + rr], b2);
    const double colsum = reduce4(b2, sh);
    if (tid < 64) pcol[((int64_t)blockIdx.x) * 64 + tid] = colsum;
  }
}

// The last block row to arrive also closes the refinement step: ||s||^2 (a fixed-order sum of
// the per-block-row norms) against tol^2 ||g||^2 sets refine_done, else counts a step.  The
// norms travel as messages (slots holding kEmpty until written, restored by the closing
// workgroup), so no workgroup needs a fence, which would write back and invalidate the cache.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_symv_combine(
    int T, const double* __restrict__ mu_dev, const double* __restrict__ g,
    const double* __restrict__ d, const double* __restrict__ prow,
    const double* __restrict__ pcol, double* __restrict__ s, uint64_t* norms, LMState* lm,
    int gate, SyncArea* sync, double tol2) {
  if (gated(lm, gate)) return;
  __shared__ double sh[kThreads];
  const int B = blockIdx.x;           // block row
  const int tid = threadIdx.x, r = tid & 63, part = tid >> 6;
  // block row B gathers prow of tiles (B, J), J <= B, and pcol of tiles (I, B), I > B; each
  // thread takes every fourth one, eight loads in flight at a time, added in a fixed order
  double acc = 0.0;
  for (int J0 = part; J0 <= B; J0 += 32) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int J = J0 + 4 * u;
      const uint32_t ti = (uint32_t)(J * T - (J * (J - 1)) / 2 + (B - J));
      v[u] = J <= B ? prow[(int64_t)ti * 64 + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  const uint32_t cstart = (uint32_t)(B * T - (B * (B - 1)) / 2);
  for (int I0 = B + 1 + part; I0 < T; I0 += 32) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int I = I0 + 4 * u;
      v[u] = I < T ? pcol[((int64_t)cstart + (I - B)) * 64 + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  const double hd = reduce4(acc, sh);
  double sq = 0.0;
  if (tid < 64) {
    const int64_t row = 64 * (int64_t)B + r;
    const double si = g[row] - (*mu_dev) * d[row] - hd;
    s[row] = si;
    sq = si * si;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if (tid == 0) msg_put(norms + B, sq);
  }
  __shared__ int s_last;
  if (tid == 0) s_last = atomicAdd(&sync->exited, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  double v = 0.0;
  for (int i = tid; i < T; i += kThreads) {
    v += __longlong_as_double((long long)msg_wait(norms + i, sync, &lm->timeout));
    __hip_atomic_store(norms + i, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  sh[tid] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    if (sh[0] <= tol2 * lm->g_norm2) lm->refine_done = 1;
    else lm->refine_steps += 1;
    sync->exited = 0u;
  }
}

}  // namespace

template <typename R>
size_t chol_smem_bytes() {
  return 4 * 64 * Mfma<R>::STR * sizeof(R);
}

// Transpose every 64x64 tile of a packed array (ntiles tiles), one workgroup per tile through
// LDS so that both the reads and the writes are coalesced, and rewrite the source tile in
// place in the solve layout.  Skipped after a failed factorisation.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_transpose_tiles(R* __restrict__ src,
                                                              R* __restrict__ dst, int n1,
                                                              R* __restrict__ src2,
                                                              R* __restrict__ dst2,
                                                              const LMState* __restrict__ lm) {
  __shared__ R t[64][65];
  if (gated(lm, 1)) return;
  // blocks [0, n1) transpose tiles of the first array, the rest those of the second
  const bool first = (int)blockIdx.x < n1;
  const int64_t k = first ? blockIdx.x : blockIdx.x - n1;
  R* s = (first ? src : src2) + k * 4096;
  R* d = (first ? dst : dst2) + k * 4096;
  // all 16 loads of a thread are issued before the first LDS write (a loop that waited for
  // each load in turn ran the kernel at half the rate)
  R v[4096 / kThreads];
#pragma unroll
  for (int q = 0; q < 4096 / kThreads; ++q) v[q] = s[threadIdx.x + q * kThreads];
#pragma unroll
  for (int q = 0; q < 4096 / kThreads; ++q) {
    const int e = threadIdx.x + q * kThreads;
    t[e >> 6][e & 63] = v[q];
  }
  __syncthreads();
  // the destination in the solve layout (the backward solve's only operands), stored in
  // order: position pos holds element w of chunk pos / V
  constexpr int V = 16 / (int)sizeof(R);
#pragma unroll
  for (int q = 0; q < 4096 / kThreads; ++q) {
    const int pos = threadIdx.x + q * kThreads;
    const int chunk = pos / V, w = pos % V;
    const int j = chunk >> 8, tl = chunk & 255;
    const int r = 16 * (tl >> 6) + ((tl & 63) >> 2), c = 16 * (tl & 3) + V * j + w;
    d[pos] = t[c][r];
    s[pos] = t[r][c];      // in place: every load of the tile is done (barrier above)
  }
}

template <typename R>
hipError_t launch_transpose_tiles(R* src, R* dst, int ntiles, R* src2, R* dst2,
                                  int ntiles2, const LMState* lm, hipStream_t st) {
  if (ntiles + ntiles2 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_tiles<R>, dim3(ntiles + ntiles2), dim3(kThreads), 0, st, src,
                     dst, ntiles, src2, dst2, lm);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_cholesky(const R* Hc, int ld, int n_pad, const double* mu_dev, double mu_host,
                           const double* g, double* y, R* Lt, R* Linv, void* part,
                           uint32_t seq, SyncArea* sync, uint32_t* flags, uint32_t* yflags,
                           int32_t* status, hipStream_t st, int n_wg) {
  const int T = n_pad / 64;
  const int ntasks = (int)chol_tasks(T);
  // at least two workgroups: the diagonal worker and one for the other tasks
  int grid = n_wg < ntasks ? n_wg : ntasks;
  if (grid < 2) grid = 2;
  hipLaunchKernelGGL(k_cholesky<R>, dim3(grid), dim3(kThreads), chol_smem_bytes<R>(), st, Hc,
                     (int64_t)ld, T, mu_dev, mu_host, g, y, Lt, Linv, part, seq, sync, flags,
                     yflags, status);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_trsv(bool forward, const R* Lt, const R* Linv, int n_pad, const double* b,
                       double* x, double* acc_out, uint64_t* psum, uint64_t* xpub,
                       SyncArea* sync, int32_t* status, const LMState* lm, int gate,
                       hipStream_t st) {
  const int T = n_pad / 64;
  const int ntasks = 1 + (T > chain_d<R>() ? T - chain_d<R>() : 0);
  // at least two workgroups, so helpers exist beside the worker whatever the task count
  const int grid = ntasks < 2 ? 2 : (ntasks < 256 ? ntasks : 256);
  if (forward)
    hipLaunchKernelGGL((k_trsv<R, true>), dim3(grid), dim3(kThreads), 0, st, Lt, Linv, T, b, x,
                       acc_out, psum, xpub, sync, status, lm, gate);
  else
    hipLaunchKernelGGL((k_trsv<R, false>), dim3(grid), dim3(kThreads), 0, st, Lt, Linv, T, b, x,
                       acc_out, psum, xpub, sync, status, lm, gate);
  return hipGetLastError();
}

// Fill n 64-bit message slots with kEmpty (once, when the message arrays are created).
__global__ void k_fill_empty(uint64_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = kEmpty;
}
hipError_t launch_fill_empty(uint64_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_empty, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_refine_resid(const R* Hc, int ld, int n_pad, const double* mu_dev,
                               const double* g, const double* d, double* s, uint64_t* norms,
                               double* prow, double* pcol, LMState* lm, int gate,
                               SyncArea* sync, double tol2, hipStream_t st) {
  const int T = n_pad / 64;
  const int ntiles = T * (T + 1) / 2;
  hipLaunchKernelGGL(k_symv_tiles<R>, dim3(ntiles), dim3(kThreads), 0, st, Hc, (int64_t)ld, T, d,
                     prow, pcol, lm, gate);
  hipLaunchKernelGGL(k_symv_combine<R>, dim3(T), dim3(kThreads), 0, st, T, mu_dev, g, d, prow,
                     pcol, s, norms, lm, gate, sync, tol2);
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
  template hipError_t launch_cholesky<R>(const R*, int, int, const double*, double,             \
                                         const double*, double*, R*, R*, void*, uint32_t,      \
                                         SyncArea*, uint32_t*, uint32_t*, int32_t*,            \
                                         hipStream_t, int);                                    \
  template hipError_t launch_transpose_tiles<R>(R*, R*, int, R*, R*, int,          \
                                                const LMState*, hipStream_t);                  \
  template hipError_t launch_trsv<R>(bool, const R*, const R*, int, const double*, double*,    \
                                     double*, uint64_t*, uint64_t*, SyncArea*, int32_t*,       \
                                     const LMState*, int, hipStream_t);                        \
  template hipError_t launch_refine_resid<R>(const R*, int, int, const double*, const double*, \
                                             const double*, double*, uint64_t*, double*,        \
                                             double*, LMState*, int, SyncArea*, double,         \
                                             hipStream_t);
DDC_INST(float)
DDC_INST(double)
#undef DDC_INST

}  // namespace ddc
