// Fixed device scratch for the entry point that allocates nothing (ddc_residual_noalloc).
//
// ddc_residual keeps its per-block cost partials and the canonical baseline table in the
// context's workspace, which it grows with hipMalloc on demand.  Callers that cannot allocate
// (code under HIP graph capture, tight serving loops) get the same computation with those
// buffers in one file-scope device array instead.  Each device holds its own copy of the
// array for the life of the process; its address is looked up once per device when a
// context is created on it (with that device current), and host code only ever uses that
// looked-up address.  Every call on a device shares the array, so calls that overlap on one
// device race; each call rebuilds everything it reads from the array before reading it.
#include "common.h"

#include <mutex>

namespace ddc {
namespace {

constexpr size_t kTableBytes =
    (2 * (size_t)kNoAllocMaxBaselines * sizeof(int32_t) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kTableBytes + (size_t)kNoAllocMaxBlocks * sizeof(double) + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Canonical baseline table of N stations: baselines of station p (< q) start at
// p(2N - p - 1)/2, one workgroup per p.
__global__ void k_baseline_table(int N, int64_t B, int32_t* __restrict__ ant_p,
                                 int32_t* __restrict__ ant_q) {
  const int p = blockIdx.x;
  const int64_t start = (int64_t)p * (2 * N - p - 1) / 2;
  for (int q = p + 1 + threadIdx.x; q < N; q += blockDim.x) {
    const int64_t b = start + (q - p - 1);
    ant_p[b] = p;
    ant_q[b] = q;
  }
  (void)B;
}

}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

NoAllocScratch noalloc_scratch(int device) {
  NoAllocScratch s{};
  if (device < 0 || device >= kMaxDevices) return s;
  std::lock_guard<std::mutex> lk(g_mu);
  char* base = reinterpret_cast<char*>(g_ptr[device]);
  if (!base) return s;
  s.ant = reinterpret_cast<int32_t*>(base);
  s.parts = reinterpret_cast<double*>(base + kTableBytes);
  s.total = reinterpret_cast<double*>(base + kTableBytes + (size_t)kNoAllocMaxBlocks * sizeof(double));
  return s;
}

hipError_t launch_baseline_table(int N, int64_t B, int32_t* ant_p, int32_t* ant_q,
                                 hipStream_t st) {
  if (N < 2) return hipSuccess;
  hipLaunchKernelGGL(k_baseline_table, dim3(N - 1), dim3(256), 0, st, N, B, ant_p, ant_q);
  return hipGetLastError();
}

}  // namespace ddc
