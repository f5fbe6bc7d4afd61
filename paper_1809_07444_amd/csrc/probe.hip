// Measurement probes for the ceilings the heap runs against: agent-scope
// 64-bit atomic throughput (distinct and shared addresses), dependent atomic
// and load latency, and a plain streaming copy.  AMD publishes no atomic
// peak, so these measured rates are the reference the allocator is compared
// with.
#include "internal.hpp"

namespace dsoar {
namespace {

// mode 0: each wavefront's leader ORs its own word `iters` times (results unused).
// mode 1: same, each atomic depending on the previous one's result (latency).
// mode 2: every leader ORs word 0 (one contended address).
// mode 3: a chain of dependent agent-scope loads (latency).
__global__ void atomic_probe_kernel(uint64_t* buf, uint32_t words, uint32_t mode, uint32_t iters, uint64_t* sink) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (lane_id() != 0) return;
  uint64_t* p = buf + ((uint64_t)wave * 8) % words;  // one 64-byte line per wavefront
  uint64_t acc = 0;
  switch (mode) {
    case 0:
      for (uint32_t i = 0; i < iters; ++i)
        __hip_atomic_fetch_or(p, 1ull << (i & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    case 1:
      for (uint32_t i = 0; i < iters; ++i) {
        // The next address depends on the previous result (stays in the line).
        const uint64_t r = __hip_atomic_fetch_or(p + ((acc >> 62) & 1), 1ull << (i & 63), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        acc = r;
      }
      break;
    case 2:
      for (uint32_t i = 0; i < iters; ++i)
        __hip_atomic_fetch_or(buf, 1ull << (i & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    default: {
      uint64_t idx = ((uint64_t)wave * 8) % words;
      for (uint32_t i = 0; i < iters; ++i) {
        const uint64_t v = __hip_atomic_load(buf + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        idx = (idx + 8 + (v >> 63)) % words;
        acc += v;
      }
    }
  }
  if (acc == 0x5eedull) sink[0] = acc;  // keeps the chains live
}

// One 16-byte element per thread and no loop: every wavefront reads and
// writes 1 KiB once and exits.  On MI355X this keeps more requests in flight
// than grid-stride loops (about 6.2 TB/s against 4.6 TB/s for a 1 GiB copy).
__global__ void copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

extern "C" {

int dsoar_probe_atomics(void* buf_dev, uint32_t words, uint32_t mode, uint32_t iters, uint32_t waves,
                        void* stream) {
  if (!buf_dev || words < 16 || mode > 3 || waves == 0 || ((uintptr_t)buf_dev & 63u)) return DSOAR_ERR_INVALID_ARG;
  const uint32_t threads = 256;
  const uint64_t total = (uint64_t)waves * 64;
  hipLaunchKernelGGL(atomic_probe_kernel, dim3((uint32_t)((total + threads - 1) / threads)), dim3(threads), 0,
                     (hipStream_t)stream, (uint64_t*)buf_dev, words - 8, mode, iters, (uint64_t*)buf_dev + words - 8);
  return hipGetLastError() == hipSuccess ? DSOAR_OK : DSOAR_ERR_HIP;
}

int dsoar_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream) {
  if (!src_dev || !dst_dev || (bytes & 15) || ((uintptr_t)src_dev & 15) || ((uintptr_t)dst_dev & 15))
    return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = bytes / 16;
  const uint64_t grid = (n + 255) / 256;
  if (grid == 0) return DSOAR_OK;
  if (grid > 0x7FFFFFFFull) return DSOAR_ERR_INVALID_ARG;
  hipLaunchKernelGGL(copy_probe_kernel, dim3((uint32_t)grid), dim3(256), 0, (hipStream_t)stream,
                     (const uint4*)src_dev, (uint4*)dst_dev, n);
  return hipGetLastError() == hipSuccess ? DSOAR_OK : DSOAR_ERR_HIP;
}

}  // extern "C"
