// Alloc/do-all microbenchmark: objects {int32 id, float32 x, float32 v};
// each step updates every object, deletes every id % 3 == 0 and creates the
// same ids again.
#include "internal.hpp"

namespace dsoar {

namespace {

enum : uint32_t { kId = 0, kX = 1, kV = 2 };

struct MicroUpdate {
  static constexpr uint32_t kKind = 20;
  struct Args { uint32_t unused; };
  struct Pre { float x, v; };
  template <class H>
  static __device__ Pre load(const H& h, uint32_t type, uint32_t self, const Args&) {
    return {*field_ptr<float>(h, self, type, kX), *field_ptr<float>(h, self, type, kV)};
  }
  template <class H>
  static __device__ bool apply(const H& h, uint32_t type, uint32_t self, const Args&, const Pre& p) {
    *field_ptr<float>(h, self, type, kX) = __builtin_fmaf(0.01f, p.v, p.x);  // one rounding
    return false;
  }
};

struct MicroCull {
  static constexpr uint32_t kKind = 21;
  static constexpr uint32_t kMinWaves = 8;
  struct Args { uint32_t unused; };
  struct Pre { int32_t id; };
  template <class H>
  static __device__ Pre load(const H& h, uint32_t type, uint32_t self, const Args&) {
    return {*field_ptr<int32_t>(h, self, type, kId)};
  }
  static __device__ bool apply(const DevHeap&, uint32_t, uint32_t, const Args&, const Pre& p) {
    return p.id % 3 == 0;
  }
};

// Object i gets id = id_mul * i and the i-th input values.  A wavefront
// creates per_lane * 64 consecutive objects, lane l those at offsets l,
// l + 64, ... (coalesced input reads), as one request of up to per_lane
// objects per lane: a wavefront asking for four blocks' worth takes them with
// one atomic on the free bitmap.  Large creations use four per lane (fewer,
// longer requests); below kCreateWideMin objects one per lane keeps enough
// wavefronts in flight to hide the allocation latency.
constexpr uint32_t kCreatePerLane = 4;
constexpr uint32_t kCreateWideMin = 1u << 22;
constexpr uint32_t kCreateThreads = 256;

// Large creations are compiled for 8 wavefronts per SIMD (the allocation
// path's scalar registers leave room for 7 otherwise): their grids are many
// times the resident wavefronts, and more of them hide more of each
// request's chain of atomics.
template <uint32_t LG, bool kWide>
__global__ void __attribute__((amdgpu_waves_per_eu(kWide ? 8 : 1)))
micro_create_kernel(DevHeapW<LG> h, uint32_t type, uint32_t n, uint32_t per_lane, uint32_t id_mul, const float* xs,
                    const float* vs) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = (uint64_t)blockIdx.x * (kCreateThreads / 64) + (threadIdx.x >> 6);
  const uint64_t base = wave * (64u * per_lane) + lane;
  uint32_t k = 0;
  for (uint32_t j = 0; j < per_lane; ++j) k += base + j * 64u < n ? 1u : 0u;
  new_many(h, type, k, [&](uint32_t j, uint32_t o) {
    if (o == kNull) return;
    const uint32_t i = (uint32_t)(base + j * 64u);
    *field_ptr<int32_t>(h, o, type, kId) = (int32_t)(id_mul * i);
    *field_ptr<float>(h, o, type, kX) = xs[i];
    *field_ptr<float>(h, o, type, kV) = vs[i];
  });
}

bool micro_type_ok(const dsoar_heap* h, uint32_t type) {
  if (type >= h->desc.num_types) return false;
  const dsoar_type_layout& L = h->desc.types[type];
  return L.num_fields >= 3 && L.field_bytes[kId] == 4 && L.field_bytes[kX] == 4 && L.field_bytes[kV] == 4;
}

int launch_create(dsoar_heap* h, uint32_t type, uint32_t n, uint32_t id_mul, const float* xs, const float* vs,
                  hipStream_t s) {
  if (n == 0) return DSOAR_OK;
  const uint32_t per_lane = n >= kCreateWideMin ? kCreatePerLane : 1u;
  const uint64_t per_block = (uint64_t)kCreateThreads * per_lane;
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    const dim3 grid((uint32_t)((n + per_block - 1) / per_block));
    if (per_lane > 1)
      launch_timed(h, kKindMicroCreate, micro_create_kernel<kLG, true>, grid, dim3(kCreateThreads), s,
                   DevHeapW<kLG>(h->dev), type, n, per_lane, id_mul, xs, vs);
    else
      launch_timed(h, kKindMicroCreate, micro_create_kernel<kLG, false>, grid, dim3(kCreateThreads), s,
                   DevHeapW<kLG>(h->dev), type, n, per_lane, id_mul, xs, vs);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

}  // namespace

int micro_doall(dsoar_heap* h, uint32_t type, uint32_t method, uint32_t flags, hipStream_t s) {
  if (!micro_type_ok(h, type)) return DSOAR_ERR_INVALID_ARG;
  if (method == DSOAR_METHOD_MICRO_UPDATE) return launch_doall_tree<MicroUpdate>(h, type, {0}, flags, s);
  return launch_doall_tree<MicroCull>(h, type, {0}, flags, s);
}

}  // namespace dsoar

using namespace dsoar;

extern "C" {

int dsoar_micro_init(dsoar_heap* h, uint32_t type, uint32_t n, const float* x0_dev, const float* v0_dev,
                     void* stream) {
  if (!heap_ok(h) || !micro_type_ok(h, type) || (n && (!x0_dev || !v0_dev)) || n > (1u << 31))
    return DSOAR_ERR_INVALID_ARG;
  return launch_create(h, type, n, 1, x0_dev, v0_dev, (hipStream_t)stream);
}

int dsoar_micro_step(dsoar_heap* h, uint32_t type, uint32_t n_renew, const float* xs_dev, const float* vs_dev,
                     uint32_t flags, void* stream) {
  if (!heap_ok(h) || !micro_type_ok(h, type) || (n_renew && (!xs_dev || !vs_dev)) || n_renew > (1u << 30))
    return DSOAR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t base = flags & DSOAR_DO_PLAIN;
  int rc = launch_doall<MicroUpdate>(h, type, {0}, base, s);
  if (rc) return rc;
  // Update neither creates nor deletes, so the cull reuses its enumeration.
  rc = launch_doall<MicroCull>(h, type, {0}, base | DSOAR_DO_REUSE_ENUM, s);
  if (rc) return rc;
  return launch_create(h, type, n_renew, 3, xs_dev, vs_dev, s);
}

}  // extern "C"
