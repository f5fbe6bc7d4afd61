// Nagel-Schreckenberg traffic as objects on open single-lane roads (the
// paper's "traffic" application, Fig. 6; the rules are the model's published
// ones).  Car {cell, speed, next speed} objects live in the heap; the roads
// are a plain cell -> car handle array.  One step t is:
//   Decide (do-all over Car): on the state at the start of the step,
//     accelerate (v = min(v + 1, vmax)), brake to the empty cells ahead
//     (cells past the road's end count as empty), and dawdle (v -= 1 when
//     v > 0 with probability p_slow, drawn from hash(seed, 32, cell, t)).
//   Move (do-all over Car, same list): advance v cells; a car that passes the
//     road's last cell deletes itself.  Moves never collide: a car ends
//     before the old cell of the car ahead, so all handle writes are distinct.
//   Entry (one thread per road): a car enters an empty first cell at speed 0
//     with probability p_in, from hash(seed, 33, road, t); the last workgroup
//     of the entry kernel to finish advances t (the step index lives on the
//     device, so a captured step replays correctly).
#include <string.h>

#include <new>

#include "internal.hpp"

namespace dsoar {
namespace {

enum : uint32_t { kCar = 0 };
enum : uint32_t { kCellF = 0, kSpeed = 1, kNext = 2 };
constexpr int32_t kMaxSpeed = 8;
constexpr uint64_t kStreamSlow = 32, kStreamIn = 33;

// SplitMix64 output finaliser (Steele, Lea, Flood, OOPSLA 2014) and the
// workload hash built on it: mix(mix(mix(seed ^ stream * golden) ^ a) ^ b).
__device__ __forceinline__ uint64_t splitmix_final(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return splitmix_final(splitmix_final(splitmix_final(seed ^ (stream * 0x9E3779B97F4A7C15ull)) ^ a) ^ b);
}

struct Road {
  uint32_t* occ;   // cell -> car handle, kNull when empty
  uint32_t* step;  // [0]: index of the step in progress; [1]: entry workgroups done
  uint32_t roads, length;
  uint64_t seed;
  int32_t vmax;
  uint32_t p_slow24, p_in24;
};

template <class F, class H>
__device__ __forceinline__ F& car(const H& h, uint32_t self, uint32_t field) {
  return *field_ptr<F>(h, self, kCar, field);
}

struct Decide {
  static constexpr uint32_t kKind = 50;
  using Args = Road;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t c = car<uint32_t>(h, self, kCellF);
    const int32_t v0 = car<int32_t>(h, self, kSpeed);
    const uint32_t i = c % a.length;
    int32_t v = v0 + 1 < a.vmax ? v0 + 1 : a.vmax;
    // The cells ahead, all read together; past the road's end they are empty.
    uint32_t ahead[kMaxSpeed];
#pragma unroll
    for (int32_t k = 1; k <= kMaxSpeed; ++k)
      ahead[k - 1] = (k <= v && i + (uint32_t)k < a.length) ? a.occ[c + (uint32_t)k] : kNull;
    int32_t gap = 0;
#pragma unroll
    for (int32_t k = 1; k <= kMaxSpeed; ++k)
      if (gap == k - 1 && k <= v && ahead[k - 1] == kNull) gap = k;
    v = v < gap ? v : gap;
    const uint64_t hs = draw(a.seed, kStreamSlow, c, a.step[0]);
    if (v > 0 && (uint32_t)(hs >> 40) < a.p_slow24) --v;
    car<int32_t>(h, self, kNext) = v;
    return false;
  }
};

struct Drive {
  static constexpr uint32_t kKind = 51;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = Road;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const int32_t v = car<int32_t>(h, self, kNext);
    car<int32_t>(h, self, kSpeed) = v;
    if (v == 0) return false;
    const uint32_t c = car<uint32_t>(h, self, kCellF);
    a.occ[c] = kNull;
    if (c % a.length + (uint32_t)v >= a.length) return true;  // leaves the road
    a.occ[c + (uint32_t)v] = self;
    car<uint32_t>(h, self, kCellF) = c + (uint32_t)v;
    return false;
  }
};

// A car enters road r's empty first cell with probability p_in.  Then the
// step advances: each workgroup counts itself done after all its threads have
// used t, and the last one to do so stores t + 1 (and resets the count), so no
// thread of this launch can read the new value.
template <uint32_t LG>
__global__ void entry_kernel(DevHeapW<LG> h, Road a) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t t = a.step[0];
  if (r < a.roads) {
    const uint32_t q = r * a.length;
    const uint64_t hs = draw(a.seed, kStreamIn, r, t);
    const bool enter = a.occ[q] == kNull && (uint32_t)(hs >> 40) < a.p_in24;
    new_many(h, kCar, enter ? 1u : 0u, [&](uint32_t, uint32_t o) {
      if (o == kNull) return;
      car<uint32_t>(h, o, kCellF) = q;
      car<int32_t>(h, o, kSpeed) = 0;
      car<int32_t>(h, o, kNext) = 0;
      a.occ[q] = o;
    });
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(a.step + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(a.step + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.step[0] = t + 1;
    }
  }
}

// Initial state: a car in every cell whose speed is >= 0.
template <uint32_t LG>
__global__ void traffic_init_kernel(DevHeapW<LG> h, Road a, const int32_t* vel, uint32_t step0) {
  const uint64_t n = (uint64_t)a.roads * a.length;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) {
    a.step[0] = step0;
    a.step[1] = 0;
  }
  if (c >= n) return;
  a.occ[c] = kNull;
  const int32_t v = vel[c];
  new_many(h, kCar, v >= 0 ? 1u : 0u, [&](uint32_t, uint32_t o) {
    if (o == kNull) return;
    car<uint32_t>(h, o, kCellF) = c;
    car<int32_t>(h, o, kSpeed) = v;
    car<int32_t>(h, o, kNext) = v;
    a.occ[c] = o;
  });
}

__global__ void traffic_read_kernel(DevHeap h, Road a, int32_t* vel) {
  const uint64_t n = (uint64_t)a.roads * a.length;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t o = a.occ[c];
  vel[c] = o == kNull ? -1 : car<int32_t>(h, o, kSpeed);
}

bool traffic_heap_ok(const dsoar_heap* h) {
  if (h->desc.num_types < 1) return false;
  const dsoar_type_layout& L = h->desc.types[kCar];
  if (L.num_fields < 3) return false;
  for (uint32_t f = 0; f < 3; ++f)
    if (L.field_bytes[f] != 4) return false;
  return true;
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

struct dsoar_traffic {
  dsoar_heap* heap;
  Road a;
  StepGraphs graphs;
};

namespace {

int traffic_one_step(dsoar_traffic* t, uint32_t flags, hipStream_t st) {
  dsoar_heap* h = t->heap;
  const uint32_t base = flags & DSOAR_DO_PLAIN;
  int rc = launch_doall<Decide>(h, kCar, t->a, base, st);
  // Decide creates and deletes nothing: Drive reuses its list.
  if (!rc) rc = launch_doall<Drive>(h, kCar, t->a, base | DSOAR_DO_REUSE_ENUM, st);
  if (rc) return rc;
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(h, kKindTrafficEntry, entry_kernel<kLG>, dim3((t->a.roads + 255) / 256), dim3(256), st, DevHeapW<kLG>(h->dev), t->a);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

}  // namespace

extern "C" {

size_t dsoar_traffic_bytes(uint32_t roads, uint32_t length) {
  const uint64_t n = (uint64_t)roads * length;
  if (roads == 0 || length == 0 || n > (1ull << 30)) return 0;
  return (size_t)(256 + (n * 4 + 255) / 256 * 256);
}

int dsoar_traffic_create(dsoar_heap* heap, uint32_t roads, uint32_t length, const dsoar_traffic_rules* rules,
                         void* dev_mem, size_t dev_bytes, dsoar_traffic** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !traffic_heap_ok(heap) || !rules || !dev_mem || ((uintptr_t)dev_mem & 255u) ||
      rules->vmax < 1 || rules->vmax > kMaxSpeed || rules->p_slow24 > (1u << 24) || rules->p_in24 > (1u << 24))
    return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_traffic_bytes(roads, length);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_traffic* t = new (std::nothrow) dsoar_traffic;
  if (!t) return DSOAR_ERR_INVALID_ARG;
  memset(t, 0, sizeof(*t));
  t->heap = heap;
  uint8_t* b = (uint8_t*)dev_mem;
  t->a.step = (uint32_t*)b;
  t->a.occ = (uint32_t*)(b + 256);
  t->a.roads = roads;
  t->a.length = length;
  t->a.seed = rules->seed;
  t->a.vmax = rules->vmax;
  t->a.p_slow24 = rules->p_slow24;
  t->a.p_in24 = rules->p_in24;
  *out = t;
  return DSOAR_OK;
}

int dsoar_traffic_destroy(dsoar_traffic* t) {
  if (!t) return DSOAR_ERR_INVALID_ARG;
  step_graphs_clear(t->graphs);
  delete t;
  return DSOAR_OK;
}

int dsoar_traffic_init(dsoar_traffic* t, const int32_t* vel_dev, uint32_t step0, void* stream) {
  if (!t || !vel_dev) return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)t->a.roads * t->a.length;
  with_width(t->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(t->heap, kKindTrafficInit, traffic_init_kernel<kLG>, dim3((uint32_t)((n + 255) / 256)), dim3(256), (hipStream_t)stream,
                     DevHeapW<kLG>(t->heap->dev), t->a, vel_dev, step0);
  });
  DSOAR_LAUNCHED(t->heap);
  return DSOAR_OK;
}

int dsoar_traffic_step(dsoar_traffic* t, uint32_t steps, uint32_t flags, void* stream) {
  if (!t) return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  dsoar_heap* h = t->heap;
  if (flags & DSOAR_GRAPH) {
    if (flags & DSOAR_DO_PLAIN) return DSOAR_ERR_INVALID_ARG;
    return step_graphs_run(h, t->graphs, steps, st, [&](hipStream_t gs) { return traffic_one_step(t, 0, gs); });
  }
  for (uint32_t i = 0; i < steps; ++i) {
    const int rc = traffic_one_step(t, flags, st);
    if (rc) return rc;
  }
  return DSOAR_OK;
}

int dsoar_traffic_read(dsoar_traffic* t, int32_t* vel_dev, void* stream) {
  if (!t || !vel_dev) return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)t->a.roads * t->a.length;
  hipLaunchKernelGGL(traffic_read_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     t->heap->dev, t->a, vel_dev);
  DSOAR_LAUNCHED(t->heap);
  return DSOAR_OK;
}

}  // extern "C"
