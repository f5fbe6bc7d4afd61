// Merging bodies in the plane as objects (the paper's "collisions"
// application, Fig. 6b).  Body {x, y, vx, vy, ax, ay, m, id} objects live in
// the heap; dense per-id arrays hold what every body reads of every other:
// P[id] = {x, y, m, 0} (m = 0 once the body merged away), V[id] = {vx, vy} and
// T[id], the merge decision.  One step is six do-alls over the same
// enumeration (nothing is created, and only the last deletes):
//   Force:  a = sum over all ids j in increasing order of
//           m_j (p_j - p) / (r2 sqrt(r2)), r2 = |p_j - p|^2 + eps2
//           (j = this body and merged bodies add exactly 0)
//   Move:   v += dt a, p += dt v; publish P and V
//   Root:   a root has no live body of lower id within the merge radius
//   Target: a live non-root merges into the lowest-id root within the radius
//   Merge:  a root adds the mass, momentum and mass-weighted position of the
//           bodies merging into it, in increasing id order
//   Remove: merged bodies mark P dead and delete themselves
// Every float operation is single precision with one rounding (explicit
// fma; correctly rounded division and square root), in the same order as the
// sequential definition, so the results are bit-identical to it.
#include <string.h>

#include <new>

#include "internal.hpp"

namespace dsoar {
namespace {

enum : uint32_t { kBody = 0 };
enum : uint32_t { kX = 0, kY = 1, kVX = 2, kVY = 3, kAX = 4, kAY = 5, kM = 6, kId = 7 };
constexpr uint32_t kRoot = 0xFFFFFFFEu, kAlone = 0xFFFFFFFFu;

struct Bodies {
  float4* P;   // id -> {x, y, m, 0}
  float2* V;   // id -> {vx, vy}
  uint32_t* T; // id -> kRoot, kAlone or the id of the root it merges into
  uint32_t n;
  float dt, eps2, r2_merge;
};

template <class F, class H>
__device__ __forceinline__ F& fld(const H& h, uint32_t self, uint32_t f) {
  return *field_ptr<F>(h, self, kBody, f);
}

// Entry k of a wavefront-wide chunk: lane k's value, read by every lane.
__device__ __forceinline__ float from_lane(float v, uint32_t k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ uint32_t from_lane(uint32_t v, uint32_t k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, k);
}

// A wavefront's own 64-entry slice of LDS (do-all workgroups hold at most 16
// wavefronts).  A chunk written there by its 64 lanes is read back entry by
// entry with one broadcast load per entry; a wavefront's LDS accesses are
// performed in program order, so no barrier is needed between them.
template <class T>
__device__ __forceinline__ T* wave_slice() {
  __shared__ T slice[16 * 64];
  return slice + (threadIdx.x >> 6) * 64;
}

// The per-id arrays are walked in chunks of 64 ids: lane l loads entry j0 + l
// of the next chunk (clamped to the last id, so every load stays in bounds)
// while the wavefront works through the current one.
__device__ __forceinline__ uint32_t chunk_id(uint32_t j0, uint32_t n) {
  const uint32_t j = j0 + lane_id();
  return j < n ? j : n - 1u;
}

struct BodyForce {
  static constexpr uint32_t kKind = 60;
  using Args = Bodies;
  static __device__ __forceinline__ void pair(const Args& a, float x, float y, float qx, float qy, float qm,
                                              float& sx, float& sy) {
    const float dx = qx - x, dy = qy - y;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, a.eps2));
    const float s = qm / (r2 * __builtin_sqrtf(r2));
    sx = __builtin_fmaf(s, dx, sx);
    sy = __builtin_fmaf(s, dy, sy);
  }
  template <class H>
  static __device__ bool run_wave(const H& h, uint32_t, uint32_t self, bool live, const Args& a) {
    const float x = fld<float>(h, self, kX), y = fld<float>(h, self, kY);
    const uint32_t n = a.n;
    float sx = 0.0f, sy = 0.0f;
    float4* const t = wave_slice<float4>();
    float4 nxt = a.P[chunk_id(0, n)];
    for (uint32_t j0 = 0; j0 < n; j0 += 64) {
      t[lane_id()] = nxt;
      nxt = a.P[chunk_id(j0 + 64, n)];
      const uint32_t m = n - j0 < 64 ? n - j0 : 64;
#pragma unroll 4
      for (uint32_t k = 0; k < m; ++k) {
        const float4 q = t[k];
        pair(a, x, y, q.x, q.y, q.z, sx, sy);
      }
    }
    if (live) {
      fld<float>(h, self, kAX) = sx;
      fld<float>(h, self, kAY) = sy;
    }
    return false;
  }
};

struct BodyMove {
  static constexpr uint32_t kKind = 61;
  using Args = Bodies;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const float vx = __builtin_fmaf(a.dt, fld<float>(h, self, kAX), fld<float>(h, self, kVX));
    const float vy = __builtin_fmaf(a.dt, fld<float>(h, self, kAY), fld<float>(h, self, kVY));
    const float x = __builtin_fmaf(a.dt, vx, fld<float>(h, self, kX));
    const float y = __builtin_fmaf(a.dt, vy, fld<float>(h, self, kY));
    fld<float>(h, self, kVX) = vx;
    fld<float>(h, self, kVY) = vy;
    fld<float>(h, self, kX) = x;
    fld<float>(h, self, kY) = y;
    const uint32_t id = fld<uint32_t>(h, self, kId);
    a.P[id] = make_float4(x, y, fld<float>(h, self, kM), 0.0f);
    a.V[id] = make_float2(vx, vy);
    return false;
  }
};

__device__ __forceinline__ bool within(const Bodies& a, float qx, float qy, float x, float y) {
  const float dx = qx - x, dy = qy - y;
  return __builtin_fmaf(dx, dx, dy * dy) < a.r2_merge;
}

struct BodyRoot {
  static constexpr uint32_t kKind = 62;
  using Args = Bodies;
  // A root has no live body of lower id within the merge radius, i.e. the
  // smallest squared distance to such a body is not below r2_merge (a NaN
  // distance is never below it, on either side of this equivalence).
  static __device__ __forceinline__ float d2(const Args& a, float4 c, uint32_t k, float x, float y) {
    const float dx = from_lane(c.x, k) - x, dy = from_lane(c.y, k) - y;
    return __builtin_fmaf(dx, dx, dy * dy);
  }
  template <class H>
  static __device__ bool run_wave(const H& h, uint32_t, uint32_t self, bool live, const Args& a) {
    const float x = fld<float>(h, self, kX), y = fld<float>(h, self, kY);
    const uint32_t id = live ? fld<uint32_t>(h, self, kId) : 0u;  // id 0: nothing to search
    const uint32_t n = a.n, lane = lane_id();
    float best = __builtin_inff();
    float4 nxt = a.P[chunk_id(0, n)];
    for (uint32_t j0 = 0; __ballot((j0 < id) & !(best < a.r2_merge)); j0 += 64) {
      const float4 cur = nxt;
      nxt = a.P[chunk_id(j0 + 64, n)];
      uint64_t alive = __ballot((cur.z > 0.0f) & (j0 + lane < n));  // live bodies of this chunk
      if (!__ballot(j0 + 64 > id)) {  // every lane's id lies above the chunk
        if (alive == ~0ull) {
#pragma unroll 8
          for (uint32_t k = 0; k < 64; ++k) best = fminf(best, d2(a, cur, k, x, y));
        } else {
          for (; alive; alive &= alive - 1ull) best = fminf(best, d2(a, cur, (uint32_t)__builtin_ctzll(alive), x, y));
        }
      } else {
        for (; alive; alive &= alive - 1ull) {
          const uint32_t k = (uint32_t)__builtin_ctzll(alive);
          const float d = d2(a, cur, k, x, y);
          if (j0 + k < id) best = fminf(best, d);
        }
      }
    }
    if (live) a.T[id] = best < a.r2_merge ? kAlone : kRoot;
    return false;
  }
};

struct BodyTarget {
  static constexpr uint32_t kKind = 63;
  using Args = Bodies;
  // Few bodies per step are not roots, so the wavefront searches for each of
  // them in turn, 64 candidate ids at a time (one id per lane).
  template <class H>
  static __device__ bool run_wave(const H& h, uint32_t, uint32_t self, bool live, const Args& a) {
    const uint32_t id = live ? fld<uint32_t>(h, self, kId) : 0u;
    const bool need = live && a.T[id] != kRoot;
    uint64_t pending = __ballot(need);
    if (!pending) return false;
    const float x = fld<float>(h, self, kX), y = fld<float>(h, self, kY);
    const uint32_t n = a.n, lane = lane_id();
    uint32_t found = kAlone;
    while (pending) {
      const uint32_t i = (uint32_t)__builtin_ctzll(pending);
      pending &= pending - 1ull;
      const float xi = from_lane(x, i), yi = from_lane(y, i);
      uint32_t hit = kAlone;
      uint32_t tn = a.T[chunk_id(0, n)];
      float4 pn = a.P[chunk_id(0, n)];
      for (uint32_t j0 = 0; j0 < n; j0 += 64) {
        const uint32_t tc = tn;
        const float4 pc = pn;
        tn = a.T[chunk_id(j0 + 64, n)];
        pn = a.P[chunk_id(j0 + 64, n)];
        // Only roots' entries are compared, and they do not change here.
        const uint64_t ok = __ballot((j0 + lane < n) & (tc == kRoot) & within(a, pc.x, pc.y, xi, yi));
        if (ok) {  // the lowest such id
          hit = j0 + (uint32_t)__builtin_ctzll(ok);
          break;
        }
      }
      if (lane == i) found = hit;
    }
    if (need && found != kAlone) a.T[id] = found;
    return false;
  }
};

struct BodyMerge {
  static constexpr uint32_t kKind = 64;
  using Args = Bodies;
  template <class H>
  static __device__ bool run_wave(const H& h, uint32_t, uint32_t self, bool live, const Args& a) {
    const uint32_t id = live ? fld<uint32_t>(h, self, kId) : 0u;
    const bool root = live && a.T[id] == kRoot;
    if (!__ballot(root)) return false;
    const uint32_t n = a.n;
    const float m = fld<float>(h, self, kM), x = fld<float>(h, self, kX), y = fld<float>(h, self, kY);
    const float vx = fld<float>(h, self, kVX), vy = fld<float>(h, self, kVY);
    float M = m, px = m * vx, py = m * vy, cx = m * x, cy = m * y;
    bool absorbed = false;
    uint32_t tn = a.T[chunk_id(0, n)];
    for (uint32_t j0 = 0; j0 < n; j0 += 64) {
      const uint32_t tc = tn;
      tn = a.T[chunk_id(j0 + 64, n)];
      uint64_t moving = __ballot(tc < n && j0 + lane_id() < n);  // ids that merge into a root
      while (moving) {  // in increasing id order
        const uint32_t k = (uint32_t)__builtin_ctzll(moving);
        moving &= moving - 1ull;
        if (root && id == from_lane(tc, k)) {
          const float4 q = a.P[j0 + k];
          const float2 w = a.V[j0 + k];
          M = M + q.z;
          px = __builtin_fmaf(q.z, w.x, px);
          py = __builtin_fmaf(q.z, w.y, py);
          cx = __builtin_fmaf(q.z, q.x, cx);
          cy = __builtin_fmaf(q.z, q.y, cy);
          absorbed = true;
        }
      }
    }
    if (!absorbed) return false;
    const float nvx = px / M, nvy = py / M;
    const float nx = cx / M, ny = cy / M;
    fld<float>(h, self, kVX) = nvx;
    fld<float>(h, self, kVY) = nvy;
    fld<float>(h, self, kX) = nx;
    fld<float>(h, self, kY) = ny;
    fld<float>(h, self, kM) = M;
    a.P[id] = make_float4(nx, ny, M, 0.0f);
    a.V[id] = make_float2(nvx, nvy);
    return false;
  }
};

struct BodyRemove {
  static constexpr uint32_t kKind = 65;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = Bodies;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t id = fld<uint32_t>(h, self, kId);
    if (a.T[id] >= a.n) return false;  // a root or alone: stays
    a.P[id].z = 0.0f;
    a.T[id] = kAlone;  // so that no later merge counts it again
    return true;
  }
};

// Bodies with m > 0 become objects; every id's P and V entries are set.
template <uint32_t LG>
__global__ void collide_init_kernel(DevHeapW<LG> h, Bodies a, const float* x, const float* y, const float* vx,
                                    const float* vy, const float* m) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  a.P[i] = make_float4(x[i], y[i], m[i] > 0.0f ? m[i] : 0.0f, 0.0f);
  a.V[i] = make_float2(vx[i], vy[i]);
  a.T[i] = kAlone;
  new_many(h, kBody, m[i] > 0.0f ? 1u : 0u, [&](uint32_t, uint32_t o) {
    if (o == kNull) return;
    fld<float>(h, o, kX) = x[i];
    fld<float>(h, o, kY) = y[i];
    fld<float>(h, o, kVX) = vx[i];
    fld<float>(h, o, kVY) = vy[i];
    fld<float>(h, o, kAX) = 0.0f;
    fld<float>(h, o, kAY) = 0.0f;
    fld<float>(h, o, kM) = m[i];
    fld<uint32_t>(h, o, kId) = i;
  });
}

__global__ void collide_read_kernel(Bodies a, float* x, float* y, float* vx, float* vy, float* m) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float4 p = a.P[i];
  const float2 v = a.V[i];
  x[i] = p.x;
  y[i] = p.y;
  vx[i] = v.x;
  vy[i] = v.y;
  m[i] = p.z;
}

bool collide_heap_ok(const dsoar_heap* h) {
  if (h->desc.num_types < 1) return false;
  const dsoar_type_layout& L = h->desc.types[kBody];
  if (L.num_fields < 8) return false;
  for (uint32_t f = 0; f < 8; ++f)
    if (L.field_bytes[f] != 4) return false;
  return true;
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

struct dsoar_collide {
  dsoar_heap* heap;
  Bodies a;
  StepGraphs graphs;
};

namespace {

int collide_one_step(dsoar_collide* c, uint32_t flags, hipStream_t st) {
  dsoar_heap* h = c->heap;
  const uint32_t base = flags & DSOAR_DO_PLAIN, reuse = base | DSOAR_DO_REUSE_ENUM;
  int rc = launch_doall<BodyForce>(h, kBody, c->a, base, st);
  if (!rc) rc = launch_doall<BodyMove>(h, kBody, c->a, reuse, st);
  // No squared distance is below a merge radius of 0: the bodies then never
  // merge (the paper's nbody application), and the merge phases would change
  // nothing.
  if (!(c->a.r2_merge > 0.0f)) return rc;
  if (!rc) rc = launch_doall<BodyRoot>(h, kBody, c->a, reuse, st);
  if (!rc) rc = launch_doall<BodyTarget>(h, kBody, c->a, reuse, st);
  if (!rc) rc = launch_doall<BodyMerge>(h, kBody, c->a, reuse, st);
  if (!rc) rc = launch_doall<BodyRemove>(h, kBody, c->a, reuse, st);
  return rc;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

size_t dsoar_collide_bytes(uint32_t n) {
  if (n == 0 || n > (1u << 24)) return 0;
  return align256((size_t)n * 16) + align256((size_t)n * 8) + align256((size_t)n * 4);
}

int dsoar_collide_create(dsoar_heap* heap, uint32_t n, const dsoar_collide_params* params, void* dev_mem,
                         size_t dev_bytes, dsoar_collide** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !collide_heap_ok(heap) || !params || !dev_mem || ((uintptr_t)dev_mem & 255u) ||
      !(params->eps2 > 0.0f) || !(params->r2_merge >= 0.0f))
    return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_collide_bytes(n);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_collide* c = new (std::nothrow) dsoar_collide;
  if (!c) return DSOAR_ERR_INVALID_ARG;
  memset(c, 0, sizeof(*c));
  c->heap = heap;
  uint8_t* b = (uint8_t*)dev_mem;
  c->a.P = (float4*)b;
  c->a.V = (float2*)(b + align256((size_t)n * 16));
  c->a.T = (uint32_t*)(b + align256((size_t)n * 16) + align256((size_t)n * 8));
  c->a.n = n;
  c->a.dt = params->dt;
  c->a.eps2 = params->eps2;
  c->a.r2_merge = params->r2_merge;
  *out = c;
  return DSOAR_OK;
}

int dsoar_collide_destroy(dsoar_collide* c) {
  if (!c) return DSOAR_ERR_INVALID_ARG;
  step_graphs_clear(c->graphs);
  delete c;
  return DSOAR_OK;
}

int dsoar_collide_init(dsoar_collide* c, const float* x_dev, const float* y_dev, const float* vx_dev,
                       const float* vy_dev, const float* m_dev, void* stream) {
  if (!c || !x_dev || !y_dev || !vx_dev || !vy_dev || !m_dev) return DSOAR_ERR_INVALID_ARG;
  with_width(c->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(c->heap, kKindCollideInit, collide_init_kernel<kLG>, dim3((uint32_t)(((uint64_t)c->a.n + 255) / 256)), dim3(256), (hipStream_t)stream, DevHeapW<kLG>(c->heap->dev),
                     c->a, x_dev, y_dev, vx_dev, vy_dev, m_dev);
  });
  DSOAR_LAUNCHED(c->heap);
  return DSOAR_OK;
}

int dsoar_collide_step(dsoar_collide* c, uint32_t steps, uint32_t flags, void* stream) {
  if (!c) return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  dsoar_heap* h = c->heap;
  if (flags & DSOAR_GRAPH) {
    if (flags & DSOAR_DO_PLAIN) return DSOAR_ERR_INVALID_ARG;
    return step_graphs_run(h, c->graphs, steps, st, [&](hipStream_t gs) { return collide_one_step(c, 0, gs); });
  }
  for (uint32_t i = 0; i < steps; ++i) {
    const int rc = collide_one_step(c, flags, st);
    if (rc) return rc;
  }
  return DSOAR_OK;
}

int dsoar_collide_read(dsoar_collide* c, float* x_dev, float* y_dev, float* vx_dev, float* vy_dev, float* m_dev,
                       void* stream) {
  if (!c || !x_dev || !y_dev || !vx_dev || !vy_dev || !m_dev) return DSOAR_ERR_INVALID_ARG;
  hipLaunchKernelGGL(collide_read_kernel, dim3((uint32_t)(((uint64_t)c->a.n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, c->a, x_dev,
                     y_dev, vx_dev, vy_dev, m_dev);
  DSOAR_LAUNCHED(c->heap);
  return DSOAR_OK;
}

}  // extern "C"
