// Host-side heap object and the do-all launcher shared by the library's
// translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dsoar.h"
#include "dsoar_device.hpp"

namespace dsoar {

// Enumeration tiling: one wavefront scans 1 word of the level-0 allocated[T]
// bitmap (64 blocks), or kEnumWideWords words when the bitmap has more than
// kEnumWideFrom words; a workgroup of kEnumWaves wavefronts is one tile of
// the decoupled look-back scan.
constexpr uint32_t kEnumWaves = 8;
constexpr uint32_t kEnumWideWords = 8;
constexpr uint32_t kEnumWideFrom = 16384;

// Per-type scan state: tile ticket, epoch (so the look-back flags never need
// clearing between launches), the resulting count, then one flag per tile.
struct ScanState {
  uint32_t tile_counter;
  uint32_t epoch;
  uint32_t count;
  uint32_t pad;
};

struct EnumOut {
  uint32_t* R;          // compacted block ids
  uint64_t* S;          // snapshot of each listed block's object bitmap
  ScanState* st;
  uint64_t* flags;      // num_tiles look-back words
  uint32_t num_tiles;
};

struct StatsOut {
  uint64_t live[kMaxTypes];
  uint32_t allocated[kMaxTypes];
  uint32_t active[kMaxTypes];
  uint32_t typed[kMaxTypes];
  uint32_t free_blocks;
  uint32_t pad;
  uint32_t viol[DSOAR_INV_COUNT];
};

}  // namespace dsoar

struct dsoar_heap {
  dsoar::DevHeap dev;
  dsoar_heap_desc desc;
  dsoar_heap_layout layout;
  uint8_t* base;
  size_t bytes;
  dsoar::EnumOut enum_out[dsoar::kMaxTypes];
  dsoar::StatsOut* stats_dev;
  uint32_t num_tiles;
  uint32_t enum_wpw;           // level-0 words per enumeration wavefront
  uint32_t num_cus;
  uint32_t doall_wg_threads;   // workgroup size of do-all launches
  uint32_t doall_wgs_per_cu;   // persistent grid = num_cus * this
  uint32_t config_epoch;       // bumped when launch shape or policy change
  hipError_t last_hip;
  // Optional per-launch timing with HIP events on the launch stream.
  int timing;
  hipEvent_t* ev_pool;         // 2 * kTimingCap events, created on enable
  uint32_t* rec_kind;          // kind of each recorded launch
  uint32_t rec_used;
};

namespace dsoar {

inline int hip_fail(dsoar_heap* h, hipError_t e) {
  if (h) h->last_hip = e;
  return DSOAR_ERR_HIP;
}

#define DSOAR_HIP(h, expr)                         \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(h, e_);  \
  } while (0)

#define DSOAR_LAUNCHED(h) DSOAR_HIP(h, hipGetLastError())

constexpr uint32_t kTimingCap = 8192;
constexpr uint32_t kKindEnumerate = 1;

// Brackets one launch with a pair of events when timing is on.  Returns the
// record index (or -1 when off or full).
inline int timing_begin(dsoar_heap* h, uint32_t kind, hipStream_t s) {
  if (!h->timing || h->rec_used >= kTimingCap) return -1;
  const int r = (int)h->rec_used++;
  h->rec_kind[r] = kind;
  (void)hipEventRecord(h->ev_pool[2 * r], s);
  return r;
}
inline void timing_end(dsoar_heap* h, int r, hipStream_t s) {
  if (r >= 0) (void)hipEventRecord(h->ev_pool[2 * r + 1], s);
}

int launch_enumerate(dsoar_heap* h, uint32_t type, hipStream_t s);
int read_count(dsoar_heap* h, uint32_t type, hipStream_t s, uint32_t* count);

// The do-all kernel (Sec. 2.3).  Entry e of the compacted list R is handled
// by capacity consecutive lanes: with capacity 64 one wavefront per block,
// with 32 two blocks per wavefront.  Lane slot s runs the method when bit s of
// the snapshot S[e] is set.  Deletes of `this` are collected with a ballot and
// applied as one atomic AND per block when the wavefront finishes the block.
//
// Method: struct with `struct Args`, a `static constexpr uint32_t kKind`
// (an id for per-kernel timing) and
//   static __device__ bool run(const DevHeap&, uint32_t type, uint32_t self, const Args&)
// returning true to delete self.
template <class Method>
__global__ void __launch_bounds__(1024) doall_kernel(DevHeap h, uint32_t type, const uint32_t* __restrict__ R,
                                                      const uint64_t* __restrict__ S, const uint32_t* count_ptr,
                                                      typename Method::Args args) {
  const uint32_t lane = lane_id();
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t gw = blockIdx.x * wpb + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * wpb;
  const uint32_t count = bcast32(*count_ptr);
  uint32_t visits = 0, freed = 0;
  if (h.capacity == 64) {
    for (uint32_t e = gw; e < count; e += nw) {
      const uint32_t bid = R[e];
      const uint64_t snap = S[e];
      visits += (uint32_t)__popcll(snap);
      bool del = false;
      if ((snap >> lane) & 1ull) del = Method::run(h, type, make_obj(bid, lane), args);
      const uint64_t dm = __ballot(del);
      if (dm) freed += delete_mask(h, type, bid, dm);
    }
  } else {
    const uint32_t half = lane >> 5, slot = lane & 31u;
    for (uint32_t e0 = 2 * gw; e0 < count; e0 += 2 * nw) {
      const uint32_t e = e0 + half;
      const bool valid = e < count;
      const uint32_t bid = valid ? R[e] : 0u;
      const uint64_t snap = valid ? S[e] : 0ull;
      visits += (uint32_t)__popcll(__ballot((snap >> slot) & 1ull));
      bool del = false;
      if ((snap >> slot) & 1ull) del = Method::run(h, type, make_obj(bid, slot), args);
      const uint64_t dm = __ballot(del);
      if (dm & 0xFFFFFFFFull) freed += delete_mask(h, type, __builtin_amdgcn_readlane(bid, 0), dm & 0xFFFFFFFFull);
      if (dm >> 32) freed += delete_mask(h, type, __builtin_amdgcn_readlane(bid, 32), dm >> 32);
    }
  }
  if (visits) lead_add(shard(h) + kCntVisits + type, visits);
  if (freed) lead_add(shard(h) + kCntFrees + type, freed);
}

// Enumerate (unless reusing) and launch the do-all of Method over `type`.
template <class Method>
int launch_doall(dsoar_heap* h, uint32_t type, const typename Method::Args& args, uint32_t flags,
                 hipStream_t s) {
  if (type >= h->desc.num_types) return DSOAR_ERR_INVALID_ARG;
  if (!(flags & DSOAR_DO_REUSE_ENUM)) {
    int rc = launch_enumerate(h, type, s);
    if (rc) return rc;
  }
  const EnumOut& eo = h->enum_out[type];
  const uint32_t threads = h->doall_wg_threads;
  uint32_t grid;
  if (flags & DSOAR_DO_PLAIN) {
    uint32_t count = 0;
    int rc = read_count(h, type, s, &count);
    if (rc) return rc;
    if (count == 0) return DSOAR_OK;
    const uint32_t per_wave = 64 / h->desc.block_capacity;
    const uint64_t waves = (count + per_wave - 1) / per_wave;
    grid = (uint32_t)((waves * 64 + threads - 1) / threads);
  } else {
    grid = h->num_cus * h->doall_wgs_per_cu;
  }
  const int rec = timing_begin(h, Method::kKind, s);
  hipLaunchKernelGGL(doall_kernel<Method>, dim3(grid), dim3(threads), 0, s, h->dev, type, eo.R, eo.S,
                     &eo.st->count, args);
  timing_end(h, rec, s);
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

inline bool heap_ok(const dsoar_heap* h) { return h != nullptr && h->base != nullptr; }

}  // namespace dsoar
