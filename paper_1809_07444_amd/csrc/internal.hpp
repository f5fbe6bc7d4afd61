// Host-side heap object and the do-all launcher shared by the library's
// translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/dsoar.h"
#include "dsoar_device.hpp"

namespace dsoar {

// Enumeration tiling: one wavefront scans 1 word of the level-0 allocated[T]
// bitmap (64 blocks), or kEnumWideWords words when the bitmap has more than
// kEnumWideFrom words; a workgroup of enum_waves(WPW) wavefronts is one tile
// of the decoupled look-back scan.  Wide scans take 16 wavefronts per tile:
// far fewer tiles, so a shorter look-back chain (a 2^22-block heap's scan 33
// -> 22 us, a 2^18-block one's 13.7 -> 8.5 us); narrow ones keep 8, which
// spreads a small heap's few words over more workgroups (768 words: 6.9
// against 11.5 us wide).
constexpr uint32_t kEnumWideWords = 8;
constexpr uint32_t kEnumWideFrom = 2048;
constexpr uint32_t enum_waves(uint32_t wpw) { return wpw > 1 ? 16u : 8u; }

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
  uint32_t* count_out;  // where the count also goes (nullptr: only st->count)
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
  uint32_t subtypes[dsoar::kMaxTypes];  // bit u of [t]: type u is t or inherits from t
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
// Timing ids of the kernels outside the do-alls that create objects or
// advance a step (the do-all methods carry their own).
constexpr uint32_t kKindMicroCreate = 22;
constexpr uint32_t kKindGolInit = 36;
constexpr uint32_t kKindGolAdmit = 37;
constexpr uint32_t kKindSugarRegrow = 46;
constexpr uint32_t kKindSugarAdmit = 47;
constexpr uint32_t kKindTrafficEntry = 52;
constexpr uint32_t kKindTrafficInit = 53;
constexpr uint32_t kKindCollideInit = 66;
constexpr uint32_t kKindWatorInit = 77;
constexpr uint32_t kKindWatorTick = 78;

// Launches `kernel` on stream s.  With timing on (and room in the record), the
// launch itself carries a start and a stop event (hipExtLaunchKernel): they
// take the dispatch's own begin and end timestamps, so the recorded time is
// the kernel's execution without the gaps around it.
template <class K, class... A>
inline void launch_timed(dsoar_heap* h, uint32_t kind, K kernel, dim3 grid, dim3 block, hipStream_t s,
                         A... args) {
  if (h->timing && h->rec_used < kTimingCap) {
    const uint32_t r = h->rec_used++;
    h->rec_kind[r] = kind;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, h->ev_pool[2 * r], h->ev_pool[2 * r + 1], 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

// Kernels that touch the block-state bitmaps are instantiated once per
// container width, taking their heap as a DevHeapW<LG>; with_width calls f
// with the width of this heap as a compile-time constant, for the launch of
// the matching instance.
template <class F>
inline void with_width(const dsoar_heap* h, F&& f) {
  if (h->dev.bm_lg == 6)
    f(std::integral_constant<uint32_t, 6>{});
  else
    f(std::integral_constant<uint32_t, 5>{});
}

int launch_enumerate(dsoar_heap* h, uint32_t type, hipStream_t s);
int read_count(dsoar_heap* h, uint32_t type, hipStream_t s, uint32_t* count);

// A method may split into a load phase and an apply phase:
//   struct Pre { ... };                      // values the load phase reads
//   static __device__ Pre load(const DevHeap&, uint32_t type, uint32_t self, const Args&);
//   static __device__ bool apply(const DevHeap&, uint32_t type, uint32_t self, const Args&, const Pre&);
// load must not write memory and may read only fields of `self` (it also runs
// for the empty slots of a listed block, whose values it must not use); apply
// may write the fields of `self`, create objects of other types, and write
// state that no load phase of the do-all reads (objects of other types,
// grids), since the loads of later blocks are issued before earlier blocks
// are applied.  (Creating objects of the do-all's own type is left to the
// run form: the split do-all settles a pass's return of full blocks to
// active[type] only after the next pass is applied, and a reservation in that
// pass that filled such a block again would wait on it.)  The do-all then issues the loads of U blocks
// before it applies the method to any of them, so a wavefront keeps U times
// more bytes in flight; this is what lets a do-all over a heap larger than
// the caches approach the HBM bandwidth.
template <class M, class = void>
struct HasSplit : std::false_type {};
template <class M>
struct HasSplit<M, std::void_t<typename M::Pre>> : std::true_type {};

// Or a method may take the whole wavefront:
//   static __device__ bool run_wave(const DevHeap&, uint32_t type, uint32_t self, bool live, const Args&);
// The do-all calls it with every lane active; `live` tells whether `self` is
// an allocated object of the do-all.  The other lanes carry an empty slot of
// a listed block (or of block 0 past the end of the list): their field reads
// stay inside the heap but return nothing meaningful, and they must write
// nothing.  With all lanes active, a wavefront can load a chunk of a shared
// array with one coalesced access and hand its entries around with
// cross-lane reads, where a per-lane loop would wait on one load per entry.
// Only a live lane's true return deletes its object.
template <class M, class = void>
struct HasWave : std::false_type {};
template <class M>
struct HasWave<M, std::void_t<decltype(&M::template run_wave<DevHeap>)>> : std::true_type {};

// Or a method may take two list entries per wavefront pass (capacity 64, on
// lists of at least two entries per wavefront):
//   static __device__ void run_pair(const DevHeap&, uint32_t type, uint32_t self0, bool live0,
//                                   uint32_t self1, bool live1, const Args&, bool& del0, bool& del1);
// Lane l holds slot l of both blocks and enters when either slot is live.
// The method issues the loads of both objects before it uses any, and makes
// one wavefront request for the objects both create, so one chain of
// dependent loads and allocation atomics serves two blocks.  Empty slots'
// fields hold anything: the method must not index memory with them.  It
// still provides `run` (capacity 32, lists of fewer than two entries per
// wavefront, and callers of single objects).
template <class M, class = void>
struct HasPair : std::false_type {};
template <class M>
struct HasPair<M, std::void_t<decltype(&M::template run_pair<DevHeap>)>> : std::true_type {};

// A method may also declare
//   static constexpr bool kDeletesOnlyThis = true;
// when it deletes no object but `this` (and a two-list do-all pairs it only
// with another such method).  Then a block whose snapshot is full is still
// exactly full when its wavefront deletes from it: no other wavefront
// removes its objects, and a full block is not active, so no allocation adds
// to it.  Its object-bitmap AND needs no result, and the OR that returns the
// block to active[type] is settled after the next entry's list reads, before
// that entry's method runs.
template <class M, class = void>
struct DeletesOnlyThis : std::false_type {};
template <class M>
struct DeletesOnlyThis<M, std::void_t<decltype(M::kDeletesOnlyThis)>>
    : std::integral_constant<bool, M::kDeletesOnlyThis> {};

// A method may also declare
//   static constexpr uint32_t kMinWaves = 8;
// to have its do-all kernels on large heaps compiled for at least that many
// wavefronts per SIMD: the allocation path holds about 104 scalar registers,
// which leaves room for seven, and on long lists chains of dependent atomics
// want every wavefront the SIMD can hold (scalar values beyond the budget
// live in vector lanes).  On small heaps, whose lists give a wavefront about
// one entry, more resident wavefronts gain nothing and the spills of the
// tighter budget lengthen the chain, so they keep the unconstrained kernel.
template <class M, class = void>
struct MinWaves : std::integral_constant<uint32_t, 1> {};
template <class M>
struct MinWaves<M, std::void_t<decltype(M::kMinWaves)>> : std::integral_constant<uint32_t, M::kMinWaves> {};

template <class Method, class H>
__device__ __forceinline__ bool run_method(const H& h, uint32_t type, uint32_t self,
                                           const typename Method::Args& a) {
  if constexpr (HasSplit<Method>::value)
    return Method::apply(h, type, self, a, Method::load(h, type, self, a));
  else
    return Method::run(h, type, self, a);
}

// The method on one lane's slot: every lane enters for a wavefront method,
// only live lanes otherwise.
template <class Method, class H>
__device__ __forceinline__ bool run_slot(const H& h, uint32_t type, uint32_t self, bool live,
                                         const typename Method::Args& a) {
  if constexpr (HasWave<Method>::value) {
    const bool del = Method::run_wave(h, type, self, live, a);
    return live && del;
  } else {
    bool del = false;
    if (live) del = run_method<Method>(h, type, self, a);
    return del;
  }
}

// Makes the value's registers an input of an empty asm statement: the
// compiler then waits for the loads that produce it at this point (and not
// later, at a conditional use).  No instruction is emitted.
template <class T>
__device__ __forceinline__ void ready(const T& v) {
  if constexpr (sizeof(T) % 4 == 0) {
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (uint32_t i = 0; i < sizeof(T) / 4; ++i) __asm__ volatile("" ::"v"(w[i]));
  }
}

// One pass of the split do-all: U list entries, their snapshots and the
// values the load phase read for them.
template <class Method, uint32_t U>
struct SplitPass {
  uint32_t bid[U];
  uint64_t snap[U];
  typename Method::Pre pre[U];
};

// Capacity 64, U blocks per wavefront pass, software-pipelined over two
// passes: the list entries of pass k+2 and the field loads of pass k+1 are
// issued before pass k is applied, so neither the list reads nor the stores
// of pass k wait for each other.  List entries [e, e + U) are read by lane
// groups (index clamped to the list, so the loads are unconditional) and
// broadcast with readlane.  Every lane runs the load phase, live slot or not
// (all slots of a listed block are addressable): the loads are straight-line
// code.  The two pass buffers alternate so that no loaded value is copied
// between registers before it is used.
template <class Method, uint32_t U, class H>
__device__ __forceinline__ void doall_split64(const H& h, uint32_t type, const uint32_t* __restrict__ R,
                                              const uint64_t* __restrict__ S, uint32_t count, uint32_t gw,
                                              uint32_t nw, const typename Method::Args& args, uint32_t& visits,
                                              uint32_t& freed) {
  const uint32_t lane = lane_id();
  const uint32_t stride = nw * U;
  constexpr uint64_t kFull64 = ~0ull;  // capacity 64: every bit is a slot
  uint32_t rl;
  uint64_t sl;
  auto fetch = [&](uint32_t e) {
    const uint32_t ei = min(e + (lane & (U - 1)), count - 1);
    rl = R[ei];
    sl = S[ei];
  };
  auto take = [&](SplitPass<Method, U>& p, uint32_t e) {
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      p.bid[u] = (uint32_t)__builtin_amdgcn_readlane(rl, u);
      // readlane returns int: widen through uint32_t, never sign-extend.
      const uint64_t sn = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(sl >> 32), u) << 32) |
                          (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)sl, u);
      p.snap[u] = e + u < count ? sn : 0ull;
    }
  };
  auto issue = [&](SplitPass<Method, U>& p) {
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) p.pre[u] = Method::load(h, type, make_obj(p.bid[u], lane), args);
    // Compiler barrier (no instruction): keeps the loads here instead of
    // letting them sink to their conditional uses after the next pass.
    __asm__ volatile("" ::: "memory");
  };
  // The active-bitmap OR of the last pass, settled (its result used) one
  // pass later, when it has long returned.
  const Bitmap act = active_bm(h, type);
  uint32_t pend_word = 0;
  uint64_t pend_bits = 0, pend_prev = 0;
  auto settle = [&]() {
    if (pend_bits) bm_set_bits0_settle(act, pend_word, pend_bits, pend_prev);
    pend_bits = 0;
  };
  auto finish = [&](SplitPass<Method, U>& p) {
    // Take delivery of every value of the pass here, unconditionally: the
    // applies below run under per-lane conditions, and a load whose value a
    // skipped apply never used would otherwise make the compiler wait
    // before reusing its register in the next pass.
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) ready(p.pre[u]);
    uint64_t dm[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      visits += (uint32_t)__popcll(p.snap[u]);
      bool del = false;
      if ((p.snap[u] >> lane) & 1ull) del = Method::apply(h, type, make_obj(p.bid[u], lane), args, p.pre[u]);
      dm[u] = __ballot(del);
    }
    // Deferred deletes of the pass: the leader issues every object-bitmap
    // AND before it waits for any result; the blocks that were full go back
    // to active[type] with one OR per level-0 word (the pass's blocks are
    // consecutive in the ascending list, so they mostly share one word).
    // A block whose snapshot is full is still exactly full here: during a
    // do-all only the wavefront visiting a block removes its objects
    // (methods delete only `this`), and a full block is not active, so no
    // allocation adds to it.  Its AND needs no result and is not waited for.
    uint64_t any = 0;
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) any |= dm[u];
    if (any) {
      const bool leader = is_first_active();
      // Two separate loops, so the compiler keeps the first kind of AND
      // without a return value instead of merging it with the second.
#pragma unroll
      for (uint32_t u = 0; u < U; ++u)
        if (dm[u] && p.snap[u] == kFull64 && leader)
          __hip_atomic_fetch_and(h.obj_bitmap + p.bid[u], ~dm[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t prev[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        prev[u] = 0;
        if (dm[u] && p.snap[u] != kFull64 && leader)
          prev[u] = __hip_atomic_fetch_and(h.obj_bitmap + p.bid[u], ~dm[u], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      }
      uint32_t act_word = 0xFFFFFFFFu;
      uint64_t act_bits = 0;
      uint32_t emptied = 0;  // bit u: this pass's deletes left block u empty
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (!dm[u]) continue;
        const uint64_t pv = p.snap[u] == kFull64 ? kFull64 : bcast64(prev[u]);
        if ((pv & dm[u]) != dm[u]) lead_flag(h.ctrl + kCtlDoubleFree);
        const uint64_t removed = pv & dm[u];
        freed += (uint32_t)__popcll(removed);
        if (removed && (pv & ~dm[u]) == 0) emptied |= 1u << u;
        if (removed && (pv & kFull64) == kFull64) {
          const uint32_t w = p.bid[u] >> 6;
          if (w != act_word) {
            if (act_bits) bm_set_bits0(act, act_word, act_bits);
            act_word = w;
            act_bits = 0;
          }
          act_bits |= 1ull << (p.bid[u] & 63u);
        }
      }
      if (act_bits) {
        if (h.online_reclaim) {
          bm_set_bits0(act, act_word, act_bits);  // settled before the releases below
        } else {
          settle();
          pend_word = act_word;
          pend_bits = act_bits;
          pend_prev = bm_set_bits0_issue(act, act_word, act_bits);
        }
      }
      if (h.online_reclaim && emptied) {
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
          if ((emptied >> u) & 1u) try_release(h, type, p.bid[u]);
      }
    }
  };
  uint32_t e = gw * U;
  if (e >= count) return;
  SplitPass<Method, U> A, B;
  fetch(e);
  take(A, e);
  fetch(e + stride);
  issue(A);
  // The next pass is issued unconditionally (past the end of the list its
  // snapshots are empty), so the compiler's wait counts never have to allow
  // for a skipped batch of loads.
  for (;;) {
    const uint32_t e1 = e + stride;
    take(B, e1);
    fetch(e1 + stride);
    issue(B);
    finish(A);
    if (e1 >= count) break;
    const uint32_t e2 = e1 + stride;
    take(A, e2);
    fetch(e2 + stride);
    issue(A);
    finish(B);
    if (e2 >= count) break;
    e = e2;
  }
  settle();
}

// The do-all kernel (Sec. 2.3).  Entry e of the compacted list R is handled
// by capacity consecutive lanes: with capacity 64 one wavefront per block,
// with 32 two blocks per wavefront.  Lane slot s runs the method when bit s of
// the snapshot S[e] is set.  Deletes of `this` are collected with a ballot and
// applied as one atomic AND per block when the wavefront finishes the block.
//
// Method: struct with `struct Args`, a `static constexpr uint32_t kKind`
// (an id for per-kernel timing) and either
//   static __device__ bool run(const DevHeap&, uint32_t type, uint32_t self, const Args&)
// returning true to delete self, or the load / apply pair described above.
// One wavefront's share of a do-all over one list: entries gw, gw + nw, ...
// (or passes of several entries), visit and free counts accumulated.
template <class Method, bool kOnlyThis, class H>
__device__ __forceinline__ void doall_list(const H& h, uint32_t type, const uint32_t* __restrict__ R,
                                           const uint64_t* __restrict__ S, uint32_t count, uint32_t gw,
                                           uint32_t nw, const typename Method::Args& args, uint32_t& visits,
                                           uint32_t& freed) {
  const uint32_t lane = lane_id();
  const uint32_t c = cap_of(h, type);
  if constexpr (HasSplit<Method>::value) {
    // Several blocks per pass only when every wavefront gets that many.
    if (c == 64 && h.doall_unroll > 1 && count >= nw * h.doall_unroll) {
      if (h.doall_unroll >= 8)
        doall_split64<Method, 8>(h, type, R, S, count, gw, nw, args, visits, freed);
      else if (h.doall_unroll >= 4)
        doall_split64<Method, 4>(h, type, R, S, count, gw, nw, args, visits, freed);
      else
        doall_split64<Method, 2>(h, type, R, S, count, gw, nw, args, visits, freed);
      return;
    }
  }
  if (c == 64) {
    const bool fast = kOnlyThis && !h.online_reclaim;
    const Bitmap act = active_bm(h, type);
    uint32_t pend_word = 0;
    uint64_t pend_bits = 0, pend_prev = 0;
    // The last block's active-bitmap OR is settled before the next method
    // runs: a method that creates objects of this type may fill that block
    // again, and the clear of its active bit that the filling reservation
    // makes would wait for the nested set of this settle.
    auto settle = [&]() {
      if (pend_bits) bm_set_bits0_settle(act, pend_word, pend_bits, pend_prev);
      pend_bits = 0;
    };
    auto remove = [&](uint32_t bid, uint64_t snap, uint64_t dm) {
      if (fast && snap == ~0ull) {
        // A full block (see DeletesOnlyThis): nothing to wait for.
        if (is_first_active())
          __hip_atomic_fetch_and(h.obj_bitmap + bid, ~dm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        freed += (uint32_t)__popcll(dm);
        chaos_pause(kChaosDeleteActive);
        settle();
        pend_word = bid >> 6;
        pend_bits = 1ull << (bid & 63u);
        pend_prev = bm_set_bits0_issue(act, pend_word, pend_bits);
      } else {
        freed += delete_mask(h, type, bid, dm);
      }
    };
    // This wavefront's first entry of the single-object loop, loaded before
    // the count is known (R and S hold num_blocks entries, so the load stays
    // in bounds): on lists of about one entry per wavefront the count's load
    // and the entry's then take one round trip instead of two.
    const uint32_t first = gw < h.num_blocks ? gw : h.num_blocks - 1;
    const uint32_t first_bid = R[first];
    const uint64_t first_snap = S[first];
    bool pairs = false;
    if constexpr (HasPair<Method>::value) pairs = count >= 2 * nw;
    if (pairs) {
      // Pairs only when every wavefront gets two entries or more: on a short
      // list they would leave half the wavefronts without work, and the
      // method's single-object form runs instead.
      const uint32_t per = 2;
      for (uint32_t e = per * gw; e < count; e += per * nw) {
        const bool has1 = e + 1 < count;
        const uint32_t b0 = R[e], b1 = has1 ? R[e + 1] : b0;
        const uint64_t s0 = S[e], s1 = has1 ? S[e + 1] : 0ull;
        visits += (uint32_t)(__popcll(s0) + __popcll(s1));
        settle();
        const bool l0 = (s0 >> lane) & 1ull, l1 = (s1 >> lane) & 1ull;
        bool d0 = false, d1 = false;
        if constexpr (HasPair<Method>::value)
          if (l0 || l1) Method::run_pair(h, type, make_obj(b0, lane), l0, make_obj(b1, lane), l1, args, d0, d1);
        const uint64_t dm0 = __ballot(l0 && d0), dm1 = __ballot(l1 && d1);
        if (dm0) remove(b0, s0, dm0);
        if (dm1) remove(b1, s1, dm1);
      }
    } else {
      for (uint32_t e = gw; e < count; e += nw) {
        const uint32_t bid = e == gw ? first_bid : R[e];
        const uint64_t snap = e == gw ? first_snap : S[e];
        visits += (uint32_t)__popcll(snap);
        settle();
        const bool del = run_slot<Method>(h, type, make_obj(bid, lane), (snap >> lane) & 1ull, args);
        const uint64_t dm = __ballot(del);
        if (dm) remove(bid, snap, dm);
      }
    }
    settle();
  } else {
    // 64 / c blocks per wavefront: lane l handles slot l % c of entry
    // e0 + l / c (Fig. 4 with blocks smaller than a wavefront).
    const uint32_t bpw = 64u / c, sh = (uint32_t)__builtin_ctz(c);
    const uint32_t sub = lane >> sh, slot = lane & (c - 1u);
    const uint64_t group = c == 64 ? ~0ull : ((1ull << c) - 1ull);
    for (uint32_t e0 = bpw * gw; e0 < count; e0 += bpw * nw) {
      const uint32_t e = e0 + sub;
      const bool valid = e < count;
      const uint32_t bid = valid ? R[e] : 0u;
      const uint64_t snap = valid ? S[e] : 0ull;
      visits += (uint32_t)__popcll(__ballot((snap >> slot) & 1ull));
      const bool del = run_slot<Method>(h, type, make_obj(bid, slot), (snap >> slot) & 1ull, args);
      const uint64_t dm = __ballot(del);
      for (uint32_t k = 0; k < bpw && dm; ++k) {
        const uint64_t part = (dm >> (k * c)) & group;
        if (part) freed += delete_mask(h, type, (uint32_t)__builtin_amdgcn_readlane(bid, k * c), part);
      }
    }
  }
}

// Wave-uniform index of this wavefront in the grid.
__device__ __forceinline__ uint32_t grid_wave() {
  return blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

template <class Method, uint32_t LG, bool kMany = false>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kMany ? MinWaves<Method>::value : 1)))
doall_kernel(DevHeapW<LG> h, uint32_t type, const uint32_t* __restrict__ R,
                                                      const uint64_t* __restrict__ S, const uint32_t* count_ptr,
                                                      typename Method::Args args) {
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  uint32_t visits = 0, freed = 0;
  doall_list<Method, DeletesOnlyThis<Method>::value>(h, type, R, S, bcast32(*count_ptr), grid_wave(), nw, args,
                                                      visits, freed);
  if (visits) lead_add(shard(h) + kCntVisits + type, visits);
  if (freed) lead_add(shard(h) + kCntFrees + type, freed);
}

// Two do-alls in one launch, over the lists of two types: every wavefront
// takes its share of the first list, then of the second.  For methods that
// may run at the same time (neither reads what the other writes, apart from
// the heap's own atomics): one kernel boundary and one launch fewer.
template <class M1, class M2, uint32_t LG, bool kMany = false>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(!kMany ? 1u
                                          : MinWaves<M1>::value > MinWaves<M2>::value ? MinWaves<M1>::value
                                                                                      : MinWaves<M2>::value)))
doall2_kernel(DevHeapW<LG> h, uint32_t t1, const uint32_t* __restrict__ R1,
                                                       const uint64_t* __restrict__ S1, const uint32_t* c1,
                                                       typename M1::Args a1, uint32_t t2,
                                                       const uint32_t* __restrict__ R2,
                                                       const uint64_t* __restrict__ S2, const uint32_t* c2,
                                                       typename M2::Args a2) {
  const uint32_t nw = gridDim.x * (blockDim.x >> 6), gw = grid_wave();
  uint32_t visits = 0, freed = 0;
  constexpr bool kOnlyThis = DeletesOnlyThis<M1>::value && DeletesOnlyThis<M2>::value;
  doall_list<M1, kOnlyThis>(h, t1, R1, S1, bcast32(*c1), gw, nw, a1, visits, freed);
  if (visits) lead_add(shard(h) + kCntVisits + t1, visits);
  if (freed) lead_add(shard(h) + kCntFrees + t1, freed);
  visits = freed = 0;
  doall_list<M2, kOnlyThis>(h, t2, R2, S2, bcast32(*c2), gw, nw, a2, visits, freed);
  if (visits) lead_add(shard(h) + kCntVisits + t2, visits);
  if (freed) lead_add(shard(h) + kCntFrees + t2, freed);
}

// Large heaps: those whose enumeration takes wide tiles (more than
// kEnumWideFrom level-0 words, 131,072 blocks).
inline bool large_heap(const dsoar_heap* h) { return h->enum_wpw == kEnumWideWords; }

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
    const uint32_t per_wave = 64 / h->dev.capacity[type];
    const uint64_t waves = (count + per_wave - 1) / per_wave;
    grid = (uint32_t)((waves * 64 + threads - 1) / threads);
  } else {
    grid = h->num_cus * h->doall_wgs_per_cu;
  }
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    auto go = [&](auto kernel) {
      launch_timed(h, Method::kKind, kernel, dim3(grid), dim3(threads), s, DevHeapW<kLG>(h->dev), type,
                   (const uint32_t*)eo.R, (const uint64_t*)eo.S, (const uint32_t*)&eo.st->count, args);
    };
    if constexpr (MinWaves<Method>::value > 1) {
      if (large_heap(h)) go(doall_kernel<Method, kLG, true>);
      else go(doall_kernel<Method, kLG, false>);
    } else {
      go(doall_kernel<Method, kLG, false>);
    }
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

// The do-all of Method over `type` and every type that inherits from it
// (Sec. 1.2): the method reads the inherited fields by the parent's field
// indices, which each subclass lays out in its own blocks.  Every type's
// list is enumerated before any method runs, so the do-all visits exactly
// the objects live when it starts; then one launch per type.
template <class Method>
int launch_doall_tree(dsoar_heap* h, uint32_t type, const typename Method::Args& args, uint32_t flags,
                      hipStream_t s) {
  if (type >= h->desc.num_types) return DSOAR_ERR_INVALID_ARG;
  const uint32_t mask = h->subtypes[type];
  if (mask == (1u << type)) return launch_doall<Method>(h, type, args, flags, s);
  if (!(flags & DSOAR_DO_REUSE_ENUM))
    for (uint32_t u = 0; u < h->desc.num_types; ++u)
      if ((mask >> u) & 1u) {
        const int rc = launch_enumerate(h, u, s);
        if (rc) return rc;
      }
  for (uint32_t u = 0; u < h->desc.num_types; ++u)
    if ((mask >> u) & 1u) {
      const int rc = launch_doall<Method>(h, u, args, flags | DSOAR_DO_REUSE_ENUM, s);
      if (rc) return rc;
    }
  return DSOAR_OK;
}

// Both do-alls of doall2_kernel, over the lists of their types' last
// enumerations (no enumeration here), persistent grid; timed as `kind`.
template <class M1, class M2>
int launch_doall2(dsoar_heap* h, uint32_t t1, const typename M1::Args& a1, uint32_t t2,
                  const typename M2::Args& a2, uint32_t kind, hipStream_t s) {
  if (t1 >= h->desc.num_types || t2 >= h->desc.num_types) return DSOAR_ERR_INVALID_ARG;
  const EnumOut& e1 = h->enum_out[t1];
  const EnumOut& e2 = h->enum_out[t2];
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    auto go = [&](auto kernel) {
      launch_timed(h, kind, kernel, dim3(h->num_cus * h->doall_wgs_per_cu), dim3(h->doall_wg_threads), s,
                   DevHeapW<kLG>(h->dev), t1, (const uint32_t*)e1.R, (const uint64_t*)e1.S,
                   (const uint32_t*)&e1.st->count, a1, t2, (const uint32_t*)e2.R, (const uint64_t*)e2.S,
                   (const uint32_t*)&e2.st->count, a2);
    };
    if constexpr (MinWaves<M1>::value > 1 || MinWaves<M2>::value > 1) {
      if (large_heap(h)) go(doall2_kernel<M1, M2, kLG, true>);
      else go(doall2_kernel<M1, M2, kLG, false>);
    } else {
      go(doall2_kernel<M1, M2, kLG, false>);
    }
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

// The HIP graphs of an application's step: one of a single step and one of
// kGraphSteps steps, captured on first use and replayed (a long run replays
// the longer one, so graph boundaries come kGraphSteps times less often);
// captured again when the heap's launch configuration changed since.
constexpr uint32_t kGraphSteps = 10;
struct StepGraphs {
  hipGraph_t graph[2];
  hipGraphExec_t exec[2];
  uint32_t epoch;
};

inline void step_graphs_clear(StepGraphs& g) {
  for (int i = 0; i < 2; ++i) {
    if (g.exec[i]) (void)hipGraphExecDestroy(g.exec[i]);
    if (g.graph[i]) (void)hipGraphDestroy(g.graph[i]);
    g.exec[i] = nullptr;
    g.graph[i] = nullptr;
  }
}

// Runs `steps` steps of one_step(stream) (a function returning a status)
// through the graphs.
template <class F>
int step_graphs_run(dsoar_heap* h, StepGraphs& g, uint32_t steps, hipStream_t s, F&& one_step) {
  if (g.exec[0] && g.epoch != h->config_epoch) step_graphs_clear(g);
  if (!g.exec[0]) {
    const uint32_t reps[2] = {1, kGraphSteps};
    for (int i = 0; i < 2; ++i) {
      DSOAR_HIP(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      int rc = DSOAR_OK;
      for (uint32_t k = 0; k < reps[i] && rc == DSOAR_OK; ++k) rc = one_step(s);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(s, &graph);
      if (rc != DSOAR_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        step_graphs_clear(g);
        return rc != DSOAR_OK ? rc : hip_fail(h, e);
      }
      g.graph[i] = graph;
      const hipError_t ie = hipGraphInstantiate(&g.exec[i], graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        step_graphs_clear(g);
        return hip_fail(h, ie);
      }
    }
    g.epoch = h->config_epoch;
  }
  uint32_t left = steps;
  for (; left >= kGraphSteps; left -= kGraphSteps) DSOAR_HIP(h, hipGraphLaunch(g.exec[1], s));
  for (; left > 0; --left) DSOAR_HIP(h, hipGraphLaunch(g.exec[0], s));
  return DSOAR_OK;
}

inline bool heap_ok(const dsoar_heap* h) { return h != nullptr && h->base != nullptr; }

}  // namespace dsoar
