// Device side of the object heap: hierarchical bitmaps (Sec. 3, Alg. 2),
// wavefront-aggregated new (Sec. 2.2 Alg. 1 + request coalescing, Sec. 2.4),
// delete, SOA field addressing (Sec. 2), for gfx950 wave64.
//
// Execution model.  Every heap operation here is a *wavefront* operation: it
// is called by the lanes of one wavefront that want it (any subset), runs in
// wave-uniform control flow, and issues its atomics from one leader lane,
// broadcasting results with readfirstlane.  A lane never spins on another
// lane of its own wavefront, so the retry loops of the paper's lock-free
// algorithms cannot deadlock under lockstep execution.
//
// Memory model.  Heap metadata (bitmap words, object bitmaps, block types) is
// only ever accessed atomically: read with agent-scope relaxed atomic loads
// (global_load ... sc1), written with agent-scope atomic stores or RMWs, in
// every kernel, also at quiescence.  The RMWs are performed where all eight
// XCDs see one order per word; a plain load could hit a line an XCD's own L2
// still holds from before those RMWs.
// The object bitmap word is the linearisation point (Sec. 2, "Concurrency");
// block-state bitmaps are eventually consistent hints.  No release/acquire
// fences are used: object fields written in one kernel are read in later
// kernels (kernel boundaries order them), and a method that deletes `this`
// must not write this's fields in the same call.  Where one metadata access
// must be performed before another (a block's publication, the pins of
// online reclamation), the wave waits for its accesses to complete
// (wait_performed) before it issues the next.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace dsoar {

constexpr uint32_t kMaxTypes = 8;
constexpr uint32_t kMaxFields = 8;
constexpr uint32_t kMaxLevels = 8;
constexpr uint32_t kNull = 0xFFFFFFFFu;
// Block type word: the type in the low 8 bits (kTypeNone for a free block),
// above them the number of times the block was freed (its version).
constexpr uint32_t kTypeNone = 0xFFu;
constexpr int32_t kFail = -1;
constexpr uint32_t kSpinLimit = 1u << 20;  // bound of every retry loop
constexpr uint32_t kShards = 1024;         // counter shards (spread atomics)
// s_waitcnt immediate for gfx9-family encodings: vmcnt 0 (bits 3:0 and
// 15:14), expcnt 7 (bits 6:4) and lgkmcnt 15 (bits 11:8) left unconstrained.
constexpr int kWaitVmem = 0x0F70;
constexpr uint32_t kBoundedPasses = 2;  // active lookups per request under the bounded policy
constexpr uint32_t kMultiBlocks = 8;  // active blocks one lookup may reserve in
// Where a wavefront's bitmap searches start (C8: any set bit may be taken):
// a hash of the wavefront's index (searches spread over the whole bitmap),
// the lowest set bit at every level (the oracle's choice), or a hash whose
// top-level digit names one eighth of the top container per XCD (the eight
// XCDs mostly search disjoint parts of the heap).
enum : uint32_t { kStartHashed = 0, kStartLowest = 1, kStartXcd = 2 };
// Rounds a request keeps waiting while the free-block count says a block is
// free or being opened but neither lookup finds one (a summary bit still on
// its way); then it gives up with the retry-limit flag.
constexpr uint32_t kFreeWaitLimit = 1u << 12;

// Control words (uint64 array at DevHeap::ctrl).
enum : uint32_t {
  kCtlOom = 0,
  kCtlRetryLimit = 1,
  kCtlDoubleFree = 2,
  kCtlWords = 8,
  // Counter shards follow: shard s occupies kCtlWords + s*kShardStride ...
  kCntAllocs = 0,                  // + type
  kCntFrees = kMaxTypes,           // + type
  kCntReserveRetries = 2 * kMaxTypes,
  kCntSlowPaths = 2 * kMaxTypes + 1,
  kCntFindFails = 2 * kMaxTypes + 2,
  kCntVisits = 2 * kMaxTypes + 3,  // + type: objects visited by do-alls
  kCntMethodAtomics = 3 * kMaxTypes + 3,  // atomic RMWs methods issue on their own data
  kCntReleases = 3 * kMaxTypes + 4,       // blocks freed online by the delete that emptied them
  // The free-block count: blocks taken from the free bitmap (counted once the
  // request that took them has made them findable) and blocks returned to it
  // (counted before their free bit is set).  Both only grow.
  kCntBlocksTaken = 3 * kMaxTypes + 5,
  kCntBlocksReturned = 3 * kMaxTypes + 6,
  kShardStride = 32,
};
static_assert(kCntBlocksReturned < kShardStride, "counter slots exceed a shard");


struct DevHeap {
  uint8_t* data;            // M * block_stride bytes of SOA segments
  uint64_t* obj_bitmap;     // M words: bit s = slot s holds an object
  uint32_t* block_type;     // M words: version << 8 | type (kTypeNone if free)
  uint32_t* pins;           // M words: reservations in progress (online reclamation only)
  uint32_t* bitmaps;        // (1 + 2T) hierarchical bitmaps, bm_units apart
  uint64_t* ctrl;           // flags + counter shards
  uint64_t block_stride;
  uint64_t cap_mask[kMaxTypes];  // per type: low `capacity` bits
  uint32_t capacity[kMaxTypes];  // per type: slots per block, a power of two <= 64
  uint32_t num_blocks;
  uint32_t num_types;
  uint32_t nlevels;
  uint32_t bm_lg;           // log2 of the bitmap container width (6 or 5)
  uint32_t bm_units;        // 32-bit units per bitmap (all levels, padded)
  uint32_t bm_off[kMaxLevels];  // unit offset of each level in a bitmap
  uint32_t search_start;    // kStartHashed, kStartLowest or kStartXcd
  uint32_t bulk_min;        // requests of at least this many take whole free blocks
  uint32_t fresh_types;     // bit t: requests of type t skip the active lookup
  uint32_t bounded_types;   // bit t: at most kBoundedPasses active lookups per request of type t
  uint32_t doall_unroll;    // blocks per wavefront pass of split do-alls (1, 2, 4, 8)
  uint32_t online_reclaim;  // 1: the delete that empties a block frees it at once
  // Field f of type t: byte offset of its array in a block (low 24 bits)
  // and log2 of its width (high 8 bits), in one dword so that a kernel reads
  // it with one scalar load.
  uint32_t field_loc[kMaxTypes][kMaxFields];
};

// A heap whose bitmap container width is known when the kernel is compiled:
// the same data as DevHeap, with the width also a constant of the type.
// Every device function of the heap takes its heap as a template parameter,
// so a kernel that receives a DevHeapW<LG> runs code in which every width
// test has folded away (as lean as if the heap had one width), while one
// that receives a plain DevHeap reads the width at run time.
template <uint32_t LG>
struct DevHeapW : DevHeap {
  static_assert(LG == 5 || LG == 6, "containers are 32 or 64 bits");
  static constexpr uint32_t kLG = LG;
  DevHeapW() = default;
  __host__ __device__ explicit DevHeapW(const DevHeap& d) : DevHeap(d) {}
};

template <class H, class = void>
struct HasFixedWidth : std::false_type {};
template <class H>
struct HasFixedWidth<H, std::void_t<decltype(H::kLG)>> : std::true_type {};

// log2 of the heap's container width: the type's constant when it has one.
template <class H>
__device__ __forceinline__ uint32_t heap_lg(const H& h) {
  if constexpr (HasFixedWidth<H>::value)
    return H::kLG;
  else
    return h.bm_lg;
}

// ------------------------------------------------------------ wave helpers --

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t active_mask() { return __ballot(1); }

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t bcast32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t bcast64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool is_first_active() {
  return lane_id() == (uint32_t)(__ffsll((unsigned long long)active_mask()) - 1);
}

// Position of the k-th (0-based) set bit of m; m must have more than k bits.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t k) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t w = 32; w >= 1; w >>= 1) {
    uint32_t c = __popcll(m & ((1ull << w) - 1));
    if (k >= c) {
      k -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// Lowest n set bits of m (n <= popcount(m)).
__device__ __forceinline__ uint64_t lowest_bits(uint64_t m, uint32_t n) {
  if (n >= (uint32_t)__popcll(m)) return m;
  if (n == 0) return 0;
  uint32_t p = nth_set_bit(m, n);  // first bit not taken
  return m & ((1ull << p) - 1);
}

// OR of (1 << slot) over the lanes in `lanes` (all of them active); reads
// each lane with readlane, so inactive lanes of a divergent caller are never
// touched.
__device__ __forceinline__ uint64_t slots_of(uint64_t lanes, uint32_t slot) {
  uint64_t m = 0;
  while (lanes) {
    const uint32_t l = (uint32_t)__builtin_ctzll(lanes);
    m |= 1ull << (__builtin_amdgcn_readlane(slot, l) & 63u);
    lanes &= lanes - 1;
  }
  return m;
}

// The n set bits of m found by scanning upwards from bit r and wrapping
// (n <= popcount(m), r < 64).  Wavefronts that start at different r take
// disjoint slots of the same block more often.
__device__ __forceinline__ uint64_t take_from(uint64_t m, uint32_t n, uint32_t r) {
  const uint64_t below = (1ull << r) - 1;
  const uint64_t hi = m & ~below;
  const uint32_t c = (uint32_t)__popcll(hi);
  if (n <= c) return lowest_bits(hi, n);
  return hi | lowest_bits(m & below, n - c);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Stress builds (compiled with DSOAR_CHAOS): at each named race window a
// wavefront pauses, about one time in four, for a hash-chosen 0 to 7 sleeps
// of 63 x 64 cycles (up to about 12 us at 2.4 GHz), so that other
// wavefronts' atomics land inside windows that are otherwise a few cycles
// wide.  Every bounded wait of the heap allows milliseconds, so a pause never
// turns into a retry-limit error.  Release builds compile it away.
enum : uint32_t {
  kChaosFindReserve = 1,  // an active block's object bitmap read -> the reserving OR
  kChaosTakePublish,      // free blocks taken -> their object bitmaps and type words written
  kChaosPublishSets,      // new blocks published -> allocated / active bits set
  kChaosNested,           // a container's update -> the nested bit one level up
  kChaosDeleteActive,     // a full block's delete -> the block back in active
  kChaosRelease,          // online release: between its steps
};
__device__ __forceinline__ void chaos_pause(uint32_t site) {
#ifdef DSOAR_CHAOS
  const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane(
      (int)hash32((uint32_t)__builtin_readcyclecounter() ^ (site * 0x9E3779B9u) ^ (blockIdx.x << 6) ^
                  (threadIdx.x >> 6)));
  if ((r & 3u) != 0) return;
  for (uint32_t i = (r >> 2) & 7u; i > 0; --i) __builtin_amdgcn_s_sleep(63);
#else
  (void)site;
#endif
}

// ----------------------------------------------------------- memory access --

// Agent-coherent load, made wave-uniform.
__device__ __forceinline__ uint64_t load_u64(const uint64_t* p) {
  return bcast64(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Per-lane agent-scope loads and stores of heap metadata.
__device__ __forceinline__ uint64_t meta_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t meta_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void meta_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void meta_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t tw_type(uint32_t w) { return w & 0xFFu; }
__device__ __forceinline__ uint32_t tw_with(uint32_t w, uint32_t type) { return (w & ~0xFFu) | type; }
__device__ __forceinline__ uint32_t tw_freed(uint32_t w) { return (w & ~0xFFu) + 0x100u + kTypeNone; }

// Leader-issued RMWs; all calling lanes receive the previous value.
__device__ __forceinline__ uint64_t lead_or(uint64_t* p, uint64_t v) {
  uint64_t r = 0;
  if (is_first_active()) r = __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return bcast64(r);
}

__device__ __forceinline__ uint64_t lead_and(uint64_t* p, uint64_t v) {
  uint64_t r = 0;
  if (is_first_active()) r = __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return bcast64(r);
}

__device__ __forceinline__ void lead_add(uint64_t* p, uint64_t v) {
  if (is_first_active()) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lead_flag(uint64_t* p) {
  if (is_first_active()) __hip_atomic_store(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Counters are sharded by global wavefront index: same-address atomics
// serialise (about 0.1 G/s on one word against about 20 G/s spread out).
template <class H>
__device__ __forceinline__ uint64_t* shard(const H& h) {
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return h.ctrl + kCtlWords + (uint64_t)(wave & (kShards - 1)) * kShardStride;
}

// Blocks that are free or being opened, M + returned - taken, as of one
// instant.  Called by any subset of a wavefront's lanes (wave-uniform
// result).  The counts are spread over the counter shards; two collects of
// all shards whose totals agree saw the same values (each count only grows,
// and the second collect's loads are issued after the first one's have
// returned), so their sum is the state at the instant between them.
// Returns -1 when no two successive collects agreed (the counts are
// changing: blocks may be free).
template <class H>
__device__ inline int64_t free_block_count(const H& h) {
  const uint64_t am = active_mask();
  const uint32_t me = lanes_below(am), nact = (uint32_t)__popcll(am);
  uint64_t prev_sum = ~0ull;
  for (uint32_t round = 0; round < 8; ++round) {
    uint64_t taken = 0, returned = 0;
    for (uint32_t s = me; s < kShards; s += nact) {
      const uint64_t* sh = h.ctrl + kCtlWords + (uint64_t)s * kShardStride;
      taken += __hip_atomic_load(sh + kCntBlocksTaken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      returned += __hip_atomic_load(sh + kCntBlocksReturned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint64_t tt = 0, rr = 0;
    for (uint64_t m = am; m; m &= m - 1) {
      const uint32_t l = (uint32_t)__builtin_ctzll(m);
      tt += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(taken >> 32), l) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((uint32_t)taken, l);
      rr += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(returned >> 32), l) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((uint32_t)returned, l);
    }
    if (tt + rr == prev_sum) return (int64_t)h.num_blocks + (int64_t)rr - (int64_t)tt;
    prev_sum = tt + rr;
  }
  return -1;
}

// Adds the active lanes' counts (each below 256) to counter `slot` of this
// wavefront's shard with one atomic; exact under divergence (bit-sliced
// ballots).  For methods that report their own atomic operations.
template <class H>
__device__ inline void wave_count(const H& h, uint32_t slot, uint32_t k) {
  uint32_t n = 0;
#pragma unroll
  for (uint32_t b = 0; b < 8; ++b) n += (uint32_t)__popcll(__ballot((k >> b) & 1u)) << b;
  if (n) lead_add(shard(h) + slot, n);
}

// ------------------------------------------------------ hierarchical bitmap --
// Bitmap k of the heap: k = 0 free, 1 + 2t allocated[t], 2 + 2t active[t].
// A container is 2^lg bits, lg = 6 (64-bit containers) or 5 (32-bit ones),
// one choice per heap: the bitmap's fan-out.  Level l + 1 holds one bit per
// container of level l; the top level is one container (Sec. 3: a nested
// bitmap exists while a level has more bits than one container).
//
// Storage is in 32-bit units; level l is a plain bit array (bit j in unit
// j / 32) starting at an even unit, so a 64-bit container is two units.
// Level 0 is read and written only as 64-bit groups (bits [64g, 64g + 64)):
// one container at lg = 6, two at lg = 5, in one atomic; the containers of
// a group are then updated together and their nested bits one container at
// a time.  Block-indexed code thus works in groups of 64 blocks at either
// width.  Levels above 0 are accessed one container at a time.

// Bits of level l of a bitmap of nbits bits.
__host__ __device__ __forceinline__ uint32_t level_bits(uint32_t nbits, uint32_t lg, uint32_t l) {
  return ((nbits - 1) >> (lg * l)) + 1;
}
// Levels: a nested level exists while a level has more than 2^lg bits.
__host__ __device__ __forceinline__ uint32_t num_levels(uint32_t nbits, uint32_t lg) {
  uint32_t l = 1;
  while (level_bits(nbits, lg, l - 1) > (1u << lg)) ++l;
  return l;
}
// 32-bit units of a level of n bits (even, so that every level starts at an
// 8-byte boundary).
__host__ __device__ __forceinline__ uint32_t level_units(uint32_t n) { return (((n - 1) >> 6) + 1) * 2; }
// Unit offset of level l (levels stored bottom-up).
__host__ __device__ __forceinline__ uint32_t level_offset(uint32_t nbits, uint32_t lg, uint32_t l) {
  uint32_t off = 0;
  for (uint32_t k = 0; k < l; ++k) off += level_units(level_bits(nbits, lg, k));
  return off;
}

struct Bitmap {
  uint32_t* units;
  uint32_t nbits;
  uint32_t nlevels;
  uint32_t lg;  // log2 of the container width: 6 or 5
  uint64_t* retry_flag;
  const uint32_t* off;  // unit offset of each level (in the kernel's arguments)

  // 64-bit group g of level 0.
  __device__ __forceinline__ uint64_t* group(uint32_t g) const { return reinterpret_cast<uint64_t*>(units) + g; }
  __device__ __forceinline__ uint32_t* level(uint32_t l) const { return units + off[l]; }
  __device__ __forceinline__ uint32_t cmask() const { return (1u << lg) - 1u; }
};

template <class H>
__device__ __forceinline__ Bitmap heap_bitmap(const H& h, uint32_t k) {
  return Bitmap{h.bitmaps + (uint64_t)k * h.bm_units, h.num_blocks, h.nlevels, heap_lg(h), h.ctrl + kCtlRetryLimit,
                h.bm_off};
}
template <class H>
__device__ __forceinline__ Bitmap free_bm(const H& h) { return heap_bitmap(h, 0); }
template <class H>
__device__ __forceinline__ Bitmap allocated_bm(const H& h, uint32_t t) { return heap_bitmap(h, 1 + 2 * t); }
template <class H>
__device__ __forceinline__ Bitmap active_bm(const H& h, uint32_t t) { return heap_bitmap(h, 2 + 2 * t); }

// The container of level-0 bit `pos` inside the group value v that holds it.
__device__ __forceinline__ uint64_t group_part(const Bitmap& b, uint64_t v, uint32_t pos) {
  return __builtin_expect(b.lg == 6, 1) ? v : ((v >> (pos & 32u)) & 0xFFFFFFFFull);
}

// The 32-bit-container forms of the operations below are kept out of line:
// inlined beside the 64-bit forms at every call site they would lengthen the
// straight-line code each wavefront fetches, whatever width the heap uses.
__device__ inline uint64_t load_unit32(const uint32_t* p) {
  return bcast32(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Agent-coherent, wave-uniform load of container c of level l >= 1.
__device__ __forceinline__ uint64_t load_container(const Bitmap& b, uint32_t l, uint32_t c) {
  if (__builtin_expect(b.lg == 6, 1)) return load_u64(reinterpret_cast<const uint64_t*>(b.level(l)) + c);
  return load_unit32(b.level(l) + c);
}

// Top container (level nlevels - 1, container 0); with one level that is
// group 0 of level 0 (at lg = 5 its second container is always empty).
__device__ __forceinline__ uint64_t load_top(const Bitmap& b) {
  return b.nlevels == 1 ? load_u64(b.group(0)) : load_container(b, b.nlevels - 1, 0);
}

__device__ inline uint64_t bit_rmw32(uint32_t* w, uint32_t m, bool set) {
  uint32_t r = 0;
  if (is_first_active())
    r = set ? __hip_atomic_fetch_or(w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
            : __hip_atomic_fetch_and(w, ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return bcast32(r);
}

// One leader atomic on the bit `pos` of level `level` (OR when set, AND-NOT
// otherwise); returns the previous value of the bit's container.
__device__ __forceinline__ uint64_t bit_rmw(const Bitmap& b, uint32_t level, uint32_t pos, bool set) {
  if (__builtin_expect(level == 0 || b.lg == 6, 1)) {
    uint64_t* w = reinterpret_cast<uint64_t*>(b.level(level)) + (pos >> 6);
    const uint64_t m = 1ull << (pos & 63u);
    const uint64_t prev = set ? lead_or(w, m) : lead_and(w, ~m);
    return level == 0 ? group_part(b, prev, pos) : prev;
  }
  return bit_rmw32(b.level(level) + (pos >> 5), 1u << (pos & 31u), set);
}

// set(pos) / clear(pos) of Sec. 2.1: retry the try_ operation until it
// succeeds, then do the nested update this success made us responsible for
// (Alg. 2: the clear that empties a container clears its nested bit; the set
// that makes a container non-empty sets it).  Iterative, one level at a time.
// Returns false only if the retry limit was hit (sticky flag set).
__device__ inline bool bm_set_from(const Bitmap& b, uint32_t level, uint32_t pos) {
  for (;;) {
    const uint64_t bit = 1ull << (pos & b.cmask());
    uint64_t prev;
    uint32_t spins = 0;
    for (;;) {
      prev = bit_rmw(b, level, pos, true);
      if (!(prev & bit)) break;
      if (++spins >= kSpinLimit) {
        lead_flag(b.retry_flag);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (prev != 0 || level + 1 >= b.nlevels) return true;
    pos >>= b.lg;
    ++level;
    chaos_pause(kChaosNested);
  }
}

__device__ inline bool bm_clear_from(const Bitmap& b, uint32_t level, uint32_t pos) {
  for (;;) {
    const uint64_t bit = 1ull << (pos & b.cmask());
    uint64_t prev;
    uint32_t spins = 0;
    for (;;) {
      prev = bit_rmw(b, level, pos, false);
      if (prev & bit) break;
      if (++spins >= kSpinLimit) {
        lead_flag(b.retry_flag);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (__popcll(prev) != 1 || level + 1 >= b.nlevels) return true;
    pos >>= b.lg;
    ++level;
    chaos_pause(kChaosNested);
  }
}

__device__ __forceinline__ bool bm_set(const Bitmap& b, uint32_t pos) { return bm_set_from(b, 0, pos); }
__device__ __forceinline__ bool bm_clear(const Bitmap& b, uint32_t pos) { return bm_clear_from(b, 0, pos); }

// The nested updates that an OR of m into level-0 group g (previous value
// prev) makes: each container of the group that was empty and gained bits
// sets its bit one level up (set's cascade, Sec. 2.1).
__device__ inline void group_set_nested32(const Bitmap& b, uint32_t g, uint64_t prev, uint64_t m) {
  for (uint32_t half = 0; half < 2; ++half) {
    const uint64_t hm = 0xFFFFFFFFull << (32 * half);
    if ((m & hm) && !(prev & hm)) bm_set_from(b, 1, 2 * g + half);
  }
}
__device__ inline void group_set_nested(const Bitmap& b, uint32_t g, uint64_t prev, uint64_t m) {
  if (b.nlevels == 1) return;
  chaos_pause(kChaosNested);
  if (__builtin_expect(b.lg == 6, 1)) {
    if (prev == 0 && m) bm_set_from(b, 1, g);
    return;
  }
  group_set_nested32(b, g, prev, m);
}

// The nested updates that an AND-NOT of m on level-0 group g (previous value
// prev) makes: each container whose last set bits it removed clears its bit
// one level up (Alg. 2 for several bits at once).
__device__ inline void group_clear_nested32(const Bitmap& b, uint32_t g, uint64_t prev,
                                                               uint64_t m) {
  for (uint32_t half = 0; half < 2; ++half) {
    const uint64_t hm = 0xFFFFFFFFull << (32 * half);
    if ((prev & m & hm) && (prev & ~m & hm) == 0) bm_clear_from(b, 1, 2 * g + half);
  }
}
__device__ inline void group_clear_nested(const Bitmap& b, uint32_t g, uint64_t prev, uint64_t m) {
  if (b.nlevels == 1) return;
  chaos_pause(kChaosNested);
  if (__builtin_expect(b.lg == 6, 1)) {
    if ((prev & m) && (prev & ~m) == 0) bm_clear_from(b, 1, g);
    return;
  }
  group_clear_nested32(b, g, prev, m);
}

// One leader atomic on the bits m of container c of level l >= 1 (OR when
// set, AND-NOT otherwise); returns the container's previous value.
__device__ inline uint64_t container_rmw(const Bitmap& b, uint32_t l, uint32_t c, uint64_t m, bool set) {
  if (__builtin_expect(b.lg == 6, 1)) {
    uint64_t* w = reinterpret_cast<uint64_t*>(b.level(l)) + c;
    return set ? lead_or(w, m) : lead_and(w, ~m);
  }
  uint32_t* w = b.level(l) + c;
  uint32_t r = 0;
  if (is_first_active())
    r = set ? __hip_atomic_fetch_or(w, (uint32_t)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
            : __hip_atomic_fetch_and(w, ~(uint32_t)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return bcast32(r);
}

// set(pos) / clear(pos) of Sec. 2.1 for every bit of m in container c of
// level l >= 1, with one atomic: a container this made non-empty (empty)
// sets (clears) its bit one level up, and bits another operation holds are
// set (cleared) again one by one with the single-bit retry.
__device__ inline void bm_set_bits_at(const Bitmap& b, uint32_t l, uint32_t c, uint64_t m) {
  const uint64_t prev = container_rmw(b, l, c, m, true);
  if (prev == 0 && l + 1 < b.nlevels) bm_set_from(b, l + 1, c);
  uint64_t busy = prev & m;
  while (busy) {
    bm_set_from(b, l, (c << b.lg) + (uint32_t)__builtin_ctzll(busy));
    busy &= busy - 1;
  }
}
__device__ inline void bm_clear_bits_at(const Bitmap& b, uint32_t l, uint32_t c, uint64_t m) {
  const uint64_t prev = container_rmw(b, l, c, m, false);
  if ((prev & m) && (prev & ~m) == 0 && l + 1 < b.nlevels) bm_clear_from(b, l + 1, c);
  uint64_t busy = m & ~prev;
  while (busy) {
    bm_clear_from(b, l, (c << b.lg) + (uint32_t)__builtin_ctzll(busy));
    busy &= busy - 1;
  }
}

// set(pos) for every bit of m in level-0 group g, with one atomic OR when no
// other operation holds any of them: bits that were already set are set
// again one by one with set's retry, so each still pairs with the clear that
// is about to take it away.  A container that was empty sets its nested bit.
__device__ inline void bm_set_bits0(const Bitmap& b, uint32_t g, uint64_t m) {
  const uint64_t prev = lead_or(b.group(g), m);
  group_set_nested(b, g, prev, m & ~prev);
  uint64_t busy = prev & m;
  while (busy) {
    bm_set(b, g * 64 + (uint32_t)__builtin_ctzll(busy));
    busy &= busy - 1;
  }
}

// bm_set_bits0 in two halves, so that the wait for the OR's result can be
// put off: _issue returns the previous group in the leader lane only (call
// both halves with the same lanes active), _settle finishes the operation.
__device__ __forceinline__ uint64_t bm_set_bits0_issue(const Bitmap& b, uint32_t g, uint64_t m) {
  uint64_t r = 0;
  if (is_first_active()) r = __hip_atomic_fetch_or(b.group(g), m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return r;
}
__device__ inline void bm_set_bits0_settle(const Bitmap& b, uint32_t g, uint64_t m, uint64_t leader_prev) {
  const uint64_t prev = bcast64(leader_prev);
  group_set_nested(b, g, prev, m & ~prev);
  uint64_t busy = prev & m;
  while (busy) {
    bm_set(b, g * 64 + (uint32_t)__builtin_ctzll(busy));
    busy &= busy - 1;
  }
}

// clear(pos) for every bit of m in level-0 group g: one atomic AND; bits
// that were not set yet (their set is still on its way) are cleared one by
// one with clear's retry.  A container this AND emptied clears its nested
// bit (Alg. 2 for several bits at once).
__device__ inline void bm_clear_bits0(const Bitmap& b, uint32_t g, uint64_t m) {
  const uint64_t prev = lead_and(b.group(g), ~m);
  group_clear_nested(b, g, prev, m);
  uint64_t busy = m & ~prev;
  while (busy) {
    bm_clear(b, g * 64 + (uint32_t)__builtin_ctzll(busy));
    busy &= busy - 1;
  }
}

// try_set(pos): one atomic OR; on success from an empty container, set the
// nested bit (retrying).
__device__ inline bool bm_try_set(const Bitmap& b, uint32_t pos) {
  const uint64_t bit = 1ull << (pos & 63u);
  const uint64_t prev = lead_or(b.group(pos >> 6), bit);
  const bool ok = !(prev & bit);
  if (ok && group_part(b, prev, pos) == 0 && b.nlevels > 1) bm_set_from(b, 1, pos >> b.lg);
  return ok;
}

// Alg. 2, try_clear(pos): one atomic AND; success if the bit was set; if this
// cleared the container's last bit, clear the nested bit (retrying).
__device__ inline bool bm_try_clear(const Bitmap& b, uint32_t pos) {
  const uint64_t bit = 1ull << (pos & 63u);
  const uint64_t prev = lead_and(b.group(pos >> 6), ~bit);
  const bool ok = (prev & bit) != 0;
  if (ok && __popcll(group_part(b, prev, pos)) == 1 && b.nlevels > 1) bm_clear_from(b, 1, pos >> b.lg);
  return ok;
}

// The set bit of w (w != 0) that an lg-bit digit d selects: the
// floor(d * popcount / 2^lg)-th one, so digits spread evenly over the set
// bits whatever their positions (a plain "first set bit at or after d" would
// send every digit beyond the last set bit to the first one).
__device__ __forceinline__ uint32_t pick_bit(uint64_t w, uint32_t d, uint32_t lg) {
  return nth_set_bit(w, (d * (uint32_t)__popcll(w)) >> lg);
}

// The digit of `start` that chooses among the set bits at level l.
__device__ __forceinline__ uint32_t level_digit(uint32_t start, uint32_t l, uint32_t lg) {
  const uint32_t sh = lg * l;  // at most 6 * 7: the digits wrap round after 30 bits
  return (start >> (sh >= 30 ? sh - 30 : sh)) & ((1u << lg) - 1u);
}

// First container of a descent.  With three or more levels the search starts
// one level below the top, at the container that `start`'s top digit names
// among that level's containers, and reads the top container only if that
// one is empty: the top container is the bitmap's most contended word, and
// a bitmap with set bits usually has few empty containers one level down.
// Either way the descent goes on from a non-empty container, so it still
// finds a set bit when there is one.  False: the whole bitmap reads empty.
__device__ inline bool bm_descend_start(const Bitmap& b, uint32_t start, uint32_t* level, uint32_t* idx,
                                        uint64_t* w) {
  const uint32_t top = b.nlevels - 1;
  if (top >= 2) {
    const uint32_t nc = level_bits(b.nbits, b.lg, top);  // containers one level below the top
    const uint32_t i = (level_digit(start, top, b.lg) * nc) >> b.lg;
    const uint64_t v = load_container(b, top - 1, i);
    if (v != 0) {
      *level = top - 1;
      *idx = i;
      *w = v;
      return true;
    }
  }
  const uint64_t v = load_top(b);
  *level = top;
  *idx = 0;
  *w = v;
  return v != 0;
}

// try_find_set() stopped one level early: the index of a non-empty level-0
// group (chosen as try_find_set chooses) and its bits, or FAIL.  One load per
// level (a logarithmic number of accesses, Sec. 2.4); at each level the
// digit of `start` for that level picks one of the container's set bits, so
// concurrent searches with different starts spread over the whole bitmap.
// An empty container on the way down means the summary is momentarily ahead
// of it: FAIL.
__device__ inline int32_t bm_find_word(const Bitmap& b, uint32_t start, uint64_t* bits) {
  uint32_t l, idx;
  uint64_t w;
  if (!bm_descend_start(b, start, &l, &idx, &w)) return kFail;
  if (l == 0) {  // a single level: the top is group 0
    *bits = w;
    return 0;
  }
  while (l > 1) {
    idx = (idx << b.lg) | pick_bit(w, level_digit(start, l, b.lg), b.lg);
    --l;
    w = load_container(b, l, idx);
    if (w == 0) return kFail;
  }
  // Level 1 -> a container of level 0, read with its group.
  idx = (idx << b.lg) | pick_bit(w, level_digit(start, 1, b.lg), b.lg);
  const uint32_t g = idx >> (6 - b.lg);
  w = load_u64(b.group(g));
  if (w == 0) return kFail;
  *bits = w;
  return (int32_t)g;
}

// try_find_set(): descend to a non-empty level-0 group and pick one of its
// set bits with the digit of `start` for level 0.
__device__ inline int32_t bm_try_find_set(const Bitmap& b, uint32_t start) {
  uint64_t w = 0;
  const int32_t g = bm_find_word(b, start, &w);
  if (g == kFail) return kFail;
  const uint32_t idx = ((uint32_t)g << 6) | pick_bit(w, level_digit(start, 0, 6), 6);
  return idx < b.nbits ? (int32_t)idx : kFail;
}

// clear() of Sec. 2.1: find a set bit and clear it, repeating until this
// wavefront's clear succeeds.  FAIL when the top container reads empty.
// That does not prove the bitmap empty: with online reclamation a released
// block's level-0 bit is set before its upper levels, so the top can read 0
// while a bit is set below it.  The caller decides out of memory by the
// free-block count, not by this FAIL.
// `hint` (optional) names a level-0 group to try first, one load and no
// descent; a hint whose group reads empty or is out of range costs that load.
__device__ inline int32_t bm_find_clear(const Bitmap& b, uint32_t start, uint32_t hint = kNull) {
  if (hint < ((b.nbits + 63) >> 6)) {
    const uint64_t w = load_u64(b.group(hint));
    if (w) {
      const uint32_t i = (hint << 6) | pick_bit(w, level_digit(start, 0, 6), 6);
      if (i < b.nbits && bm_try_clear(b, i)) return (int32_t)i;
    }
  }
  for (uint32_t spins = 0; spins < kSpinLimit; ++spins) {
    const int32_t i = bm_try_find_set(b, start);
    if (i != kFail && bm_try_clear(b, (uint32_t)i)) return i;
    if (i == kFail && load_top(b) == 0) return kFail;
    start = hash32(start + 0x9e3779b9u + spins);
  }
  lead_flag(b.retry_flag);
  return kFail;
}

// Takes up to `want` (1..64) set bits of one level-0 group of a bitmap that
// is only cleared during kernels (the free bitmap): descend as try_find_set
// to a non-empty group, clear the chosen bits with one atomic AND, and clear
// the nested bits of the containers this emptied (Alg. 2 for several bits at
// once).  Returns the bits gained (0 = the bitmap reads empty) and the group
// in *word.
// `hint` as for bm_find_clear.
__device__ inline uint64_t bm_take_word(const Bitmap& b, uint32_t start, uint32_t want, uint32_t* word,
                                        uint32_t hint = kNull) {
  for (uint32_t spins = 0; spins < kSpinLimit; ++spins) {
    uint64_t w = 0;
    int32_t found = kFail;
    if (spins == 0 && hint < ((b.nbits + 63) >> 6)) {
      w = load_u64(b.group(hint));
      if (w) found = (int32_t)hint;
    }
    if (found == kFail) found = bm_find_word(b, start, &w);
    const uint32_t idx = found == kFail ? 0u : (uint32_t)found;
    if (found != kFail) {
      const uint64_t take = take_from(w, want < (uint32_t)__popcll(w) ? want : (uint32_t)__popcll(w), start & 63u);
      const uint64_t prev = lead_and(b.group(idx), ~take);
      const uint64_t got = prev & take;
      if (got) group_clear_nested(b, idx, prev, got);
      if (got) {
        *word = idx;
        return got;
      }
    } else if (load_top(b) == 0) {
      return 0;
    }
    start = hash32(start + 0x9e3779b9u + spins);
  }
  lead_flag(b.retry_flag);
  return 0;
}

// ------------------------------------------------------------------ objects --

__device__ __forceinline__ uint32_t obj_block(uint32_t obj) { return obj >> 6; }
__device__ __forceinline__ uint32_t obj_slot(uint32_t obj) { return obj & 63u; }
__device__ __forceinline__ uint32_t make_obj(uint32_t block, uint32_t slot) { return (block << 6) | slot; }

// Slots per block and the mask of valid object-bitmap bits of a type (the
// type must be wave-uniform: read with scalar loads).
template <class H>
__device__ __forceinline__ uint32_t cap_of(const H& h, uint32_t type) {
  return h.capacity[__builtin_amdgcn_readfirstlane(type)];
}
template <class H>
__device__ __forceinline__ uint64_t capmask_of(const H& h, uint32_t type) {
  return h.cap_mask[__builtin_amdgcn_readfirstlane(type)];
}

// Address of field `field` of object `obj` of type `type` (SOA: the field's
// array inside the object's block, indexed by slot).  type and field must be
// wave-uniform; they are read into scalar registers so that the layout table
// is fetched with scalar loads, which never wait on the vector loads in flight.
template <class F, class H>
__device__ __forceinline__ F* field_ptr(const H& h, uint32_t obj, uint32_t type, uint32_t field) {
  const uint32_t t = __builtin_amdgcn_readfirstlane(type), f = __builtin_amdgcn_readfirstlane(field);
  const uint32_t loc = h.field_loc[t][f];
  return reinterpret_cast<F*>(h.data + (uint64_t)obj_block(obj) * h.block_stride + (loc & 0xFFFFFFu) +
                              ((uint64_t)obj_slot(obj) << (loc >> 24)));
}

// Waits until every memory access this wave has issued has completed; for
// the agent-scope atomics of the heap metadata that means performed where all
// XCDs see them.  The signal fences keep the compiler from moving memory
// accesses across the wait.  Every ordering the allocator needs is between
// such atomics, so this wait is what it uses instead of release / acquire
// fences, which on this part also write back or invalidate the XCD's whole L2
// (needed only for plain stores and loads).
__device__ __forceinline__ void wait_performed() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(kWaitVmem);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Reservation side of online reclamation: pin block `bid` (per lane) if its
// type word still reads `w`; false (and no pin held) otherwise.  The pin is
// performed before the type word is read again, and the releaser's type-word
// store before it reads the pins, so at least one of the two sees the other.
template <class H>
__device__ __forceinline__ bool pin_block(const H& h, uint32_t bid, uint32_t w) {
  __hip_atomic_fetch_add(h.pins + bid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wait_performed();
  if (__hip_atomic_load(h.block_type + bid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == w) return true;
  __hip_atomic_fetch_sub(h.pins + bid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return false;
}
// The reservation made under the pin is performed before the pin goes.
template <class H>
__device__ __forceinline__ void unpin_block(const H& h, uint32_t bid) {
  wait_performed();
  __hip_atomic_fetch_sub(h.pins + bid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A block just taken from the free bitmap: its object bitmap first, then its
// type word, so that a reservation that reads the new type word also reads the
// initialised bitmap, and the bitmap complete before the allocated / active
// sets that follow make the block findable (else a reservation's OR could
// land before it and be overwritten).  Per lane.  The type word is read only
// after the free-bitmap update that handed the block over has returned (the
// block id comes from it), so with online reclamation it reads the version
// the releaser stored before it set the free bit.
template <class H>
__device__ __forceinline__ uint32_t publish_block(const H& h, uint32_t bid, uint32_t type, uint64_t bits) {
  const uint32_t w = tw_with(__hip_atomic_load(h.block_type + bid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), type);
  __hip_atomic_store(h.obj_bitmap + bid, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wait_performed();
  __hip_atomic_store(h.block_type + bid, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return w;
}

// Per-wavefront search hints in LDS, kept across the allocation requests a
// wavefront makes within one kernel: slot kMaxTypes holds the level-0 group
// of the free bitmap where it last took blocks, slot t the group of
// active[t] where it last found a block with room.  A hint only replaces a
// descent: its group is read again and used only if it still has set bits,
// so a stale or never-written value costs one load.
__device__ __forceinline__ uint32_t* wave_hints() {
  __shared__ uint32_t s_hints[16 * (kMaxTypes + 1)];
  return s_hints + ((threadIdx.x >> 6) & 15u) * (kMaxTypes + 1);
}

// Start value of this wavefront's bitmap searches (and slot rotation) under
// the heap's search-start policy.  Workgroups are dispatched to the eight
// XCDs round-robin, so blockIdx.x mod 8 is the XCD.
template <class H>
__device__ __forceinline__ uint32_t search_start(const H& h) {
  if (h.search_start == kStartLowest) return 0u;
  const uint32_t r = bcast32(hash32((blockIdx.x << 5) ^ (threadIdx.x >> 6) ^ 0x5bd1e995u));
  if (h.search_start != kStartXcd) return r;
  const uint32_t lg = heap_lg(h);
  const uint32_t tsh = lg * (h.nlevels - 1);
  const uint32_t sh = tsh >= 30 ? tsh - 30 : tsh;  // the top level's digit (as level_digit)
  const uint32_t span = (1u << lg) >> 3;                  // an eighth of its values
  const uint32_t digit = (blockIdx.x & 7u) * span + ((r >> sh) & (span - 1u));
  return (r & ~(((1u << lg) - 1u) << sh)) | (digit << sh);
}

// Alg. 1 for all lanes of this wavefront that call it with the same `type`
// (the caller guarantees a wave-uniform type); lane i asks for k_i objects
// (0 <= k_i < 256).  f(j, obj) is then called by lane i for j = 0 .. k_i - 1
// with its j-th new handle, or kNull if the heap ran out of free blocks
// (sticky OOM flag set).  f must not itself call wavefront heap operations.
//
// Request coalescing (Sec. 2.4): the n = sum k_i requests of the wavefront
// are served together, one leader lane issuing every atomic.  A pass looks
// up an active block of the type first (dense policy, Sec. 2.2) and takes a
// free block only when none is found (slow path: set the type, mark it
// allocated and, unless this pass fills it, active).  Once no active block
// was found, and while at least `capacity` requests remain, a pass takes
// whole free blocks, several at once from one free-bitmap word (full blocks
// are dense by construction).  With bulk_min set, requests of at least that
// many skip the active lookup and take whole free blocks directly.
// Reservation in an active block is one atomic OR of the wanted number of
// bits among those a snapshot shows free (after our own OR, the bits it left
// free); the bits gained are take & ~prev, and a block that still has room is
// used again without a new lookup.  The pass
// whose OR fills the block clears active[type] (Alg. 1, FULL).
// Requests are numbered by lane order (exclusive prefix sums from bit-sliced
// ballots, exact under any divergence) and handed out in that order.
template <class F, class H>
__device__ __forceinline__ void new_many(const H& h, uint32_t type, uint32_t k, F&& f) {
  uint32_t prefix = 0, n = 0;
#pragma unroll
  for (uint32_t b = 0; b < 8; ++b) {
    const uint64_t m = __ballot((k >> b) & 1u);
    prefix += lanes_below(m) << b;
    n += (uint32_t)__popcll(m) << b;
  }
  if (n == 0) return;
  const Bitmap active = active_bm(h, type);
  const uint32_t rot = search_start(h);
  const uint32_t c = cap_of(h, type);
  const uint64_t cap = capmask_of(h, type);
  uint32_t start = rot;
  uint32_t served = 0, retries = 0, slow = 0, fails = 0, oom_rounds = 0, wait_rounds = 0;
  bool oom = false, gave_up = false, active_first = false, none_active = false;
  int32_t cur = kFail;     // block of the last reservation, if it still had room
  uint64_t cur_avail = 0;  // its free bits right after that reservation
  uint32_t cur_tw = 0;     // its type word then (online reclamation: checked on reuse)
  // A type with the fresh policy looks for active blocks only once no free
  // block is left (active_first); until then the request goes on as if the
  // lookup had found none.
  const bool fresh = (h.fresh_types >> type) & 1u;
  if (fresh) none_active = true;
  // The bounded policy stops looking for active blocks after kBoundedPasses
  // lookups (until no free block is left).
  const uint32_t max_lookups = (h.bounded_types >> type) & 1u ? kBoundedPasses : kSpinLimit;
  uint32_t lookups = 0;
  uint32_t* const hints = wave_hints();
  uint32_t free_hint = bcast32(hints[kMaxTypes]), act_hint = bcast32(hints[type]);
  const uint32_t groups = (h.num_blocks + 63) >> 6;
  for (uint32_t it = 0; served < n; ++it) {
    if (it >= kSpinLimit) {
      lead_flag(h.ctrl + kCtlRetryLimit);
      gave_up = true;  // hand NULL to the lanes still waiting
      break;
    }
    const uint32_t want = n - served;
    if (want >= c && (want >= h.bulk_min || none_active) && !active_first) {
      // Whole free blocks, several from one free-bitmap word per atomic.  A
      // type with the fresh policy would open a block of its own for the
      // rest of the request right after: that block is taken in the same
      // atomic and published holding only the rest (and marked active).
      uint32_t word = 0;
      const uint32_t full = want / c, rest = want - full * c;
      const bool with_rest = fresh && rest != 0 && full < 64;
      const uint32_t nb = full < 64 ? full + (with_rest ? 1u : 0u) : 64u;
      const uint64_t blocks = bm_take_word(free_bm(h), start, nb, &word, free_hint);
      if (blocks == 0) {
        active_first = true;  // no free block: use space left in active blocks
        continue;
      }
      free_hint = word;
      chaos_pause(kChaosTakePublish);
      const uint32_t cnt_b = (uint32_t)__popcll(blocks);
      // With fewer blocks than asked for, all of them are filled.
      const bool partial = with_rest && cnt_b == nb;
      const uint64_t rest_bits = (1ull << rest) - 1;  // rest < c <= 64
      // Type words and object bitmaps of the new blocks, spread over the
      // active lanes; the blocks are ours alone until published.
      const uint64_t am = active_mask();
      const uint32_t me = lanes_below(am), nact = (uint32_t)__popcll(am);
      uint32_t my_tw = 0;
      for (uint32_t j = me; j < cnt_b; j += nact) {
        const bool last = partial && j + 1 == cnt_b;
        const uint32_t w = publish_block(h, word * 64 + nth_set_bit(blocks, j), type, last ? rest_bits : cap);
        if (last) my_tw = w;
      }
      chaos_pause(kChaosPublishSets);
      const Bitmap alloc = allocated_bm(h, type);
      const uint64_t pa = lead_or(alloc.group(word), blocks);
      group_set_nested(alloc, word, pa, blocks & ~pa);
      uint32_t span = cnt_b * c;
      if (partial) {
        // The block holding the rest stays findable for later requests.
        const uint32_t lb = nth_set_bit(blocks, cnt_b - 1);
        bm_set_bits0(active, word, 1ull << lb);
        cur = (int32_t)(word * 64 + lb);
        cur_avail = ~rest_bits & cap;
        cur_tw = (uint32_t)__builtin_amdgcn_readlane(my_tw, nth_set_bit(am, (cnt_b - 1) % nact));
        span = (cnt_b - 1) * c + rest;
      }
      // Counted as taken once nothing of them is left to publish.
      lead_add(shard(h) + kCntBlocksTaken, cnt_b);
      slow += cnt_b;
      const uint32_t lo = prefix > served ? prefix : served;
      const uint32_t hi = prefix + k < served + span ? prefix + k : served + span;
      for (uint32_t r = lo; r < hi; ++r) {
        const uint32_t q = r - served;
        f(r - prefix, make_obj(word * 64 + nth_set_bit(blocks, q / c), q % c));
      }
      served += span;
      continue;
    }
    int32_t bid = cur;
    uint64_t avail = cur_avail;
    uint64_t got;
    if (bid == kFail && (active_first || (!fresh && lookups < max_lookups))) {
      ++lookups;
      uint64_t wbits = 0;
      int32_t aw = kFail;
      if (lookups == 1 && act_hint < groups) {  // where this wavefront last found room
        wbits = load_u64(active.group(act_hint));
        if (wbits) aw = (int32_t)act_hint;
      }
      if (aw == kFail) aw = bm_find_word(active, start, &wbits);
      if (aw == kFail) {
        ++fails;
        // No active block: whole free blocks for the rest while it fills them.
        none_active = true;
        if (want >= c && !active_first) continue;
      } else {
        // Up to kMultiBlocks active blocks of this word, one active lane per
        // block: their object bitmaps are read and reserved in parallel, so a
        // request larger than one block's room costs one lookup, not one per
        // block.  Requests are spread over the blocks in rank order.
        const uint64_t am = active_mask();
        const uint32_t me = lanes_below(am), nact = (uint32_t)__popcll(am);
        uint32_t nb = (uint32_t)__popcll(wbits);
        nb = nb < kMultiBlocks ? nb : kMultiBlocks;
        nb = nb < nact ? nb : nact;
        const uint64_t sel = take_from(wbits, nb, start & 63u);
        uint32_t my_bid = 0, my_tw = 0;
        uint64_t my_av = 0;
        bool my_pin = false;
        if (me < nb) {
          my_bid = (uint32_t)aw * 64 + nth_set_bit(sel, me);
          bool ok = my_bid < h.num_blocks;
          if (ok && h.online_reclaim) {
            // The block may have been freed and reused since the lookup:
            // reserve only while pinned to the type word read now.
            my_tw = meta_load(h.block_type + my_bid);
            ok = tw_type(my_tw) == type && pin_block(h, my_bid, my_tw);
            my_pin = ok;
          }
          if (ok) my_av = ~meta_load(h.obj_bitmap + my_bid) & cap;
        }
        chaos_pause(kChaosFindReserve);
        const uint32_t cnt = (uint32_t)__popcll(my_av);
        uint32_t excl = 0;
#pragma unroll
        for (uint32_t b = 0; b < 7; ++b) excl += lanes_below(__ballot((cnt >> b) & 1u)) << b;
        const uint32_t my_t = want > excl ? (cnt < want - excl ? cnt : want - excl) : 0u;
        const uint64_t my_take = my_t ? take_from(my_av, my_t, rot & (c - 1)) : 0ull;
        uint64_t my_prev = 0;
        if (my_take)
          my_prev = __hip_atomic_fetch_or(h.obj_bitmap + my_bid, my_take, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (my_pin) unpin_block(h, my_bid);
        const uint64_t my_got = my_take & ~my_prev;
        const uint64_t my_after = (my_prev | my_take) & cap;
        // The reservation that set a block's last free bit takes it out of active.
        const uint64_t fill_lanes = __ballot(my_take && my_after == cap && (my_prev & cap) != cap);
        if (fill_lanes) bm_clear_bits0(active, (uint32_t)aw, slots_of(fill_lanes, my_bid & 63u));
        if (__ballot(my_got != my_take)) ++retries;
        const uint64_t room_lanes = __ballot(my_take && my_after != cap);
        if (room_lanes) {
          const uint32_t l = 63u - (uint32_t)__builtin_clzll(room_lanes);
          cur = (int32_t)__builtin_amdgcn_readlane(my_bid, l);
          cur_tw = (uint32_t)__builtin_amdgcn_readlane(my_tw, l);
          cur_avail = ~(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(my_after >> 32), l) << 32) |
                        (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)my_after, l)) &
                      cap;
        }
        // Hand the gained slots out, block by block in rank order.
        uint64_t lanes = __ballot(me < nb);
        uint32_t gained = 0;
        while (lanes) {
          const uint32_t l = (uint32_t)__builtin_ctzll(lanes);
          lanes &= lanes - 1;
          const uint64_t g = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(my_got >> 32), l) << 32) |
                             (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)my_got, l);
          if (!g) continue;
          const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane(my_bid, l);
          const uint32_t gc = (uint32_t)__popcll(g);
          const uint32_t lo = prefix > served ? prefix : served;
          const uint32_t hi = prefix + k < served + gc ? prefix + k : served + gc;
          for (uint32_t r = lo; r < hi; ++r) f(r - prefix, make_obj(gb, nth_set_bit(g, r - served)));
          served += gc;
          gained += gc;
        }
        if (gained) act_hint = (uint32_t)aw;
        if (gained == 0 && cur == kFail) start = hash32(start + it + 1);
        continue;
      }
    }
    cur = kFail;
    if (bid == kFail) {
      bid = bm_find_clear(free_bm(h), start, free_hint);
      if (bid != kFail) free_hint = (uint32_t)bid >> 6;
      if (bid == kFail) {
        // The free bitmap reads empty.  Out of memory only when the free-block
        // count (free blocks and blocks other wavefronts are still opening)
        // reads 0 twice with a failed active lookup in between: a request
        // fails only when no block has room (Sec. 2.2).
        const int64_t nfree = free_block_count(h);
        active_first = true;
        start = hash32(start + it + 1);
        if (nfree != 0) {
          // A block is free or about to become findable: look again.
          if (++wait_rounds >= kFreeWaitLimit) {
            lead_flag(h.ctrl + kCtlRetryLimit);
            gave_up = true;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
          continue;
        }
        if (++oom_rounds < 2) continue;
        oom = true;
        break;
      }
      ++slow;
      chaos_pause(kChaosTakePublish);
      // Fresh block: nobody else can see it until it is marked active.
      got = want >= c ? cap : ((1ull << want) - 1);
      uint32_t w = 0;
      if (is_first_active()) w = publish_block(h, (uint32_t)bid, type, got);
      chaos_pause(kChaosPublishSets);
      // allocated[type] and, unless full, active[type]: both ORs are issued
      // before either result is used (each keeps set's retry and cascade).
      const Bitmap alloc = allocated_bm(h, type);
      const uint32_t bw = (uint32_t)bid >> 6;
      const uint64_t bm = 1ull << ((uint32_t)bid & 63u);
      const uint64_t pa = bm_set_bits0_issue(alloc, bw, bm);
      const uint64_t pc = got != cap ? bm_set_bits0_issue(active, bw, bm) : 0ull;
      bm_set_bits0_settle(alloc, bw, bm, pa);
      if (got != cap) {
        bm_set_bits0_settle(active, bw, bm, pc);
        cur = bid;
        cur_avail = ~got & cap;
        cur_tw = bcast32(w);
      }
      // Counted as taken only now that its sets have returned: until then the
      // free-block count keeps other requests looking instead of failing.
      lead_add(shard(h) + kCntBlocksTaken, 1);
    } else {
      if (h.online_reclaim) {
        uint32_t pinned = 0;
        if (is_first_active()) pinned = pin_block(h, (uint32_t)bid, cur_tw) ? 1u : 0u;
        if (!bcast32(pinned)) continue;  // freed since: look up another block
      }
      const uint64_t take = take_from(avail, want < (uint32_t)__popcll(avail) ? want : (uint32_t)__popcll(avail),
                                      rot & (c - 1));
      const uint64_t prev = lead_or(h.obj_bitmap + bid, take);
      if (h.online_reclaim && is_first_active()) unpin_block(h, (uint32_t)bid);
      got = take & ~prev;
      const uint64_t after = (prev | take) & cap;
      if (after == cap && (prev & cap) != cap) bm_clear(active, (uint32_t)bid);
      if (after != cap) {
        cur = bid;  // still has room: the next pass can use it without a lookup
        cur_avail = ~after & cap;
      }
      if (got != take) ++retries;
      if (got == 0) {
        if (cur == kFail) start = hash32(start + it + 1);
        continue;
      }
    }
    const uint32_t cnt = (uint32_t)__popcll(got);
    const uint32_t lo = prefix > served ? prefix : served;
    const uint32_t hi = prefix + k < served + cnt ? prefix + k : served + cnt;
    for (uint32_t r = lo; r < hi; ++r) f(r - prefix, make_obj((uint32_t)bid, nth_set_bit(got, r - served)));
    served += cnt;
  }
  if (is_first_active()) {
    hints[kMaxTypes] = free_hint;
    hints[type] = act_hint;
  }
  if (oom) lead_flag(h.ctrl + kCtlOom);
  if (oom || gave_up)
    for (uint32_t r = prefix > served ? prefix : served; r < prefix + k; ++r) f(r - prefix, kNull);
  uint64_t* sh = shard(h);
  if (served) lead_add(sh + kCntAllocs + type, served);
  if (retries) lead_add(sh + kCntReserveRetries, retries);
  if (slow) lead_add(sh + kCntSlowPaths, slow);
  if (fails) lead_add(sh + kCntFindFails, fails);
}

// Device `new`: every calling lane gets one object of `type`.  Lanes may pass
// different types; each distinct type is served as one coalesced request.
template <class H>
__device__ inline uint32_t dsoar_new(const H& h, uint32_t type) {
  uint32_t result = kNull;
  for (;;) {
    const uint32_t t0 = bcast32(type);
    if (type == t0) {
      new_many(h, t0, 1u, [&](uint32_t, uint32_t o) { result = o; });
      break;
    }
  }
  return result;
}

// Online reclamation: the wavefront whose delete left block `bid` of `type`
// empty frees it at once (the block-state figure's return to free, inside a
// kernel).  Used when the heap's online_reclaim is set.
//  1 Invalidate: compare-and-swap the object bitmap from 0 to all ones.  If
//    that fails an allocation got in first and the block stays.  All ones
//    reads as full, so no reservation can gain a slot from here on.
//  2 Bump the version in the type word and mark it free, and leave
//    active[type] (clear with retry: it pairs with the set that made the
//    bit true), so that no further lookup selects the block; then wait until
//    no reservation holds it.  A reservation pins the block and then
//    re-reads the type word (both sequentially consistent), so either it
//    sees the change and withdraws, or this wait sees its pin.  (Waiting
//    with the block still active let the lookups of every other wavefront
//    keep pinning it, and the wait could starve.)
//  3 Leave allocated[type] (clear with retry).
//  4 Reset the object bitmap and count the block as returned, then set the
//    free bit once both are performed: an allocator that takes the block from
//    the free bitmap sees the reset bitmap and the new type word, and a
//    request that finds no free block still finds it in the count.
// Returns whether the block was freed (wave-uniform).
template <class H>
__device__ inline bool try_release(const H& h, uint32_t type, uint32_t bid) {
  uint32_t ok = 0;
  if (is_first_active()) {
    uint64_t expected = 0;
    ok = __hip_atomic_compare_exchange_strong(h.obj_bitmap + bid, &expected, ~0ull, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
             ? 1u
             : 0u;
    if (ok) {
      const uint32_t w = __hip_atomic_load(h.block_type + bid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(h.block_type + bid, tw_freed(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // The freed type word is performed before the pins are read (pin_block).
  wait_performed();
  if (!bcast32(ok)) return false;
  chaos_pause(kChaosRelease);
  bm_clear(active_bm(h, type), bid);
  for (uint32_t spins = 0;; ++spins) {
    uint32_t p = 0;
    if (is_first_active()) p = __hip_atomic_load(h.pins + bid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bcast32(p) == 0) break;
    if (spins >= kSpinLimit) {
      lead_flag(h.ctrl + kCtlRetryLimit);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  bm_clear(allocated_bm(h, type), bid);
  if (is_first_active()) __hip_atomic_store(h.obj_bitmap + bid, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  lead_add(shard(h) + kCntBlocksReturned, 1);  // counted before it can be found
  wait_performed();
  chaos_pause(kChaosRelease);
  bm_set(free_bm(h), bid);
  lead_add(shard(h) + kCntReleases, 1);
  return true;
}

// Delete a set of slots of one block (a wavefront's lanes, coalesced): one
// atomic AND on the object bitmap.  A block that was full becomes active
// again.  Blocks that become empty stay allocated until quiescent reclaim.
// Returns the number of objects removed (the caller counts them).
template <class H>
__device__ inline uint32_t delete_mask(const H& h, uint32_t type, uint32_t bid, uint64_t mask) {
  const uint64_t prev = lead_and(h.obj_bitmap + bid, ~mask);
  if ((prev & mask) != mask) lead_flag(h.ctrl + kCtlDoubleFree);
  const uint64_t removed = prev & mask;
  const uint64_t cap = capmask_of(h, type);
  chaos_pause(kChaosDeleteActive);
  if (removed && (prev & cap) == cap) bm_set(active_bm(h, type), bid);
  if (h.online_reclaim && removed && ((prev & ~mask) & cap) == 0) try_release(h, type, bid);
  return (uint32_t)__popcll(removed);
}

// Device `delete` of arbitrary objects: lanes are grouped by block; each group
// is one coalesced delete_mask.  NULL handles are ignored.
template <class H>
__device__ inline void dsoar_delete(const H& h, uint32_t obj) {
  const bool valid = obj == kNull || (obj >> 6) < h.num_blocks;
  if (!__builtin_expect(__ballot(!valid) == 0, 1)) lead_flag(h.ctrl + kCtlDoubleFree);
  const bool mine = obj != kNull && valid;
  uint64_t pending = __ballot(mine);
  while (pending) {
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1;
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane(obj, leader) >> 6;
    const bool in = mine && (obj >> 6) == b0 && ((pending >> lane_id()) & 1);
    const uint64_t grp = __ballot(in);
    const uint64_t m = slots_of(grp, obj_slot(obj));
    const uint32_t type =
        tw_type(bcast32(__hip_atomic_load(h.block_type + b0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    if (type < h.num_types) {
      const uint32_t freed = delete_mask(h, type, b0, m);
      if (freed) lead_add(shard(h) + kCntFrees + type, freed);
    } else {
      lead_flag(h.ctrl + kCtlDoubleFree);
    }
    pending &= ~grp;
  }
}

}  // namespace dsoar
