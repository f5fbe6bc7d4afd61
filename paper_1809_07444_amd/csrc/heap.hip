// Heap creation and layout, quiescent reclamation, parallel enumeration,
// statistics and invariant checks, the stand-alone bitmap entry points, and
// the C ABI of the heap.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace dsoar {

namespace {

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// 32-bit units of all levels of a bitmap of nbits bits with containers of
// 2^lg bits, padded to 256 bytes.
uint32_t bitmap_units(uint32_t nbits, uint32_t lg) {
  return (uint32_t)align_up(level_offset(nbits, lg, num_levels(nbits, lg)), 64);
}

uint32_t width_lg(uint32_t width) { return width == 32 ? 5u : 6u; }

bool desc_valid(const dsoar_heap_desc* d) {
  if (!d || (d->bitmap_width != 0 && d->bitmap_width != 32 && d->bitmap_width != 64)) return false;
  // Handles are block << 6 | slot in 32 bits and all ones is NULL: in a heap
  // of 2^26 blocks slot 63 of the last block would have the NULL handle.
  if (d->num_blocks < 1 || d->num_blocks >= (1u << 26)) return false;
  if (d->block_capacity != 0 && d->block_capacity != 32 && d->block_capacity != 64) return false;
  if (d->num_types < 1 || d->num_types > DSOAR_MAX_TYPES) return false;
  for (uint32_t t = 0; t < d->num_types; ++t) {
    const dsoar_type_layout& L = d->types[t];
    if (L.num_fields < 1 || L.num_fields > DSOAR_MAX_FIELDS) return false;
    for (uint32_t f = 0; f < L.num_fields; ++f)
      if (L.field_bytes[f] != 4 && L.field_bytes[f] != 8) return false;
    // A subclass names an earlier type and begins with its fields.
    if (L.parent != 0) {
      if (L.parent > t) return false;
      const dsoar_type_layout& P = d->types[L.parent - 1];
      if (L.num_fields < P.num_fields) return false;
      for (uint32_t f = 0; f < P.num_fields; ++f)
        if (L.field_bytes[f] != P.field_bytes[f]) return false;
    }
  }
  return true;
}

// Slots per block of each type.  A fixed block capacity (32 or 64) applies to
// every type.  Capacity 0 asks for the byte-size rule of Sec. 2: the smallest
// type has 64 slots and fixes the block size, 64 times its object size; a
// larger type gets the largest power of two of slots that fits that size.
void type_capacities(const dsoar_heap_desc* d, uint32_t* cap) {
  uint64_t smin = ~0ull, size[DSOAR_MAX_TYPES] = {0};
  for (uint32_t t = 0; t < d->num_types; ++t) {
    for (uint32_t f = 0; f < d->types[t].num_fields; ++f) size[t] += d->types[t].field_bytes[f];
    smin = std::min(smin, size[t]);
  }
  for (uint32_t t = 0; t < d->num_types; ++t) {
    if (d->block_capacity) {
      cap[t] = d->block_capacity;
      continue;
    }
    uint32_t c = 64;
    while (c > 1 && (uint64_t)c * size[t] > 64 * smin) c >>= 1;
    cap[t] = c;
  }
}

// Computes the layout of a heap in one caller buffer.  Block b's data segment
// holds, for its type, one SOA array per field (Sec. 2).  With a fixed
// capacity each array is padded to 128 bytes (Sec. 2 "Coalesced Access") and
// every block has the size of the widest type's segment.  With per-type
// capacities the arrays of a type are packed largest first (their sizes are
// powers of two, so each stays aligned to its own size, or to 128 bytes) and
// the block size is that of the smallest type's 64 objects.
struct Plan {
  dsoar_heap_layout L;
  uint64_t ctrl_off, stats_off, pins_off;
  uint64_t R_off[kMaxTypes], S_off[kMaxTypes], scan_off[kMaxTypes];
  uint32_t num_tiles;
  uint32_t enum_wpw;
};

Plan make_plan(const dsoar_heap_desc* d) {
  Plan p;
  memset(&p, 0, sizeof(p));
  const uint64_t M = d->num_blocks;
  type_capacities(d, p.L.type_capacity);
  uint64_t stride = 0;
  for (uint32_t t = 0; t < d->num_types; ++t) {
    const uint64_t c = p.L.type_capacity[t];
    const uint32_t nf = d->types[t].num_fields;
    uint64_t off = 0;
    if (d->block_capacity) {
      for (uint32_t f = 0; f < nf; ++f) {
        p.L.field_offset[t][f] = (uint32_t)off;
        off += align_up(c * d->types[t].field_bytes[f], 128);
      }
    } else {
      for (uint32_t w = 8; w >= 4; w -= 4)  // 8-byte fields first, then 4-byte ones
        for (uint32_t f = 0; f < nf; ++f)
          if (d->types[t].field_bytes[f] == w) {
            p.L.field_offset[t][f] = (uint32_t)off;
            off += c * w;
          }
    }
    stride = std::max(stride, off);
  }
  p.L.block_stride = align_up(stride, kAlign);
  uint64_t off = 0;
  p.L.data_offset = off;
  off = align_up(off + M * p.L.block_stride, kAlign);
  p.L.obj_bitmap_offset = off;
  off = align_up(off + M * 8, kAlign);
  p.L.block_type_offset = off;
  off = align_up(off + M * 4, kAlign);
  p.pins_off = off;
  off = align_up(off + M * 4, kAlign);
  p.L.bitmaps_offset = off;
  const uint32_t lg = width_lg(d->bitmap_width);
  p.L.bitmap_width = 1u << lg;
  p.L.bitmap_stride = (uint64_t)bitmap_units((uint32_t)M, lg) * 4;
  p.L.num_levels = num_levels((uint32_t)M, lg);
  for (uint32_t l = 0; l < p.L.num_levels && l < 8; ++l) {
    // In containers of the bitmap's width (levels start at even units).
    p.L.level_word_offset[l] = level_offset((uint32_t)M, lg, l) >> (lg - 5);
    p.L.level_words[l] = level_bits((uint32_t)M, lg, l + 1);
  }
  off = align_up(off + (1 + 2 * (uint64_t)d->num_types) * p.L.bitmap_stride, kAlign);
  p.ctrl_off = off;
  off = align_up(off + (kCtlWords + kShards * kShardStride) * 8, kAlign);
  p.stats_off = off;
  off = align_up(off + sizeof(StatsOut), kAlign);
  const uint64_t W0 = (M + 63) / 64;
  p.enum_wpw = W0 > kEnumWideFrom ? kEnumWideWords : 1;
  const uint64_t tile_words = (uint64_t)enum_waves(p.enum_wpw) * p.enum_wpw;
  p.num_tiles = (uint32_t)((W0 + tile_words - 1) / tile_words);
  for (uint32_t t = 0; t < d->num_types; ++t) {
    p.R_off[t] = off;
    off = align_up(off + M * 4, kAlign);
    p.S_off[t] = off;
    off = align_up(off + M * 8, kAlign);
    p.scan_off[t] = off;
    off = align_up(off + sizeof(ScanState) + (uint64_t)p.num_tiles * 8, kAlign);
  }
  p.L.total_bytes = off;
  return p;
}

// ------------------------------------------------------------------ kernels

// Bitmap initialisation, one 32-bit unit at a time: unit j of level l holds
// the level's bits [32j, 32j + 32) at either container width; when all_set,
// exactly the bits below the level's size are set (so every level is the OR
// of the level below).
__device__ inline uint32_t init_unit(uint32_t nbits, uint32_t lg, uint32_t u, bool all_set) {
  if (!all_set) return 0;
  const uint32_t L = num_levels(nbits, lg);
  uint32_t off = 0;
  for (uint32_t l = 0; l < L; ++l) {
    const uint32_t n = level_bits(nbits, lg, l), units = level_units(n);
    if (u < off + units) {
      const uint32_t lo = (u - off) * 32;
      if (lo >= n) return 0;
      return n - lo >= 32 ? 0xFFFFFFFFu : ((1u << (n - lo)) - 1u);
    }
    off += units;
  }
  return 0;
}

__global__ void init_bitmap_kernel(uint32_t* units, uint32_t nbits, uint32_t lg, uint32_t total_units, int all_set) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < total_units; u += gridDim.x * blockDim.x)
    __hip_atomic_store(units + u, init_unit(nbits, lg, u, all_set != 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void init_heap_kernel(DevHeap h, uint64_t ctrl_words) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nth = gridDim.x * blockDim.x;
  for (uint32_t b = tid; b < h.num_blocks; b += nth) {
    meta_store(h.obj_bitmap + b, 0ull);
    meta_store(h.block_type + b, kTypeNone);
    meta_store(h.pins + b, 0u);
  }
  for (uint64_t w = tid; w < ctrl_words; w += nth) meta_store(h.ctrl + w, 0ull);
  // Bitmap 0 (free) all set, the others clear.
  const uint64_t total = (uint64_t)(1 + 2 * h.num_types) * h.bm_units;
  for (uint64_t w = tid; w < total; w += nth) {
    const uint32_t k = (uint32_t)(w / h.bm_units);
    const uint32_t u = (uint32_t)(w % h.bm_units);
    meta_store(h.bitmaps + w, init_unit(h.num_blocks, h.bm_lg, u, k == 0));
  }
}

__global__ void init_scan_kernel(ScanState* st, uint64_t* flags, uint32_t num_tiles) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    st->tile_counter = 0;
    st->epoch = 1;
    st->count = 0;
    st->pad = 0;
  }
  for (uint32_t i = tid; i < num_tiles; i += gridDim.x * blockDim.x) flags[i] = 0;
}

// Quiescent reclamation of the blocks in `rc` (a wave's lanes, word `word`),
// all of type t and empty: they leave allocated[t] and active[t] and become
// free again (the block-state figure's transition back to free).  The three
// level-0 updates are issued together; each does the nested update its
// single-bit counterpart would (Alg. 2).
template <class H>
__device__ inline void reclaim_word(const H& h, uint32_t t, uint32_t word, uint64_t rc) {
  if ((rc >> lane_id()) & 1ull) {
    uint32_t* tw = h.block_type + word * 64 + lane_id();
    meta_store(tw, tw_freed(meta_load(tw)));
  }
  const Bitmap al = allocated_bm(h, t), ac = active_bm(h, t), fr = free_bm(h);
  lead_add(shard(h) + kCntBlocksReturned, (uint64_t)__popcll(rc));
  uint64_t pa = 0, pc = 0, pf = 0;
  if (is_first_active()) {
    pa = __hip_atomic_fetch_and(al.group(word), ~rc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pc = __hip_atomic_fetch_and(ac.group(word), ~rc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pf = __hip_atomic_fetch_or(fr.group(word), rc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  pa = bcast64(pa);
  pc = bcast64(pc);
  pf = bcast64(pf);
  group_clear_nested(al, word, pa, rc);
  group_clear_nested(ac, word, pc, rc);
  group_set_nested(fr, word, pf, rc & ~pf);
}

// Quiescent reclamation of the empty blocks rc[j] of WPW consecutive level-0
// groups word0 + j (word0 a multiple of WPW), as reclaim_word does for each,
// with the atomics batched: every group's three level-0 updates are issued
// before any result is used, and the nested updates they call for land in
// one level-1 container per bitmap (WPW groups of 64 blocks have consecutive
// bits one level up), one atomic each.
template <uint32_t WPW, class H>
__device__ inline void reclaim_words(const H& h, uint32_t t, uint32_t word0, const uint64_t (&rc)[WPW]) {
  uint64_t total = 0;
#pragma unroll
  for (uint32_t j = 0; j < WPW; ++j) {
    if ((rc[j] >> lane_id()) & 1ull) {
      uint32_t* tw = h.block_type + (word0 + j) * 64 + lane_id();
      meta_store(tw, tw_freed(meta_load(tw)));
    }
    total += (uint64_t)__popcll(rc[j]);
  }
  if (total == 0) return;
  const Bitmap al = allocated_bm(h, t), ac = active_bm(h, t), fr = free_bm(h);
  lead_add(shard(h) + kCntBlocksReturned, total);
  uint64_t pa[WPW], pc[WPW], pf[WPW];
  const bool leader = is_first_active();
#pragma unroll
  for (uint32_t j = 0; j < WPW; ++j) {
    pa[j] = pc[j] = pf[j] = 0;
    if (rc[j] && leader) {
      pa[j] = __hip_atomic_fetch_and(al.group(word0 + j), ~rc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      pc[j] = __hip_atomic_fetch_and(ac.group(word0 + j), ~rc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      pf[j] = __hip_atomic_fetch_or(fr.group(word0 + j), rc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (al.nlevels == 1) return;
  const uint32_t lg = al.lg, parts = 1u << (6 - lg);  // containers per group
  const uint32_t first = word0 * parts;                // level-1 bit of the first container
  const uint32_t c1 = first >> lg;                     // their level-1 container
  uint64_t ma = 0, mc = 0, mf = 0;
#pragma unroll
  for (uint32_t j = 0; j < WPW; ++j) {
    if (!rc[j]) continue;
    const uint64_t a = bcast64(pa[j]), c = bcast64(pc[j]), f = bcast64(pf[j]);
    for (uint32_t p = 0; p < parts; ++p) {
      const uint64_t pm = parts == 1 ? ~0ull : (0xFFFFFFFFull << (32 * p));
      const uint64_t bit = 1ull << ((first + j * parts + p) & ((1u << lg) - 1u));
      if ((a & rc[j] & pm) && !(a & ~rc[j] & pm)) ma |= bit;
      if ((c & rc[j] & pm) && !(c & ~rc[j] & pm)) mc |= bit;
      if ((rc[j] & ~f & pm) && !(f & pm)) mf |= bit;
    }
  }
  if (ma) bm_clear_bits_at(al, 1, c1, ma);
  if (mc) bm_clear_bits_at(ac, 1, c1, mc);
  if (mf) bm_set_bits_at(fr, 1, c1, mf);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int off = 32; off >= 1; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
  return v;
}

constexpr uint64_t kFlagAgg = 1ull << 30, kFlagIncl = 2ull << 30;
__device__ __forceinline__ uint64_t pack_flag(uint32_t epoch, uint64_t status, uint32_t value) {
  return ((uint64_t)epoch << 32) | status | (uint64_t)value;
}

// Parallel enumeration (Sec. 2.3): scan allocated[type] level 0 (step 1, set
// bits -> block ids), drop the empty blocks (reclaiming them once the tile's
// entries are out) and compact the rest into R with their object-bitmap
// snapshots (step 2, prefix sum).  One pass: tile prefixes come from a
// decoupled look-back over per-tile flags, tiles taken in launch order from a
// ticket counter.  Each wavefront covers
// WPW level-0 words (64 blocks each); all their loads are issued before any
// is used.  The heap is quiescent, so plain loads see the previous kernels.
template <uint32_t WPW, uint32_t LG>
__global__ void __launch_bounds__(enum_waves(WPW) * 64) enumerate_kernel(DevHeapW<LG> h, uint32_t type, EnumOut out) {
  constexpr uint32_t kEnumWaves = enum_waves(WPW);
  __shared__ uint32_t s_tile, s_epoch, s_prefix;
  __shared__ uint32_t s_wave_total[kEnumWaves];
  if (threadIdx.x == 0) {
    s_epoch = __hip_atomic_load(&out.st->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_tile = __hip_atomic_fetch_add(&out.st->tile_counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const uint32_t tile = s_tile, epoch = s_epoch;
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const uint32_t W0 = (h.num_blocks + 63) >> 6;
  const uint32_t word0 = (tile * kEnumWaves + wave) * WPW;
  const uint64_t* alloc0 = allocated_bm(h, type).group(0);  // level 0 as 64-bit groups
  uint64_t w[WPW], live[WPW], snap[WPW];
  if constexpr (WPW == 1) {
    // Narrow tiles (heaps of at most kEnumWideFrom words, 1 MiB of object
    // bitmaps): every block's object bitmap is loaded together with the
    // allocated word, one round trip instead of two, and kept where the
    // allocated bit is set.
    const uint32_t b = word0 * 64 + lane;
    const uint64_t ob = b < h.num_blocks ? meta_load(h.obj_bitmap + b) : 0ull;
    w[0] = word0 < W0 ? load_u64(alloc0 + word0) : 0ull;
    snap[0] = ((w[0] >> lane) & 1ull) ? ob : 0ull;
  } else {
#pragma unroll
    for (uint32_t j = 0; j < WPW; ++j) w[j] = word0 + j < W0 ? load_u64(alloc0 + word0 + j) : 0ull;
#pragma unroll
    for (uint32_t j = 0; j < WPW; ++j) {
      const uint32_t b = (word0 + j) * 64 + lane;
      const bool bit = ((w[j] >> lane) & 1ull) && b < h.num_blocks;
      snap[j] = bit ? meta_load(h.obj_bitmap + b) : 0ull;
    }
  }
  uint32_t wave_total = 0;
  uint64_t empty[WPW];  // allocated blocks without objects: reclaimed at the end
#pragma unroll
  for (uint32_t j = 0; j < WPW; ++j) {
    const bool bit = (w[j] >> lane) & 1ull;
    live[j] = __ballot(bit && snap[j] != 0);
    empty[j] = __ballot(bit && snap[j] == 0);
    wave_total += (uint32_t)__popcll(live[j]);
  }
  if (lane == 0) s_wave_total[wave] = wave_total;
  __syncthreads();
  uint32_t wave_off = 0, tile_total = 0;
  for (uint32_t k = 0; k < kEnumWaves; ++k) {
    const uint32_t v = s_wave_total[k];
    wave_off += k < wave ? v : 0u;
    tile_total += v;
  }
  if (wave == 0) {
    uint32_t exclusive = 0;
    if (tile == 0) {
      if (lane == 0)
        __hip_atomic_store(out.flags + tile, pack_flag(epoch, kFlagIncl, tile_total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(out.flags + tile, pack_flag(epoch, kFlagAgg, tile_total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      int32_t pred = (int32_t)tile - 1;
      for (uint32_t spins = 0;; ++spins) {
        const int32_t t = pred - (int32_t)lane;
        uint64_t f = t >= 0 ? __hip_atomic_load(out.flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : pack_flag(epoch, kFlagIncl, 0);
        const bool ready = (uint32_t)(f >> 32) == epoch && (f & (3ull << 30)) != 0;
        const bool incl = ready && (f & (3ull << 30)) == kFlagIncl;
        const uint64_t inclm = __ballot(incl), notready = __ballot(!ready);
        const uint32_t first = inclm ? (uint32_t)__builtin_ctzll(inclm) : 64u;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
        if (notready & need) {
          if (spins >= kSpinLimit) {
            lead_flag(h.ctrl + kCtlRetryLimit);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        exclusive += wave_sum(lane <= first ? (uint32_t)(f & ((1ull << 30) - 1)) : 0u);
        if (first < 64) break;
        pred -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(out.flags + tile, pack_flag(epoch, kFlagIncl, exclusive + tile_total),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) s_prefix = exclusive;
  }
  __syncthreads();
  uint32_t base = s_prefix + wave_off;
#pragma unroll
  for (uint32_t j = 0; j < WPW; ++j) {
    if ((live[j] >> lane) & 1ull) {
      const uint32_t pos = base + lanes_below(live[j]);
      out.R[pos] = (word0 + j) * 64 + lane;
      out.S[pos] = snap[j];
    }
    base += (uint32_t)__popcll(live[j]);
  }
  // Reclamation does not change the list, so it comes after the tile's
  // prefix is published and its entries are written: later tiles' look-back
  // never waits for these atomics.
  reclaim_words<WPW>(h, type, word0, empty);
  if (tile == out.num_tiles - 1 && threadIdx.x == 0) {
    __hip_atomic_store(&out.st->count, s_prefix + tile_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (out.count_out) *out.count_out = s_prefix + tile_total;
    __hip_atomic_store(&out.st->tile_counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&out.st->epoch, epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Reclaims every empty typed block (all types), one wavefront per 64 blocks.
__global__ void reclaim_kernel(DevHeap h) {
  const uint32_t W0 = (h.num_blocks + 63) >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t lane = lane_id();
  for (uint32_t word = blockIdx.x * wpb + (threadIdx.x >> 6); word < W0; word += gridDim.x * wpb) {
    const uint32_t b = word * 64 + lane;
    const bool in = b < h.num_blocks;
    const uint32_t t = in ? tw_type(meta_load(h.block_type + b)) : kTypeNone;
    const bool empty = in && t != kTypeNone && meta_load(h.obj_bitmap + b) == 0;
    uint64_t pending = __ballot(empty);
    while (pending) {
      const uint32_t t0 = __builtin_amdgcn_readlane(t, (uint32_t)__builtin_ctzll(pending));
      const uint64_t rc = __ballot(empty && t == t0);
      if (t0 < h.num_types) reclaim_word(h, t0, word, rc);
      pending &= ~rc;
    }
  }
}

// Statistics and invariants at quiescence, one wavefront per 64 blocks, plus
// container consistency of every level of every bitmap.
__global__ void stats_kernel(DevHeap h, StatsOut* out, int check) {
  const uint32_t W0 = (h.num_blocks + 63) >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t lane = lane_id();
  const uint32_t gw = blockIdx.x * wpb + (threadIdx.x >> 6), nw = gridDim.x * wpb;
  for (uint32_t word = gw; word < W0; word += nw) {
    const uint32_t b = word * 64 + lane;
    const bool in = b < h.num_blocks;
    const uint32_t t = in ? tw_type(meta_load(h.block_type + b)) : kTypeNone;
    const uint64_t ob = in ? meta_load(h.obj_bitmap + b) : 0;
    const uint64_t cm = t < h.num_types ? h.cap_mask[t] : ~0ull;  // this block's type's slots
    const uint64_t obc = ob & cm;
    const bool fr = (load_u64(free_bm(h).group(word)) >> lane) & 1ull;
    uint32_t v[DSOAR_INV_COUNT] = {0};
    if (in) {
      v[DSOAR_INV_BITMAP_RANGE] += (ob & ~cm) != 0;
      v[DSOAR_INV_FREE] += fr != (t == kTypeNone && obc == 0);
      if (t != kTypeNone && t >= h.num_types) v[DSOAR_INV_FREE] += 1;
    }
    for (uint32_t u = 0; u < h.num_types; ++u) {
      const bool al = (load_u64(allocated_bm(h, u).group(word)) >> lane) & 1ull;
      const bool ac = (load_u64(active_bm(h, u).group(word)) >> lane) & 1ull;
      if (in) {
        v[DSOAR_INV_ALLOCATED] += al != (t == u && obc != 0);
        v[DSOAR_INV_ACTIVE] += ac != (al && obc != cm);
        v[DSOAR_INV_ACTIVE_IMPLIES_ALLOCATED] += ac && !al;
        v[DSOAR_INV_FREE] += (al || ac) && fr;
      } else {
        v[DSOAR_INV_ALLOCATED] += al;
        v[DSOAR_INV_ACTIVE] += ac;
      }
      const uint64_t al_w = __ballot(al), ac_w = __ballot(ac);
      const uint32_t live = wave_sum(in && t == u ? (uint32_t)__popcll(obc) : 0u);
      const uint32_t typed = (uint32_t)__popcll(__ballot(in && t == u));
      if (lane == 0) {
        atomicAdd((unsigned long long*)&out->live[u], (unsigned long long)live);
        atomicAdd(&out->allocated[u], (uint32_t)__popcll(al_w));
        atomicAdd(&out->active[u], (uint32_t)__popcll(ac_w));
        atomicAdd(&out->typed[u], typed);
      }
    }
    if (!in) v[DSOAR_INV_FREE] += fr;
    const uint32_t nfree = (uint32_t)__popcll(__ballot(fr && in));
    if (lane == 0) atomicAdd(&out->free_blocks, nfree);
    if (check)
      for (uint32_t k = 0; k < DSOAR_INV_COUNT; ++k) {
        const uint32_t s = wave_sum(v[k]);
        if (lane == 0 && s) atomicAdd(&out->viol[k], s);
      }
  }
  if (!check) return;
  // Container consistency (Sec. 3): bit i of level l+1 == (container i of
  // level l != 0), and no bit set at or beyond a level's size.
  const uint32_t nbm = 1 + 2 * h.num_types;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  const uint32_t lg = h.bm_lg, cw = 1u << lg;
  for (uint32_t k = 0; k < nbm; ++k) {
    const Bitmap bm = heap_bitmap(h, k);
    for (uint32_t l = 0; l < bm.nlevels; ++l) {
      const uint32_t n = level_bits(h.num_blocks, lg, l);
      const uint32_t containers = level_bits(h.num_blocks, lg, l + 1);
      const uint32_t* lv = bm.level(l);
      for (uint32_t i = tid; i < containers; i += nth) {
        uint64_t w = meta_load(lv + (i << (lg - 5)));
        if (lg == 6) w |= (uint64_t)meta_load(lv + 2 * i + 1) << 32;
        const uint32_t lo = i * cw;
        const uint64_t valid = n - lo >= cw ? (lg == 6 ? ~0ull : 0xFFFFFFFFull) : ((1ull << (n - lo)) - 1);
        uint32_t bad = (w & ~valid) != 0;
        if (l + 1 < bm.nlevels) {
          const uint32_t* up = bm.level(l + 1);
          const bool set = (meta_load(up + ((i >> lg) << (lg - 5)) + ((i & (cw - 1)) >> 5)) >> (i & 31)) & 1u;
          bad += set != (w != 0);
        }
        if (bad) atomicAdd(&out->viol[DSOAR_INV_CONTAINER], bad);
      }
    }
  }
}

__global__ void zero_kernel(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------- stand-alone bitmap ops
// One wavefront per op, all lanes of the wavefront running it together.
struct LevelOffsets {
  uint32_t off[kMaxLevels];
};

__global__ void bitmap_ops_kernel(uint32_t* units, uint32_t nbits, uint32_t lg, LevelOffsets lv, const uint32_t* ops,
                                  uint32_t n, const uint32_t* starts, int32_t* results, uint64_t* retry_flag) {
  const Bitmap b{units, nbits, num_levels(nbits, lg), lg, retry_flag, lv.off};
  // One wavefront per operation, with the grid's stride in wavefronts.
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t op = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; op < n; op += waves) {
    const uint32_t kind = ops[2 * op], pos = ops[2 * op + 1];
    const uint32_t start = starts ? starts[op] : 0u;
    int32_t r = 0;
    const bool pos_ok = pos < nbits;
    switch (kind) {
      case DSOAR_BM_TRY_SET: r = pos_ok ? (bm_try_set(b, pos) ? 1 : 0) : -2; break;
      case DSOAR_BM_TRY_CLEAR: r = pos_ok ? (bm_try_clear(b, pos) ? 1 : 0) : -2; break;
      case DSOAR_BM_SET: r = pos_ok ? (bm_set(b, pos) ? 0 : -3) : -2; break;
      case DSOAR_BM_CLEAR: r = pos_ok ? (bm_clear(b, pos) ? 0 : -3) : -2; break;
      case DSOAR_BM_TRY_FIND_SET: r = bm_try_find_set(b, start); break;
      case DSOAR_BM_FIND_CLEAR: r = bm_find_clear(b, start); break;
      default: r = -2;
    }
    if (lane_id() == 0) results[op] = r;
  }
}

// -------------------------------------------------------- generic kernels
// The element kernels below loop over their items with the grid's stride (a
// multiple of 64, so a wavefront's lanes stay one aligned group of items and
// only the last group can be partial): a dispatch counts its work-items in 32
// bits, so n up to 2^32 - 1 takes a capped grid, not one lane per item.
__device__ __forceinline__ uint64_t first_item() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t item_stride() { return (uint64_t)gridDim.x * blockDim.x; }

template <uint32_t LG>
__global__ void alloc_n_kernel(DevHeapW<LG> h, uint32_t type, uint32_t n, uint32_t* out) {
  for (uint64_t i = first_item(); i < n; i += item_stride()) out[i] = dsoar_new(h, type);
}

template <uint32_t LG>
__global__ void free_n_kernel(DevHeapW<LG> h, const uint32_t* objs, uint32_t n) {
  for (uint64_t i = first_item(); i < n; i += item_stride()) dsoar_delete(h, objs[i]);
}

// Allocation/deletion stress: lane i runs `rounds` rounds; in round r its
// wavefront creates objects of type (spread * wave + r) mod num_types, one per lane,
// each lane writes its handle into field 0 of its object and, unless the
// round's draw keeps it, checks the field still holds the handle and deletes
// the object at once.  Kept handles go to out[i * rounds + r] (DSOAR_NULL
// otherwise).  A field found overwritten (a slot handed out twice) counts in
// errors[0].  Every lane of a wavefront runs every round (the heap calls are
// wavefront operations).
template <uint32_t LG>
__global__ void churn_kernel(DevHeapW<LG> h, uint32_t n, uint32_t rounds, uint32_t keep, uint32_t spread, uint32_t seed,
                             uint32_t* out, uint32_t* errors) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(i >> 6);
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t t = (spread * wave + r) % h.num_types;
    uint32_t o = kNull;
    new_many(h, t, in ? 1u : 0u, [&](uint32_t, uint32_t obj) { o = obj; });
    uint32_t del = kNull;
    if (o != kNull) {
      uint32_t* f0 = field_ptr<uint32_t>(h, o, t, 0);
      *f0 = o;
      const bool kept = hash32(seed ^ (i * 0x9E3779B1u) ^ (r * 0x85EBCA77u)) % keep == 0;
      if (kept) {
        out[(uint64_t)i * rounds + r] = o;
      } else {
        if (*f0 != o) atomicAdd(errors, 1u);
        del = o;
        out[(uint64_t)i * rounds + r] = kNull;
      }
    } else if (in) {
      out[(uint64_t)i * rounds + r] = kNull;
    }
    dsoar_delete(h, del);
  }
}

__global__ void field_rw_kernel(DevHeap h, uint32_t type, uint32_t field, const uint32_t* objs, uint32_t n,
                                uint32_t* data, int write) {
  for (uint64_t i = first_item(); i < n; i += item_stride()) {
    const uint32_t o = objs[i];
    // NULL and handles outside the heap's blocks or the type's slots are skipped.
    if (o == kNull || obj_block(o) >= h.num_blocks || obj_slot(o) >= h.capacity[type]) continue;
    uint32_t* p = field_ptr<uint32_t>(h, o, type, field);
    if (write) *p = data[i];
    else data[i] = *p;
  }
}

// ---------------------------------------------------------- built-in methods
struct VisitCount {
  static constexpr uint32_t kKind = 10;
  struct Args { uint32_t* counts; };
  struct Pre {};
  static __device__ Pre load(const DevHeap&, uint32_t, uint32_t, const Args&) { return {}; }
  static __device__ bool apply(const DevHeap&, uint32_t, uint32_t self, const Args& a, const Pre&) {
    atomicAdd(a.counts + self, 1u);
    return false;
  }
};

struct DeleteIfMod {
  static constexpr uint32_t kKind = 11;
  static constexpr bool kDeletesOnlyThis = true;
  struct Args { uint32_t field; int32_t modulus; int32_t residue; };
  struct Pre { int32_t v; };
  template <class H>
  static __device__ Pre load(const H& h, uint32_t type, uint32_t self, const Args& a) {
    return {*field_ptr<int32_t>(h, self, type, a.field)};
  }
  static __device__ bool apply(const DevHeap&, uint32_t, uint32_t, const Args& a, const Pre& p) {
    return (p.v % a.modulus) == a.residue;
  }
};

struct FieldGather {
  static constexpr uint32_t kKind = 12;
  struct Args { uint32_t key_field, field, num_keys, wide; uint8_t* out; uint8_t* present; };
  template <class H>
  static __device__ bool run(const H& h, uint32_t type, uint32_t self, const Args& a) {
    const uint32_t key = *field_ptr<uint32_t>(h, self, type, a.key_field);
    if (key >= a.num_keys) return false;
    if (a.wide) reinterpret_cast<uint64_t*>(a.out)[key] = *field_ptr<uint64_t>(h, self, type, a.field);
    else reinterpret_cast<uint32_t*>(a.out)[key] = *field_ptr<uint32_t>(h, self, type, a.field);
    if (a.present) a.present[key] = 1;
    return false;
  }
};

}  // namespace

// ------------------------------------------------------ shared host helpers

int launch_enumerate_into(dsoar_heap* h, uint32_t type, const EnumOut& eo, hipStream_t s) {
  if (h->enum_wpw == kEnumWideWords)
    with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(h, kKindEnumerate, enumerate_kernel<kEnumWideWords, kLG>, dim3(h->num_tiles),
                 dim3(enum_waves(kEnumWideWords) * 64),
                 s, DevHeapW<kLG>(h->dev), type, eo);
  });
  else
    with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(h, kKindEnumerate, enumerate_kernel<1, kLG>, dim3(h->num_tiles), dim3(enum_waves(1) * 64), s,
                 DevHeapW<kLG>(h->dev),
                 type, eo);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

int launch_enumerate(dsoar_heap* h, uint32_t type, hipStream_t s) {
  return launch_enumerate_into(h, type, h->enum_out[type], s);
}

// Scratch of the allocation-free enumeration (dsoar_enumerate_noalloc): the
// scan state and one look-back word per tile, sized for the largest heap
// (2^26 - 1 blocks: 2^20 level-0 groups, at least 64 per tile).  Each device holds
// its own copy; host code uses the address hipGetSymbolAddress returns for
// the current device, never the symbol itself.
constexpr uint32_t kStaticTiles = 16384;
static_assert((1u << 20) / (enum_waves(kEnumWideWords) * kEnumWideWords) <= kStaticTiles &&
                  kEnumWideFrom / enum_waves(1) <= kStaticTiles,
              "the scratch covers the tiles of every heap size");
constexpr uint32_t kScratchWords = 2 + kStaticTiles;  // ScanState, then the tile flags
static_assert(sizeof(ScanState) == 16, "scan state is two words");
static __device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// This device's copy of the scratch array (looked up once per device).
static int scratch_ptr(dsoar_heap* h, uint64_t** out) {
  int dev = 0;
  DSOAR_HIP(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return DSOAR_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DSOAR_HIP(h, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = (uint64_t*)g_scratch_ptr[dev];
  return DSOAR_OK;
}

int read_count(dsoar_heap* h, uint32_t type, hipStream_t s, uint32_t* count) {
  DSOAR_HIP(h, hipMemcpyAsync(count, &h->enum_out[type].st->count, 4, hipMemcpyDeviceToHost, s));
  DSOAR_HIP(h, hipStreamSynchronize(s));
  return DSOAR_OK;
}

// Do-all methods implemented in the workload translation units.
int micro_doall(dsoar_heap* h, uint32_t type, uint32_t method, uint32_t flags, hipStream_t s);

}  // namespace dsoar

using namespace dsoar;

namespace {

// Workgroups for n items of `threads` lanes: enough to cover them, at most
// `cap`, and fewer than 2^32 work-items in all (a dispatch's 32-bit limit).
// Kernels launched with a capped grid loop over their items.
uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap = 65535u * 16u) {
  uint64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  g = std::min<uint64_t>(g, cap);
  return (uint32_t)std::min<uint64_t>(g, 0xFFFFFFFFull / threads);
}

int init_device_state(dsoar_heap* h, hipStream_t s) {
  const uint64_t ctrl_words = kCtlWords + kShards * kShardStride;
  const uint64_t work = std::max<uint64_t>(h->desc.num_blocks, (1 + 2 * h->desc.num_types) * (uint64_t)h->dev.bm_units);
  hipLaunchKernelGGL(init_heap_kernel, dim3(grid_for(work, 256, 8192)), dim3(256), 0, s, h->dev, ctrl_words);
  DSOAR_LAUNCHED(h);
  for (uint32_t t = 0; t < h->desc.num_types; ++t) {
    hipLaunchKernelGGL(init_scan_kernel, dim3(grid_for(h->num_tiles, 256, 1024)), dim3(256), 0, s,
                       h->enum_out[t].st, h->enum_out[t].flags, h->num_tiles);
    DSOAR_LAUNCHED(h);
  }
  return DSOAR_OK;
}

int sticky_status(const dsoar_stats& st) {
  if (st.oom) return DSOAR_ERR_OOM;
  if (st.retry_limit_hit) return DSOAR_ERR_RETRY_LIMIT;
  if (st.double_free) return DSOAR_ERR_DOUBLE_FREE;
  return DSOAR_OK;
}

int collect_stats(dsoar_heap* h, dsoar_stats* out, uint32_t* viol, int check, hipStream_t s) {
  const uint32_t n32 = sizeof(StatsOut) / 4;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)h->stats_dev, n32);
  DSOAR_LAUNCHED(h);
  const uint32_t W0 = (h->desc.num_blocks + 63) / 64;
  hipLaunchKernelGGL(stats_kernel, dim3(grid_for((uint64_t)W0 * 64, 256, 4096)), dim3(256), 0, s, h->dev,
                     h->stats_dev, check);
  DSOAR_LAUNCHED(h);
  StatsOut so;
  const uint64_t ctrl_words = kCtlWords + kShards * kShardStride;
  std::vector<uint64_t> ctrl_buf(ctrl_words);
  uint64_t* ctrl = ctrl_buf.data();
  DSOAR_HIP(h, hipMemcpyAsync(&so, h->stats_dev, sizeof(so), hipMemcpyDeviceToHost, s));
  DSOAR_HIP(h, hipMemcpyAsync(ctrl, h->dev.ctrl, ctrl_words * 8, hipMemcpyDeviceToHost, s));
  DSOAR_HIP(h, hipStreamSynchronize(s));
  dsoar_stats st;
  memset(&st, 0, sizeof(st));
  for (uint32_t sh = 0; sh < kShards; ++sh) {
    const uint64_t* c = ctrl + kCtlWords + sh * kShardStride;
    for (uint32_t t = 0; t < kMaxTypes; ++t) {
      st.allocs[t] += c[kCntAllocs + t];
      st.frees[t] += c[kCntFrees + t];
      st.visits[t] += c[kCntVisits + t];
    }
    st.reserve_retries += c[kCntReserveRetries];
    st.slow_paths += c[kCntSlowPaths];
    st.find_fails += c[kCntFindFails];
    st.method_atomics += c[kCntMethodAtomics];
    st.online_releases += c[kCntReleases];
    st.blocks_taken += c[kCntBlocksTaken];
    st.blocks_returned += c[kCntBlocksReturned];
  }
  for (uint32_t t = 0; t < kMaxTypes; ++t) {
    st.live_objects[t] = so.live[t];
    st.allocated_blocks[t] = so.allocated[t];
    st.active_blocks[t] = so.active[t];
    st.typed_blocks[t] = so.typed[t];
  }
  st.free_blocks = so.free_blocks;
  st.num_blocks = h->desc.num_blocks;
  st.oom = ctrl[kCtlOom] != 0;
  st.retry_limit_hit = ctrl[kCtlRetryLimit] != 0;
  st.double_free = ctrl[kCtlDoubleFree] != 0;
  if (out) *out = st;
  if (viol) {
    for (uint32_t k = 0; k < DSOAR_INV_COUNT; ++k) viol[k] = so.viol[k];
    for (uint32_t t = 0; t < h->desc.num_types; ++t)
      if (st.live_objects[t] != st.allocs[t] - st.frees[t]) viol[DSOAR_INV_LIVE_COUNT] += 1;
    if ((uint64_t)st.free_blocks + st.blocks_taken != (uint64_t)st.num_blocks + st.blocks_returned)
      viol[DSOAR_INV_FREE_COUNT] += 1;
  }
  return sticky_status(st);
}

}  // namespace

extern "C" {

size_t dsoar_heap_bytes(const dsoar_heap_desc* desc) {
  if (!desc_valid(desc)) return 0;
  return (size_t)make_plan(desc).L.total_bytes;
}

int dsoar_heap_create(const dsoar_heap_desc* desc, void* dev_mem, size_t dev_bytes, void* stream,
                      dsoar_heap** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!desc_valid(desc) || !dev_mem || ((uintptr_t)dev_mem & 255u)) return DSOAR_ERR_INVALID_ARG;
  const Plan p = make_plan(desc);
  if (dev_bytes < p.L.total_bytes) return DSOAR_ERR_TOO_SMALL;
  dsoar_heap* h = new (std::nothrow) dsoar_heap;
  if (!h) return DSOAR_ERR_INVALID_ARG;
  memset(h, 0, sizeof(*h));
  h->desc = *desc;
  h->layout = p.L;
  h->base = (uint8_t*)dev_mem;
  h->bytes = dev_bytes;
  h->num_tiles = p.num_tiles;
  h->enum_wpw = p.enum_wpw;
  DevHeap& d = h->dev;
  d.data = h->base + p.L.data_offset;
  d.obj_bitmap = (uint64_t*)(h->base + p.L.obj_bitmap_offset);
  d.block_type = (uint32_t*)(h->base + p.L.block_type_offset);
  d.pins = (uint32_t*)(h->base + p.pins_off);
  d.bitmaps = (uint32_t*)(h->base + p.L.bitmaps_offset);
  d.ctrl = (uint64_t*)(h->base + p.ctrl_off);
  d.block_stride = p.L.block_stride;
  for (uint32_t t = 0; t < kMaxTypes; ++t) {
    const uint32_t c = t < desc->num_types ? p.L.type_capacity[t] : 64u;
    d.capacity[t] = c;
    d.cap_mask[t] = c == 64 ? ~0ull : ((1ull << c) - 1);
  }
  d.num_blocks = desc->num_blocks;
  d.num_types = desc->num_types;
  d.nlevels = p.L.num_levels;
  d.bm_lg = width_lg(desc->bitmap_width);
  d.bm_units = (uint32_t)(p.L.bitmap_stride / 4);
  for (uint32_t l = 0; l < kMaxLevels; ++l) d.bm_off[l] = level_offset(d.num_blocks, d.bm_lg, l);
  d.search_start = kStartHashed;
  for (uint32_t t = 0; t < desc->num_types; ++t)
    for (uint32_t f = 0; f < desc->types[t].num_fields; ++f) {
      d.field_loc[t][f] = p.L.field_offset[t][f] | ((desc->types[t].field_bytes[f] == 8 ? 3u : 2u) << 24);
    }
  // Inheritance (Sec. 1.2): each type's own bit and those of every type
  // whose chain of parents reaches it (parents are declared earlier).
  for (uint32_t u = 0; u < desc->num_types; ++u)
    for (uint32_t a = u + 1; a != 0; a = desc->types[a - 1].parent) h->subtypes[a - 1] |= 1u << u;
  h->stats_dev = (StatsOut*)(h->base + p.stats_off);
  for (uint32_t t = 0; t < desc->num_types; ++t) {
    EnumOut& e = h->enum_out[t];
    e.R = (uint32_t*)(h->base + p.R_off[t]);
    e.S = (uint64_t*)(h->base + p.S_off[t]);
    e.st = (ScanState*)(h->base + p.scan_off[t]);
    e.flags = (uint64_t*)(h->base + p.scan_off[t] + sizeof(ScanState));
    e.num_tiles = p.num_tiles;
    e.count_out = nullptr;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete h;
    return DSOAR_ERR_HIP;
  }
  h->num_cus = (uint32_t)prop.multiProcessorCount;
  h->doall_wg_threads = 256;
  h->doall_wgs_per_cu = 8;
  d.bulk_min = 0xFFFFFFFFu;  // dense policy: active blocks first
  d.fresh_types = 0;
  d.bounded_types = 0;
  d.doall_unroll = 4;
  const int rc = init_device_state(h, (hipStream_t)stream);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return DSOAR_OK;
}

static void timing_free(dsoar_heap* h) {
  if (h->ev_pool) {
    for (uint32_t i = 0; i < 2 * kTimingCap; ++i) (void)hipEventDestroy(h->ev_pool[i]);
    free(h->ev_pool);
    free(h->rec_kind);
  }
  h->ev_pool = nullptr;
  h->rec_kind = nullptr;
  h->rec_used = 0;
  h->timing = 0;
}

int dsoar_heap_destroy(dsoar_heap* h) {
  if (!h) return DSOAR_ERR_INVALID_ARG;
  timing_free(h);
  delete h;
  return DSOAR_OK;
}

int dsoar_heap_set_timing(dsoar_heap* h, int enable) {
  if (!heap_ok(h)) return DSOAR_ERR_INVALID_ARG;
  if (!enable) {
    timing_free(h);
    return DSOAR_OK;
  }
  if (!h->ev_pool) {
    h->ev_pool = (hipEvent_t*)calloc(2 * kTimingCap, sizeof(hipEvent_t));
    h->rec_kind = (uint32_t*)calloc(kTimingCap, sizeof(uint32_t));
    if (!h->ev_pool || !h->rec_kind) {
      free(h->ev_pool);
      free(h->rec_kind);
      h->ev_pool = nullptr;
      h->rec_kind = nullptr;
      return DSOAR_ERR_INVALID_ARG;
    }
    for (uint32_t i = 0; i < 2 * kTimingCap; ++i) DSOAR_HIP(h, hipEventCreate(&h->ev_pool[i]));
  }
  h->rec_used = 0;
  h->timing = 1;
  return DSOAR_OK;
}

int dsoar_heap_timing(dsoar_heap* h, uint32_t* kinds, uint32_t* counts, double* total_ms, uint32_t max_kinds,
                      uint32_t* num_kinds) {
  if (!heap_ok(h) || !num_kinds || (max_kinds && (!kinds || !counts || !total_ms))) return DSOAR_ERR_INVALID_ARG;
  *num_kinds = 0;
  if (!h->timing) return DSOAR_OK;
  if (h->rec_used) DSOAR_HIP(h, hipEventSynchronize(h->ev_pool[2 * (h->rec_used - 1) + 1]));
  uint32_t n = 0;
  for (uint32_t r = 0; r < h->rec_used; ++r) {
    float ms = 0.f;
    DSOAR_HIP(h, hipEventElapsedTime(&ms, h->ev_pool[2 * r], h->ev_pool[2 * r + 1]));
    uint32_t k = 0;
    while (k < n && kinds[k] != h->rec_kind[r]) ++k;
    if (k == n) {
      if (n == max_kinds) continue;
      kinds[n] = h->rec_kind[r];
      counts[n] = 0;
      total_ms[n] = 0.0;
      ++n;
    }
    counts[k] += 1;
    total_ms[k] += ms;
  }
  *num_kinds = n;
  h->rec_used = 0;
  return DSOAR_OK;
}

int dsoar_heap_reset(dsoar_heap* h, void* stream) {
  if (!heap_ok(h)) return DSOAR_ERR_INVALID_ARG;
  return init_device_state(h, (hipStream_t)stream);
}

int dsoar_heap_get_layout(const dsoar_heap* h, dsoar_heap_layout* out) {
  if (!heap_ok(h) || !out) return DSOAR_ERR_INVALID_ARG;
  *out = h->layout;
  return DSOAR_OK;
}

int dsoar_heap_set_launch(dsoar_heap* h, uint32_t wg_threads, uint32_t wgs_per_cu) {
  if (!heap_ok(h) || wg_threads < 64 || wg_threads > 1024 || (wg_threads & 63) || wgs_per_cu < 1 ||
      wgs_per_cu > 64)
    return DSOAR_ERR_INVALID_ARG;
  h->doall_wg_threads = wg_threads;
  h->doall_wgs_per_cu = wgs_per_cu;
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_heap_set_policy(dsoar_heap* h, uint32_t bulk_min) {
  if (!heap_ok(h)) return DSOAR_ERR_INVALID_ARG;
  h->dev.bulk_min = bulk_min;  // below a type's capacity it acts as that capacity
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_heap_set_type_policy(dsoar_heap* h, uint32_t type, uint32_t policy) {
  if (!heap_ok(h) || type >= h->desc.num_types || policy > DSOAR_POLICY_BOUNDED) return DSOAR_ERR_INVALID_ARG;
  const uint32_t bit = 1u << type;
  h->dev.fresh_types = policy == DSOAR_POLICY_FRESH ? (h->dev.fresh_types | bit) : (h->dev.fresh_types & ~bit);
  h->dev.bounded_types =
      policy == DSOAR_POLICY_BOUNDED ? (h->dev.bounded_types | bit) : (h->dev.bounded_types & ~bit);
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_heap_set_search(dsoar_heap* h, uint32_t policy) {
  if (!heap_ok(h) || policy > DSOAR_SEARCH_XCD) return DSOAR_ERR_INVALID_ARG;
  static_assert(DSOAR_SEARCH_HASHED == kStartHashed && DSOAR_SEARCH_LOWEST == kStartLowest &&
                    DSOAR_SEARCH_XCD == kStartXcd,
                "search policy numbering");
  h->dev.search_start = policy;
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_heap_set_reclaim(dsoar_heap* h, int online) {
  if (!heap_ok(h)) return DSOAR_ERR_INVALID_ARG;
  h->dev.online_reclaim = online ? 1u : 0u;
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_heap_set_unroll(dsoar_heap* h, uint32_t blocks_per_pass) {
  if (!heap_ok(h) || (blocks_per_pass != 1 && blocks_per_pass != 2 && blocks_per_pass != 4 && blocks_per_pass != 8))
    return DSOAR_ERR_INVALID_ARG;
  h->dev.doall_unroll = blocks_per_pass;
  h->config_epoch++;
  return DSOAR_OK;
}

int dsoar_enumerate(dsoar_heap* h, uint32_t type, void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types) return DSOAR_ERR_INVALID_ARG;
  return launch_enumerate(h, type, (hipStream_t)stream);
}

int dsoar_enumerate_noalloc(dsoar_heap* h, uint32_t type, uint32_t* R_dev, uint64_t* S_dev, uint32_t* count_dev,
                            void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types || !R_dev || !S_dev || !count_dev) return DSOAR_ERR_INVALID_ARG;
  if (h->num_tiles > kStaticTiles) return DSOAR_ERR_INVALID_ARG;  // larger than the scratch covers
  uint64_t* sp = nullptr;
  const int rc = scratch_ptr(h, &sp);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  ScanState* st = reinterpret_cast<ScanState*>(sp);
  uint64_t* flags = sp + 2;
  // The scratch keeps the last call's contents: the ticket, epoch and this
  // heap's tile flags start from zero (a fill kernel, so that the call can
  // be captured in a graph).
  hipLaunchKernelGGL(init_scan_kernel, dim3(grid_for(h->num_tiles, 256, 1024)), dim3(256), 0, s, st, flags,
                     h->num_tiles);
  DSOAR_LAUNCHED(h);
  const EnumOut eo{R_dev, S_dev, st, flags, h->num_tiles, count_dev};
  return launch_enumerate_into(h, type, eo, s);
}

int dsoar_enum_count(dsoar_heap* h, uint32_t type, uint32_t* count, void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types || !count) return DSOAR_ERR_INVALID_ARG;
  return read_count(h, type, (hipStream_t)stream, count);
}

int dsoar_enum_arrays(dsoar_heap* h, uint32_t type, uint64_t* R_dev, uint64_t* S_dev) {
  if (!heap_ok(h) || type >= h->desc.num_types || !R_dev || !S_dev) return DSOAR_ERR_INVALID_ARG;
  *R_dev = (uint64_t)(uintptr_t)h->enum_out[type].R;
  *S_dev = (uint64_t)(uintptr_t)h->enum_out[type].S;
  return DSOAR_OK;
}

int dsoar_reclaim(dsoar_heap* h, void* stream) {
  if (!heap_ok(h)) return DSOAR_ERR_INVALID_ARG;
  const uint32_t W0 = (h->desc.num_blocks + 63) / 64;
  hipLaunchKernelGGL(reclaim_kernel, dim3(grid_for((uint64_t)W0 * 64, 256, 8192)), dim3(256), 0,
                     (hipStream_t)stream, h->dev);
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

int dsoar_parallel_do(dsoar_heap* h, uint32_t type, uint32_t method, const void* args, size_t args_bytes,
                      uint32_t flags, void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types) return DSOAR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  switch (method) {
    case DSOAR_METHOD_VISIT_COUNT: {
      if (!args || args_bytes != sizeof(dsoar_visit_args)) return DSOAR_ERR_INVALID_ARG;
      const dsoar_visit_args* a = (const dsoar_visit_args*)args;
      if (!a->counts_dev) return DSOAR_ERR_INVALID_ARG;
      return launch_doall_tree<VisitCount>(h, type, VisitCount::Args{a->counts_dev}, flags, s);
    }
    case DSOAR_METHOD_DELETE_IF_MOD: {
      if (!args || args_bytes != sizeof(dsoar_mod_args)) return DSOAR_ERR_INVALID_ARG;
      const dsoar_mod_args* a = (const dsoar_mod_args*)args;
      if (a->field >= h->desc.types[type].num_fields || h->desc.types[type].field_bytes[a->field] != 4 ||
          a->modulus <= 0)
        return DSOAR_ERR_INVALID_ARG;
      return launch_doall_tree<DeleteIfMod>(h, type, DeleteIfMod::Args{a->field, a->modulus, a->residue}, flags,
                                            s);
    }
    case DSOAR_METHOD_FIELD_GATHER: {
      if (!args || args_bytes != sizeof(dsoar_gather_args)) return DSOAR_ERR_INVALID_ARG;
      const dsoar_gather_args* a = (const dsoar_gather_args*)args;
      const dsoar_type_layout& L = h->desc.types[type];
      if (a->key_field >= L.num_fields || a->field >= L.num_fields || L.field_bytes[a->key_field] != 4 ||
          !a->out_dev)
        return DSOAR_ERR_INVALID_ARG;
      FieldGather::Args g{a->key_field, a->field, a->num_keys, L.field_bytes[a->field] == 8 ? 1u : 0u,
                          (uint8_t*)a->out_dev, a->present_dev};
      return launch_doall_tree<FieldGather>(h, type, g, flags, s);
    }
    case DSOAR_METHOD_MICRO_UPDATE:
    case DSOAR_METHOD_MICRO_CULL:
      return micro_doall(h, type, method, flags, s);
    default:
      return DSOAR_ERR_UNSUPPORTED;
  }
}

int dsoar_heap_stats(dsoar_heap* h, dsoar_stats* out, void* stream) {
  if (!heap_ok(h) || !out) return DSOAR_ERR_INVALID_ARG;
  return collect_stats(h, out, nullptr, 0, (hipStream_t)stream);
}

int dsoar_heap_check(dsoar_heap* h, uint32_t* violations, void* stream) {
  if (!heap_ok(h) || !violations) return DSOAR_ERR_INVALID_ARG;
  int rc = dsoar_reclaim(h, stream);
  if (rc) return rc;
  return collect_stats(h, nullptr, violations, 1, (hipStream_t)stream);
}

int dsoar_alloc_n(dsoar_heap* h, uint32_t type, uint32_t n, dsoar_obj* out_dev, void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types || (!out_dev && n)) return DSOAR_ERR_INVALID_ARG;
  if (n == 0) return DSOAR_OK;
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    hipLaunchKernelGGL(alloc_n_kernel<kLG>, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, (hipStream_t)stream, DevHeapW<kLG>(h->dev),
                     type, n, out_dev);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

int dsoar_stress_churn(dsoar_heap* h, uint32_t n, uint32_t rounds, uint32_t keep, uint32_t spread, uint32_t seed,
                       dsoar_obj* out_dev, uint32_t* errors_dev, void* stream) {
  if (!heap_ok(h) || n == 0 || n > (1u << 31) || rounds == 0 || keep == 0 || !out_dev || !errors_dev ||
      (uint64_t)n * rounds > (1ull << 32))
    return DSOAR_ERR_INVALID_ARG;
  for (uint32_t t = 0; t < h->desc.num_types; ++t)
    if (h->desc.types[t].field_bytes[0] != 4) return DSOAR_ERR_INVALID_ARG;
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    hipLaunchKernelGGL(churn_kernel<kLG>, dim3((uint32_t)(((uint64_t)n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, DevHeapW<kLG>(h->dev), n, rounds, keep,
                     spread, seed, out_dev, errors_dev);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

int dsoar_free_n(dsoar_heap* h, const dsoar_obj* objs_dev, uint32_t n, void* stream) {
  if (!heap_ok(h) || (!objs_dev && n)) return DSOAR_ERR_INVALID_ARG;
  if (n == 0) return DSOAR_OK;
  with_width(h, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    hipLaunchKernelGGL(free_n_kernel<kLG>, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, (hipStream_t)stream, DevHeapW<kLG>(h->dev),
                     objs_dev, n);
  });
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

static int field_rw(dsoar_heap* h, uint32_t type, uint32_t field, const dsoar_obj* objs, uint32_t n, uint32_t* data,
                    int write, void* stream) {
  if (!heap_ok(h) || type >= h->desc.num_types || field >= h->desc.types[type].num_fields ||
      h->desc.types[type].field_bytes[field] != 4 || (n && (!objs || !data)))
    return DSOAR_ERR_INVALID_ARG;
  if (n == 0) return DSOAR_OK;
  hipLaunchKernelGGL(field_rw_kernel, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, (hipStream_t)stream, h->dev,
                     type, field, objs, n, data, write);
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

int dsoar_field_read(dsoar_heap* h, uint32_t type, uint32_t field, const dsoar_obj* objs, uint32_t n,
                     uint32_t* out_dev, void* stream) {
  return field_rw(h, type, field, objs, n, out_dev, 0, stream);
}

int dsoar_field_write(dsoar_heap* h, uint32_t type, uint32_t field, const dsoar_obj* objs, uint32_t n,
                      const uint32_t* in_dev, void* stream) {
  return field_rw(h, type, field, objs, n, (uint32_t*)in_dev, 1, stream);
}

const char* dsoar_error_string(int status) {
  switch (status) {
    case DSOAR_OK: return "ok";
    case DSOAR_ERR_INVALID_ARG: return "invalid argument";
    case DSOAR_ERR_OOM: return "out of memory: a device new found no free block";
    case DSOAR_ERR_RETRY_LIMIT: return "a bounded device retry loop gave up";
    case DSOAR_ERR_HIP: return "HIP runtime error";
    case DSOAR_ERR_DOUBLE_FREE: return "delete of an unallocated slot";
    case DSOAR_ERR_TOO_SMALL: return "device buffer too small";
    case DSOAR_ERR_UNSUPPORTED: return "unsupported method";
    default: return "unknown status";
  }
}

int dsoar_abi_version(void) { return DSOAR_ABI_VERSION; }

int dsoar_last_hip_error(const dsoar_heap* h) { return h ? (int)h->last_hip : -1; }

size_t dsoar_bitmap_bytes(uint32_t nbits, uint32_t width) {
  if (nbits == 0 || nbits > (1u << 30) || (width != 32 && width != 64)) return 0;
  return (size_t)bitmap_units(nbits, width_lg(width)) * 4 + 256;  // + a retry-flag line
}

int dsoar_bitmap_init(void* bm_dev, uint32_t nbits, uint32_t width, int all_set, void* stream) {
  if (!bm_dev || nbits == 0 || nbits > (1u << 30) || (width != 32 && width != 64) || ((uintptr_t)bm_dev & 7u))
    return DSOAR_ERR_INVALID_ARG;
  const uint32_t lg = width_lg(width);
  const uint32_t units = bitmap_units(nbits, lg) + 64;
  // The padding and the flag line after the levels are cleared by the same
  // kernel (init_unit is 0 past the last level).
  hipLaunchKernelGGL(init_bitmap_kernel, dim3(grid_for(units, 256, 8192)), dim3(256), 0, (hipStream_t)stream,
                     (uint32_t*)bm_dev, nbits, lg, units, all_set);
  if (hipGetLastError() != hipSuccess) return DSOAR_ERR_HIP;
  return DSOAR_OK;
}

int dsoar_bitmap_run(void* bm_dev, uint32_t nbits, uint32_t width, const uint32_t* ops_dev, uint32_t n,
                     const uint32_t* start_dev, int32_t* results_dev, void* stream) {
  if (!bm_dev || nbits == 0 || nbits > (1u << 30) || (width != 32 && width != 64) ||
      (n && (!ops_dev || !results_dev)))
    return DSOAR_ERR_INVALID_ARG;
  if (n == 0) return DSOAR_OK;
  const uint32_t lg = width_lg(width);
  uint32_t* units = (uint32_t*)bm_dev;
  uint64_t* flag = reinterpret_cast<uint64_t*>(units + bitmap_units(nbits, lg));
  LevelOffsets lv;
  for (uint32_t l = 0; l < kMaxLevels; ++l) lv.off[l] = level_offset(nbits, lg, l);
  hipLaunchKernelGGL(bitmap_ops_kernel, dim3(grid_for((uint64_t)n * 64, 256, 1u << 20)), dim3(256), 0,
                     (hipStream_t)stream, units, nbits, lg, lv, ops_dev, n, start_dev, results_dev, flag);
  if (hipGetLastError() != hipSuccess) return DSOAR_ERR_HIP;
  return DSOAR_OK;
}

}  // extern "C"
