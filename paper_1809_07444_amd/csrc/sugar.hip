// Sugarscape-style agents as objects on a square torus (the paper's
// sugarscape application, Sec. 4; its rules are not in the paper, so this is
// a synchronous, deterministic variant).  Agent {sugar, metabolism, vision,
// age, pos, target}; the sugar, capacity, occupancy and request grids are
// plain device arrays.  One step t:
//   regrow (grid kernel): sugar = min(sugar + 1, cap)
//   1 choose  (do-all): best of the own cell and the unoccupied cells up to
//             `vision` away along the four axes: most sugar, then nearest,
//             then lowest index; a move request is an atomicMin of the own
//             cell index into req[target]
//   2 move    (do-all): the lowest requesting cell index wins the target
//   3 eat     (do-all): sugar += cell; cell = 0; sugar -= metabolism; age++;
//             die (delete) if sugar <= 0 or age >= max_age
//   4 request (do-all): fertile agents with enough sugar request their
//             lowest-index empty von Neumann neighbour (atomicMin)
//   5 birth   (do-all): the winner creates a child there with half its sugar
//             and traits drawn from hash(seed, stream, t, cell)
// Phases read occupancy only as it was when the phase started and change it
// only where no other agent of the phase looks, so the result does not depend
// on which lane or block runs first.
#include <string.h>

#include <algorithm>
#include <new>

#include "internal.hpp"

namespace dsoar {
namespace {

enum : uint32_t { kAgent = 0 };
enum : uint32_t { kSugar = 0, kMetab = 1, kVision = 2, kAge = 3, kPos = 4, kTarget = 5, kWorld = 6 };
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint64_t kStreamChildMetab = 10, kStreamChildVision = 11;

// SplitMix64 output finaliser (Steele, Lea, Flood, OOPSLA 2014) and the
// workload hash h(seed, stream, a, b) = mix(mix(mix(seed ^ stream*golden) ^ a) ^ b).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ uint64_t hash4(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(seed ^ (stream * 0x9E3779B97F4A7C15ull)) ^ a) ^ b);
}
// U{lo..hi}: lo + floor(top32(h) * (hi - lo + 1) / 2^32).
__device__ __forceinline__ int32_t uniform_int(uint64_t h, int32_t lo, int32_t hi) {
  return lo + (int32_t)(((h >> 32) * (uint64_t)(hi - lo + 1)) >> 32);
}

// World table and grids.  Every world lives in its own range [off, off +
// side^2) of the cell arena; pos and target are arena indices.  Each slot has
// its own seed, step index and move count, so a world evolves exactly as it
// would alone.
// A cell's sugar is one byte, its low seven bits the amount and the top bit
// the occupancy (kOccupied), so that the cells an agent looks at take one
// load each and the grid of a 2048^2 world (4 MB) stays in an XCD's L2; occ
// keeps the agent handle.  Amounts and capacities are 0..kMaxSugar.
constexpr int32_t kOccupied = 0x80;
constexpr int32_t kMaxSugar = 0x7F;
__device__ __forceinline__ int32_t sugar_of(int32_t w) { return w & kMaxSugar; }

struct Grid {
  uint8_t* sugar;     // sugar | kOccupied when an agent stands there
  const int32_t* cap;
  uint32_t* occ;      // agent handle or kNull
  uint32_t* req;      // lowest requesting cell index or kInf
  uint32_t* breq;
  uint32_t* w_off;    // per slot
  uint32_t* w_side;
  uint64_t* w_seed;
  uint32_t* w_step;   // index of the step in progress
  uint64_t* w_moves;  // per slot, kMoveShards counters
  uint32_t arena;
  uint32_t max_worlds;
  int32_t max_age, repro_min, fertile_min, fertile_max;
};

constexpr uint32_t kMoveShards = 64;

__device__ __forceinline__ uint32_t wrap_cell(uint32_t off, int32_t side, int32_t x, int32_t y) {
  x %= side;
  if (x < 0) x += side;
  y %= side;
  if (y < 0) y += side;
  return off + (uint32_t)y * (uint32_t)side + (uint32_t)x;
}

template <class F, class H>
__device__ __forceinline__ F& af(const H& h, uint32_t self, uint32_t field) {
  return *field_ptr<F>(h, self, kAgent, field);
}

struct Where {
  uint32_t off;
  int32_t side, x, y;
};

__device__ __forceinline__ Where where(const Grid& g, uint32_t wid, uint32_t p) {
  const uint32_t off = g.w_off[wid], side = g.w_side[wid];
  const uint32_t local = p - off;
  return Where{off, (int32_t)side, (int32_t)(local % side), (int32_t)(local / side)};
}

// Cell at offset (dx*k, dy*k) from (x, y) on a torus of side `side`.
__device__ __forceinline__ uint32_t step_cell(const Where& c, int32_t dx, int32_t dy, int32_t k) {
  int32_t x = c.x + dx * k, y = c.y + dy * k;
  if (x < 0 || x >= c.side || y < 0 || y >= c.side) return wrap_cell(c.off, c.side, x, y);
  return c.off + (uint32_t)y * (uint32_t)c.side + (uint32_t)x;
}

constexpr int32_t kMaxVision = 6;

struct Choose {
  static constexpr uint32_t kKind = 40;
  using Args = Grid;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& g) {
    const uint32_t p = af<uint32_t>(h, self, kPos);
    const int32_t vision = af<int32_t>(h, self, kVision);
    const Where c = where(g, af<uint32_t>(h, self, kWorld), p);
    // The cells in sight along two axis directions at a time (beyond
    // `vision` the own cell stands in, so that the loads of a half are all
    // issued together, unconditionally), then the choice: most sugar, then
    // nearest, then lowest index.  The order in which the candidates are
    // compared does not matter for that total order.
    uint32_t best = p;
    int32_t best_sugar = sugar_of(g.sugar[p]), best_dist = 0;
#pragma unroll
    for (int32_t half = 0; half < 2; ++half) {
      uint32_t q[2 * kMaxVision];
      int32_t sg[2 * kMaxVision];
#pragma unroll
      for (int32_t j = 0; j < 2; ++j)
#pragma unroll
        for (int32_t k = 1; k <= kMaxVision; ++k) {
          const int32_t d = 2 * half + j;
          const int32_t dx = d == 0 ? 1 : (d == 1 ? -1 : 0);
          const int32_t dy = d == 2 ? 1 : (d == 3 ? -1 : 0);
          q[j * kMaxVision + k - 1] = k <= vision ? step_cell(c, dx, dy, k) : p;
        }
#pragma unroll
      for (int32_t i = 0; i < 2 * kMaxVision; ++i) sg[i] = g.sugar[q[i]];
#pragma unroll
      for (int32_t i = 0; i < 2 * kMaxVision; ++i) {
        const int32_t k = i % kMaxVision + 1;
        if (k > vision || (sg[i] & kOccupied)) continue;
        const int32_t s = sg[i];
        if (s > best_sugar || (s == best_sugar && (k < best_dist || (k == best_dist && q[i] < best)))) {
          best = q[i];
          best_sugar = s;
          best_dist = k;
        }
      }
    }
    af<uint32_t>(h, self, kTarget) = best;
    if (best != p) atomicMin(g.req + best, p);
    wave_count(h, kCntMethodAtomics, best != p ? 1u : 0u);
    return false;
  }
};

struct Move {
  static constexpr uint32_t kKind = 41;
  using Args = Grid;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& g) {
    const uint32_t p = af<uint32_t>(h, self, kPos);
    const uint32_t q = af<uint32_t>(h, self, kTarget);
    const uint32_t wid = af<uint32_t>(h, self, kWorld);
    const bool moves = q != p && __hip_atomic_load(g.req + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == p;
    if (moves) {
      // Distinct cells per mover: q was empty and p occupied when chosen.
      g.occ[q] = self;
      g.occ[p] = kNull;
      g.sugar[q] = (uint8_t)(g.sugar[q] | kOccupied);
      g.sugar[p] = (uint8_t)sugar_of(g.sugar[p]);
      af<uint32_t>(h, self, kPos) = q;
      __hip_atomic_store(g.req + q, kInf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Count moves per world: one sharded atomic per world present in the wavefront.
    uint64_t pending = __ballot(moves);
    const uint32_t sh = (blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) & (kMoveShards - 1);
    while (pending) {
      const uint32_t w0 = __builtin_amdgcn_readlane(wid, (uint32_t)__builtin_ctzll(pending));
      const uint64_t mine = __ballot(moves && wid == w0);
      lead_add(g.w_moves + (uint64_t)w0 * kMoveShards + sh, (uint64_t)__popcll(mine));
      pending &= ~mine;
    }
    return false;
  }
};

struct Eat {
  static constexpr uint32_t kKind = 42;
  static constexpr uint32_t kMinWaves = 8;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = Grid;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& g) {
    const uint32_t p = af<uint32_t>(h, self, kPos);
    const int32_t sugar = af<int32_t>(h, self, kSugar) + sugar_of(g.sugar[p]) - af<int32_t>(h, self, kMetab);
    const int32_t age = af<int32_t>(h, self, kAge) + 1;
    if (sugar <= 0 || age >= g.max_age) {
      g.sugar[p] = 0;
      g.occ[p] = kNull;
      return true;  // delete this; its fields are not written
    }
    g.sugar[p] = kOccupied;  // eaten, still here
    af<int32_t>(h, self, kSugar) = sugar;
    af<int32_t>(h, self, kAge) = age;
    return false;
  }
};

struct Request {
  static constexpr uint32_t kKind = 43;
  using Args = Grid;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& g) {
    const int32_t sugar = af<int32_t>(h, self, kSugar), age = af<int32_t>(h, self, kAge);
    uint32_t best = kNull;
    if (sugar >= g.repro_min && age >= g.fertile_min && age <= g.fertile_max) {
      const uint32_t p = af<uint32_t>(h, self, kPos);
      const Where c = where(g, af<uint32_t>(h, self, kWorld), p);
      const uint32_t nb[4] = {wrap_cell(c.off, c.side, c.x + 1, c.y), wrap_cell(c.off, c.side, c.x - 1, c.y),
                              wrap_cell(c.off, c.side, c.x, c.y + 1), wrap_cell(c.off, c.side, c.x, c.y - 1)};
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (g.occ[nb[d]] == kNull && nb[d] < best) best = nb[d];
      if (best != kNull) atomicMin(g.breq + best, p);
    }
    af<uint32_t>(h, self, kTarget) = best;
    wave_count(h, kCntMethodAtomics, best != kNull ? 1u : 0u);
    return false;
  }
};

struct Birth {
  static constexpr uint32_t kKind = 44;
  static constexpr uint32_t kMinWaves = 8;
  using Args = Grid;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& g) {
    const uint32_t n = af<uint32_t>(h, self, kTarget);
    const uint32_t p = af<uint32_t>(h, self, kPos);
    const uint32_t wid = af<uint32_t>(h, self, kWorld);
    const bool wins = n != kNull && __hip_atomic_load(g.breq + n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == p;
    int32_t give = 0;
    if (wins) {
      const int32_t sugar = af<int32_t>(h, self, kSugar);
      give = sugar / 2;
      af<int32_t>(h, self, kSugar) = sugar - give;
      __hip_atomic_store(g.breq + n, kInf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    new_many(h, kAgent, wins ? 1u : 0u, [&](uint32_t, uint32_t o) {
      if (o == kNull) return;
      const uint64_t seed = g.w_seed[wid];
      const uint32_t t = g.w_step[wid], local = n - g.w_off[wid];
      af<int32_t>(h, o, kSugar) = give;
      af<int32_t>(h, o, kMetab) = uniform_int(hash4(seed, kStreamChildMetab, t, local), 1, 4);
      af<int32_t>(h, o, kVision) = uniform_int(hash4(seed, kStreamChildVision, t, local), 1, 6);
      af<int32_t>(h, o, kAge) = 0;
      af<uint32_t>(h, o, kPos) = n;
      af<uint32_t>(h, o, kTarget) = kNull;
      af<uint32_t>(h, o, kWorld) = wid;
      g.occ[n] = o;
      g.sugar[n] = (uint8_t)(g.sugar[n] | kOccupied);
    });
    return false;
  }
};

struct SugarDeleteWorld {
  static constexpr uint32_t kKind = 45;
  struct Args { uint32_t slot; };
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    return af<uint32_t>(h, self, kWorld) == a.slot;
  }
};

// Regrow every arena cell, and advance every slot's step index (read by the
// births of this step).  Cells outside resident worlds are rewritten at
// admission, so regrowing them is harmless.
__global__ void regrow_kernel(Grid g) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.max_worlds) g.w_step[i] += 1;
  for (uint32_t c = i; c < g.arena; c += gridDim.x * blockDim.x) {
    const int32_t w = g.sugar[c], s = sugar_of(w) + 1, k = g.cap[c];
    g.sugar[c] = (uint8_t)((s < k ? s : k) | (w & kOccupied));
  }
}

__global__ void set_world_kernel(Grid g, uint32_t slot, uint32_t off, uint32_t side, uint64_t seed, uint32_t step0) {
  const uint32_t i = threadIdx.x;
  if (i == 0) {
    g.w_off[slot] = off;
    g.w_side[slot] = side;
    g.w_seed[slot] = seed;
    g.w_step[slot] = step0 - 1;  // the first regrow advances it to step0
  }
  if (i < kMoveShards) g.w_moves[(uint64_t)slot * kMoveShards + i] = 0;
}

// Admission input check: *bad = 1 if any cell's sugar or capacity lies
// outside 0..kMaxSugar (a cell keeps both in seven bits).
__global__ void sugar_zero_kernel(uint32_t* bad) { *bad = 0; }
__global__ void sugar_check_kernel(const int32_t* sugar, const int32_t* cap, uint32_t n, uint32_t* bad) {
  bool out = false;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    out |= sugar[c] < 0 || sugar[c] > kMaxSugar || cap[c] < 0 || cap[c] > kMaxSugar;
  if (__ballot(out) && is_first_active()) *bad = 1;
}

template <uint32_t LG>
__global__ void sugar_admit_kernel(DevHeapW<LG> h, Grid g, uint32_t slot, uint32_t off, uint32_t n, const int32_t* sugar,
                                   const int32_t* cap, const uint8_t* occ, const int32_t* as, const int32_t* am,
                                   const int32_t* av, const int32_t* aa) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t q = off + c;
  g.sugar[q] = (uint8_t)sugar[c];  // checked to be 0..kMaxSugar before the launch
  const_cast<int32_t*>(g.cap)[q] = cap[c];
  g.req[q] = kInf;
  g.breq[q] = kInf;
  g.occ[q] = kNull;
  new_many(h, kAgent, occ[c] ? 1u : 0u, [&](uint32_t, uint32_t o) {
    if (o == kNull) return;
    af<int32_t>(h, o, kSugar) = as[c];
    af<int32_t>(h, o, kMetab) = am[c];
    af<int32_t>(h, o, kVision) = av[c];
    af<int32_t>(h, o, kAge) = aa[c];
    af<uint32_t>(h, o, kPos) = q;
    af<uint32_t>(h, o, kTarget) = kNull;
    af<uint32_t>(h, o, kWorld) = slot;
    g.occ[q] = o;
    g.sugar[q] = (uint8_t)(g.sugar[q] | kOccupied);
  });
}

__global__ void sugar_read_kernel(DevHeap h, Grid g, uint32_t off, uint32_t n, int32_t* sugar, uint8_t* occ,
                                  int32_t* as, int32_t* am, int32_t* av, int32_t* aa) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t q = off + c;
  sugar[c] = sugar_of(g.sugar[q]);
  const uint32_t o = g.occ[q];
  occ[c] = o != kNull;
  as[c] = o != kNull ? af<int32_t>(h, o, kSugar) : 0;
  am[c] = o != kNull ? af<int32_t>(h, o, kMetab) : 0;
  av[c] = o != kNull ? af<int32_t>(h, o, kVision) : 0;
  aa[c] = o != kNull ? af<int32_t>(h, o, kAge) : 0;
}

bool sugar_heap_ok(const dsoar_heap* h) {
  const dsoar_type_layout& L = h->desc.types[0];
  if (L.num_fields < 7) return false;
  for (uint32_t f = 0; f < 7; ++f)
    if (L.field_bytes[f] != 4) return false;
  return true;
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

struct dsoar_sugar {
  dsoar_heap* heap;
  Grid g;
  uint32_t* bad_input;  // device word: admission input outside 0..kMaxSugar
  uint64_t default_seed;
  uint32_t* h_off;
  uint32_t* h_side;
  uint8_t* live;
  StepGraphs graphs;
};

namespace {

int sugar_one_step(dsoar_sugar* s, uint32_t flags, hipStream_t st) {
  dsoar_heap* h = s->heap;
  const uint32_t base = flags & DSOAR_DO_PLAIN;
  const uint32_t grid = std::min<uint32_t>(std::max<uint32_t>((s->g.arena + 255) / 256, (s->g.max_worlds + 255) / 256),
                                           std::max<uint32_t>(h->num_cus * 16, (s->g.max_worlds + 255) / 256));
  launch_timed(s->heap, kKindSugarRegrow, regrow_kernel, dim3(grid), dim3(256), st, s->g);
  DSOAR_LAUNCHED(h);
  int rc = launch_doall<Choose>(h, kAgent, s->g, base, st);
  // choose and move create and delete nothing: move and eat reuse the list.
  if (!rc) rc = launch_doall<Move>(h, kAgent, s->g, base | DSOAR_DO_REUSE_ENUM, st);
  if (!rc) rc = launch_doall<Eat>(h, kAgent, s->g, base | DSOAR_DO_REUSE_ENUM, st);
  // eat deletes: the request phase enumerates again; birth reuses that list.
  if (!rc) rc = launch_doall<Request>(h, kAgent, s->g, base, st);
  if (!rc) rc = launch_doall<Birth>(h, kAgent, s->g, base | DSOAR_DO_REUSE_ENUM, st);
  return rc;
}

size_t plane_bytes(uint64_t cells) { return (size_t)((cells * 4 + 255) / 256 * 256); }

// World table: seeds, offsets, sides, steps; the move counters; one 256-byte
// line for the admission input check.
size_t table_bytes(uint32_t max_worlds) {
  return (size_t)(((uint64_t)max_worlds * (4 + 4 + 8 + 4) + 255) / 256 * 256 +
                  ((uint64_t)max_worlds * kMoveShards * 8 + 255) / 256 * 256 + 256);
}

}  // namespace

extern "C" {

size_t dsoar_sugarpool_bytes(uint32_t max_worlds, uint32_t arena_cells) {
  if (max_worlds == 0 || max_worlds > (1u << 16) || arena_cells == 0 || arena_cells > (1u << 30)) return 0;
  return table_bytes(max_worlds) + 5 * plane_bytes(arena_cells);
}

int dsoar_sugarpool_create(dsoar_heap* heap, uint32_t max_worlds, uint32_t arena_cells,
                           const dsoar_sugar_rules* rules, void* dev_mem, size_t dev_bytes, dsoar_sugar** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !sugar_heap_ok(heap) || !rules || !dev_mem || ((uintptr_t)dev_mem & 255u))
    return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_sugarpool_bytes(max_worlds, arena_cells);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_sugar* s = new (std::nothrow) dsoar_sugar;
  if (!s) return DSOAR_ERR_INVALID_ARG;
  memset(s, 0, sizeof(*s));
  s->heap = heap;
  s->default_seed = rules->seed;
  s->h_off = (uint32_t*)calloc(max_worlds, 4);
  s->h_side = (uint32_t*)calloc(max_worlds, 4);
  s->live = (uint8_t*)calloc(max_worlds, 1);
  if (!s->h_off || !s->h_side || !s->live) {
    free(s->h_off);
    free(s->h_side);
    free(s->live);
    delete s;
    return DSOAR_ERR_INVALID_ARG;
  }
  uint8_t* b = (uint8_t*)dev_mem;
  Grid& g = s->g;
  g.w_seed = (uint64_t*)b;                                   // 8-byte entries first
  g.w_off = (uint32_t*)(b + (uint64_t)max_worlds * 8);
  g.w_side = g.w_off + max_worlds;
  g.w_step = g.w_side + max_worlds;
  g.w_moves = (uint64_t*)(b + ((uint64_t)max_worlds * 20 + 255) / 256 * 256);
  s->bad_input = (uint32_t*)(b + table_bytes(max_worlds) - 256);
  uint8_t* planes = b + table_bytes(max_worlds);
  const uint64_t plane = plane_bytes(arena_cells);
  g.sugar = planes;  // one byte per cell in a plane sized like the others
  g.cap = (const int32_t*)(planes + plane);
  g.occ = (uint32_t*)(planes + 2 * plane);
  g.req = (uint32_t*)(planes + 3 * plane);
  g.breq = (uint32_t*)(planes + 4 * plane);
  g.arena = arena_cells;
  g.max_worlds = max_worlds;
  g.max_age = rules->max_age;
  g.repro_min = rules->repro_min;
  g.fertile_min = rules->fertile_min;
  g.fertile_max = rules->fertile_max;
  *out = s;
  return DSOAR_OK;
}

int dsoar_sugar_admit(dsoar_sugar* s, uint32_t slot, uint32_t cell_offset, uint32_t side, uint64_t seed,
                      uint32_t step0, const int32_t* sugar_dev, const int32_t* cap_dev, const uint8_t* occ_dev,
                      const int32_t* a_sugar_dev, const int32_t* a_metab_dev, const int32_t* a_vision_dev,
                      const int32_t* a_age_dev, void* stream) {
  if (!s || slot >= s->g.max_worlds || s->live[slot] || side == 0 || side > 32768 || !sugar_dev || !cap_dev ||
      !occ_dev || !a_sugar_dev || !a_metab_dev || !a_vision_dev || !a_age_dev)
    return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)side * side;
  if ((uint64_t)cell_offset + n > s->g.arena) return DSOAR_ERR_INVALID_ARG;
  for (uint32_t k = 0; k < s->g.max_worlds; ++k)
    if (s->live[k] && cell_offset < s->h_off[k] + (uint64_t)s->h_side[k] * s->h_side[k] && s->h_off[k] < cell_offset + n)
      return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  // Sugar and capacities outside the seven bits a cell keeps them in are
  // refused before anything of the pool changes (synchronises the stream).
  hipLaunchKernelGGL(sugar_zero_kernel, dim3(1), dim3(1), 0, st, s->bad_input);
  DSOAR_LAUNCHED(s->heap);
  hipLaunchKernelGGL(sugar_check_kernel, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                     sugar_dev, cap_dev, (uint32_t)n, s->bad_input);
  DSOAR_LAUNCHED(s->heap);
  uint32_t bad = 0;
  DSOAR_HIP(s->heap, hipMemcpyAsync(&bad, s->bad_input, 4, hipMemcpyDeviceToHost, st));
  DSOAR_HIP(s->heap, hipStreamSynchronize(st));
  if (bad) return DSOAR_ERR_INVALID_ARG;
  hipLaunchKernelGGL(set_world_kernel, dim3(1), dim3(kMoveShards), 0, st, s->g, slot, cell_offset, side, seed, step0);
  DSOAR_LAUNCHED(s->heap);
  with_width(s->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(s->heap, kKindSugarAdmit, sugar_admit_kernel<kLG>, dim3((uint32_t)((n + 255) / 256)), dim3(256), st, DevHeapW<kLG>(s->heap->dev), s->g, slot,
                     cell_offset, (uint32_t)n, sugar_dev, cap_dev, occ_dev, a_sugar_dev, a_metab_dev, a_vision_dev,
                     a_age_dev);
  });
  DSOAR_LAUNCHED(s->heap);
  s->h_off[slot] = cell_offset;
  s->h_side[slot] = side;
  s->live[slot] = 1;
  return DSOAR_OK;
}

int dsoar_sugar_retire(dsoar_sugar* s, uint32_t slot, void* stream) {
  if (!s || slot >= s->g.max_worlds || !s->live[slot]) return DSOAR_ERR_INVALID_ARG;
  const int rc = launch_doall<SugarDeleteWorld>(s->heap, kAgent, SugarDeleteWorld::Args{slot}, 0, (hipStream_t)stream);
  if (rc) return rc;
  s->live[slot] = 0;
  return DSOAR_OK;
}

int dsoar_sugar_read_world(dsoar_sugar* s, uint32_t slot, int32_t* sugar_dev, uint8_t* occ_dev, int32_t* a_sugar_dev,
                           int32_t* a_metab_dev, int32_t* a_vision_dev, int32_t* a_age_dev, uint64_t* moves,
                           void* stream) {
  if (!s || slot >= s->g.max_worlds || !s->live[slot] || !sugar_dev || !occ_dev || !a_sugar_dev || !a_metab_dev ||
      !a_vision_dev || !a_age_dev)
    return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t n = s->h_side[slot] * s->h_side[slot];
  hipLaunchKernelGGL(sugar_read_kernel, dim3((n + 255) / 256), dim3(256), 0, st, s->heap->dev, s->g, s->h_off[slot], n,
                     sugar_dev, occ_dev, a_sugar_dev, a_metab_dev, a_vision_dev, a_age_dev);
  DSOAR_LAUNCHED(s->heap);
  if (moves) {
    uint64_t m[kMoveShards];
    DSOAR_HIP(s->heap, hipMemcpyAsync(m, s->g.w_moves + (uint64_t)slot * kMoveShards, sizeof(m), hipMemcpyDeviceToHost, st));
    DSOAR_HIP(s->heap, hipStreamSynchronize(st));
    uint64_t t = 0;
    for (uint32_t i = 0; i < kMoveShards; ++i) t += m[i];
    *moves = t;
  }
  return DSOAR_OK;
}

// Single-world interface: a pool of one slot covering the whole arena.
size_t dsoar_sugar_bytes(uint32_t side) {
  if (side < 1 || side > 32768) return 0;
  return dsoar_sugarpool_bytes(1, side * side);
}

int dsoar_sugar_create(dsoar_heap* heap, uint32_t side, const dsoar_sugar_rules* rules, void* dev_mem,
                       size_t dev_bytes, dsoar_sugar** out) {
  if (side < 1 || side > 32768) return DSOAR_ERR_INVALID_ARG;
  return dsoar_sugarpool_create(heap, 1, side * side, rules, dev_mem, dev_bytes, out);
}

int dsoar_sugar_destroy(dsoar_sugar* s) {
  if (!s) return DSOAR_ERR_INVALID_ARG;
  step_graphs_clear(s->graphs);
  free(s->h_off);
  free(s->h_side);
  free(s->live);
  delete s;
  return DSOAR_OK;
}

int dsoar_sugar_init(dsoar_sugar* s, const int32_t* sugar_dev, const int32_t* cap_dev, const uint8_t* occ_dev,
                     const int32_t* a_sugar_dev, const int32_t* a_metab_dev, const int32_t* a_vision_dev,
                     const int32_t* a_age_dev, uint32_t step0, void* stream) {
  if (!s) return DSOAR_ERR_INVALID_ARG;
  uint32_t side = 1;
  while ((uint64_t)side * side < s->g.arena) ++side;
  if ((uint64_t)side * side != s->g.arena) return DSOAR_ERR_INVALID_ARG;
  s->live[0] = 0;  // the heap is reset by the caller: slot 0 starts afresh
  return dsoar_sugar_admit(s, 0, 0, side, s->default_seed, step0, sugar_dev, cap_dev, occ_dev, a_sugar_dev,
                           a_metab_dev, a_vision_dev, a_age_dev, stream);
}

int dsoar_sugar_step(dsoar_sugar* s, uint32_t steps, uint32_t flags, void* stream) {
  if (!s) return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  dsoar_heap* h = s->heap;
  if (flags & DSOAR_GRAPH) {
    if (flags & DSOAR_DO_PLAIN) return DSOAR_ERR_INVALID_ARG;
    return step_graphs_run(h, s->graphs, steps, st, [&](hipStream_t gs) { return sugar_one_step(s, 0, gs); });
  }
  for (uint32_t i = 0; i < steps; ++i) {
    const int rc = sugar_one_step(s, flags, st);
    if (rc) return rc;
  }
  return DSOAR_OK;
}

int dsoar_sugar_read(dsoar_sugar* s, int32_t* sugar_dev, uint8_t* occ_dev, int32_t* a_sugar_dev, int32_t* a_metab_dev,
                     int32_t* a_vision_dev, int32_t* a_age_dev, uint32_t* moves, void* stream) {
  uint64_t m = 0;
  const int rc = dsoar_sugar_read_world(s, 0, sugar_dev, occ_dev, a_sugar_dev, a_metab_dev, a_vision_dev, a_age_dev,
                                        moves ? &m : nullptr, stream);
  if (!rc && moves) *moves = (uint32_t)m;
  return rc;
}

}  // extern "C"
