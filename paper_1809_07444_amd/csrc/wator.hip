// Wa-Tor as objects: fish and sharks on a square torus (the paper's "wator"
// application, Fig. 6h; Dewdney's rules, read as a synchronous step).  Fish
// {pos, age, target} and Shark {pos, age, energy, target} objects live in the
// heap; the sea is a plain cell -> kind array (0 empty, 1 fish, 2 shark) and a
// cell -> request word array.  One step t:
//   FishDecide (do-all Fish): on the sea at the start of the phase, pick the
//     k-th empty neighbour (up, right, down, left), k = U{0..n-1} from
//     hash(seed, 40, cell, t); request it (atomicMin of the phase key).
//   FishMove (same list): the lowest requesting cell wins; the winner moves
//     and, at age >= fish_breed, leaves a new Fish behind (both age 0).
//     Every fish ages by one.
//   SharkDecide (do-all Shark): on the sea after the fish phase, pick a
//     neighbouring fish (k from hash(seed, 41, cell, t)) or, with none and
//     energy above 1, an empty neighbour; request it.
//   SharkMove (same list): the lowest requesting cell wins; a winner that
//     lands on a fish eats it (energy = starve), any other shark loses one
//     unit and deletes itself at 0; breeding as for fish.
//   FishEaten (do-all Fish): a fish whose cell now holds a shark deletes
//     itself.
//   Tick: t += 1 (the step index lives on the device, so a captured step
//     replays correctly).
// Request words carry the phase in their high half (larger for earlier
// phases), so a phase's atomicMin always replaces what earlier phases left
// and the array never needs clearing.
#include <string.h>

#include <new>

#include "internal.hpp"

namespace dsoar {
namespace {

enum : uint32_t { kFish = 0, kShark = 1 };
enum : uint32_t { kPos = 0, kAge = 1, kFTarget = 2 };  // Fish fields
enum : uint32_t { kEnergy = 2, kSTarget = 3 };         // Shark fields after pos, age
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint8_t kEmpty = 0, kIsFish = 1, kIsShark = 2;
constexpr uint64_t kStreamFish = 40, kStreamShark = 41;

// SplitMix64 output finaliser (Steele, Lea, Flood, OOPSLA 2014) and the
// workload hash built on it: mix(mix(mix(seed ^ stream * golden) ^ a) ^ b).
__device__ __forceinline__ uint64_t finalise(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return finalise(finalise(finalise(seed ^ (stream * 0x9E3779B97F4A7C15ull)) ^ a) ^ b);
}
// U{0..n-1}: floor(top32(h) * n / 2^32).
__device__ __forceinline__ uint32_t pick(uint64_t h, uint32_t n) {
  return (uint32_t)(((h >> 32) * (uint64_t)n) >> 32);
}

struct Sea {
  uint8_t* kind;    // cell -> kEmpty, kIsFish or kIsShark (one byte: the sea of 2048^2 fits an L2)
  uint64_t* req;    // cell -> smallest request key of the latest phase that asked for it
  uint32_t* step;   // [0]: index of the step in progress
  uint32_t side;
  uint64_t seed;
  int32_t fish_breed, shark_breed, starve;
};

// Request key of cell c in phase `tag` (2t: fish, 2t + 1: sharks).
__device__ __forceinline__ uint64_t req_key(uint32_t tag, uint32_t c) {
  return ((uint64_t)(0xFFFFFFFFu - tag) << 32) | c;
}

// Neighbour d of cell c: up, right, down, left.
__device__ __forceinline__ uint32_t nb(uint32_t side, uint32_t c, uint32_t d) {
  const uint32_t y = c / side, x = c - y * side;
  uint32_t nx = x, ny = y;
  if (d == 0) ny = y == 0 ? side - 1 : y - 1;
  if (d == 1) nx = x + 1 == side ? 0 : x + 1;
  if (d == 2) ny = y + 1 == side ? 0 : y + 1;
  if (d == 3) nx = x == 0 ? side - 1 : x - 1;
  return ny * side + nx;
}

template <class F, class H>
__device__ __forceinline__ F& fish(const H& h, uint32_t self, uint32_t field) {
  return *field_ptr<F>(h, self, kFish, field);
}
template <class F, class H>
__device__ __forceinline__ F& shark(const H& h, uint32_t self, uint32_t field) {
  return *field_ptr<F>(h, self, kShark, field);
}

struct FishDecide {
  static constexpr uint32_t kKind = 70;
  using Args = Sea;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t t = a.step[0];
    const uint32_t c = fish<uint32_t>(h, self, kPos);
    uint32_t opt[4], m = 0;
#pragma unroll
    for (uint32_t d = 0; d < 4; ++d) {
      const uint32_t q = nb(a.side, c, d);
      if (a.kind[q] == kEmpty) opt[m++] = q;
    }
    uint32_t target = kNone;
    if (m > 0) {
      target = opt[pick(draw(a.seed, kStreamFish, c, t), m)];
      atomicMin((unsigned long long*)(a.req + target), (unsigned long long)req_key(2 * t, c));
    }
    fish<uint32_t>(h, self, kFTarget) = target;
    return false;
  }
};

struct FishMove {
  static constexpr uint32_t kKind = 71;
  static constexpr uint32_t kMinWaves = 8;
  using Args = Sea;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t t = a.step[0];
    const uint32_t c = fish<uint32_t>(h, self, kPos), target = fish<uint32_t>(h, self, kFTarget);
    const int32_t age = fish<int32_t>(h, self, kAge) + 1;
    const bool won = target != kNone && a.req[target] == req_key(2 * t, c);
    const bool breed = won && age >= a.fish_breed;
    if (won) {
      a.kind[target] = kIsFish;
      fish<uint32_t>(h, self, kPos) = target;
      if (!breed) a.kind[c] = kEmpty;  // else the newborn keeps the cell
    }
    fish<int32_t>(h, self, kAge) = breed ? 0 : age;
    new_many(h, kFish, breed ? 1u : 0u, [&](uint32_t, uint32_t o) {
      if (o == kNull) return;
      fish<uint32_t>(h, o, kPos) = c;
      fish<int32_t>(h, o, kAge) = 0;
      fish<uint32_t>(h, o, kFTarget) = kNone;
    });
    return false;
  }
};

struct SharkDecide {
  static constexpr uint32_t kKind = 72;
  using Args = Sea;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t t = a.step[0];
    const uint32_t c = shark<uint32_t>(h, self, kPos);
    uint32_t fishn[4], empty[4], nf = 0, ne = 0;
#pragma unroll
    for (uint32_t d = 0; d < 4; ++d) {
      const uint32_t q = nb(a.side, c, d);
      const uint8_t k = a.kind[q];
      if (k == kIsFish) fishn[nf++] = q;
      if (k == kEmpty) empty[ne++] = q;
    }
    const uint64_t hs = draw(a.seed, kStreamShark, c, t);
    uint32_t target = kNone;
    if (nf > 0)
      target = fishn[pick(hs, nf)];
    else if (ne > 0 && shark<int32_t>(h, self, kEnergy) > 1)
      target = empty[pick(hs, ne)];
    if (target != kNone)
      atomicMin((unsigned long long*)(a.req + target), (unsigned long long)req_key(2 * t + 1, c));
    shark<uint32_t>(h, self, kSTarget) = target;
    return false;
  }
};

struct SharkMove {
  static constexpr uint32_t kKind = 73;
  static constexpr uint32_t kMinWaves = 8;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = Sea;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t t = a.step[0];
    const uint32_t c = shark<uint32_t>(h, self, kPos), target = shark<uint32_t>(h, self, kSTarget);
    const bool won = target != kNone && a.req[target] == req_key(2 * t + 1, c);
    // Only the winner writes its target cell, and no shark targets a shark's
    // cell, so this read sees the sea as the fish phase left it.
    const bool ate = won && a.kind[target] == kIsFish;
    const int32_t energy = ate ? a.starve : shark<int32_t>(h, self, kEnergy) - 1;
    const int32_t age = shark<int32_t>(h, self, kAge) + 1;
    if (energy <= 0) {  // starved (a shark that eats never does)
      a.kind[c] = kEmpty;
      return true;
    }
    const bool breed = won && age >= a.shark_breed;
    if (won) {
      a.kind[target] = kIsShark;
      shark<uint32_t>(h, self, kPos) = target;
      if (!breed) a.kind[c] = kEmpty;
    }
    shark<int32_t>(h, self, kEnergy) = energy;
    shark<int32_t>(h, self, kAge) = breed ? 0 : age;
    new_many(h, kShark, breed ? 1u : 0u, [&](uint32_t, uint32_t o) {
      if (o == kNull) return;
      shark<uint32_t>(h, o, kPos) = c;
      shark<int32_t>(h, o, kAge) = 0;
      shark<int32_t>(h, o, kEnergy) = a.starve;
      shark<uint32_t>(h, o, kSTarget) = kNone;
    });
    return false;
  }
};

struct FishEaten {
  static constexpr uint32_t kKind = 74;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = Sea;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    return a.kind[fish<uint32_t>(h, self, kPos)] != kIsFish;
  }
};

struct ReadArgs {
  int32_t* age;
  int32_t* energy;
};

struct FishRead {
  static constexpr uint32_t kKind = 75;
  using Args = ReadArgs;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    a.age[fish<uint32_t>(h, self, kPos)] = fish<int32_t>(h, self, kAge);
    return false;
  }
};

struct SharkRead {
  static constexpr uint32_t kKind = 76;
  using Args = ReadArgs;
  template <class H>
  static __device__ bool run(const H& h, uint32_t, uint32_t self, const Args& a) {
    const uint32_t c = shark<uint32_t>(h, self, kPos);
    a.age[c] = shark<int32_t>(h, self, kAge);
    a.energy[c] = shark<int32_t>(h, self, kEnergy);
    return false;
  }
};

__global__ void tick_kernel(Sea a) { a.step[0] += 1; }

// Creates the objects of the initial sea, in cell order.
template <uint32_t LG>
__global__ void wator_init_kernel(DevHeapW<LG> h, Sea a, const int32_t* kind, const int32_t* age, const int32_t* energy,
                                  uint32_t step0) {
  const uint64_t n = (uint64_t)a.side * a.side;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) a.step[0] = step0;
  if (c >= n) return;
  const int32_t k = kind[c];
  a.kind[c] = (uint8_t)k;
  a.req[c] = ~0ull;
  new_many(h, kFish, k == kIsFish ? 1u : 0u, [&](uint32_t, uint32_t o) {
    if (o == kNull) return;
    fish<uint32_t>(h, o, kPos) = c;
    fish<int32_t>(h, o, kAge) = age[c];
    fish<uint32_t>(h, o, kFTarget) = kNone;
  });
  new_many(h, kShark, k == kIsShark ? 1u : 0u, [&](uint32_t, uint32_t o) {
    if (o == kNull) return;
    shark<uint32_t>(h, o, kPos) = c;
    shark<int32_t>(h, o, kAge) = age[c];
    shark<int32_t>(h, o, kEnergy) = energy[c];
    shark<uint32_t>(h, o, kSTarget) = kNone;
  });
}

// kind out, and zeroed age and energy (the read do-alls fill the occupied cells).
__global__ void wator_read_kernel(Sea a, int32_t* kind, int32_t* age, int32_t* energy) {
  const uint64_t n = (uint64_t)a.side * a.side;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  kind[c] = a.kind[c];
  age[c] = 0;
  energy[c] = 0;
}

bool wator_heap_ok(const dsoar_heap* h) {
  if (h->desc.num_types < 2) return false;
  const uint32_t want[2] = {3, 4};
  for (uint32_t t = 0; t < 2; ++t) {
    const dsoar_type_layout& L = h->desc.types[t];
    if (L.num_fields < want[t]) return false;
    for (uint32_t f = 0; f < want[t]; ++f)
      if (L.field_bytes[f] != 4) return false;
  }
  return true;
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

struct dsoar_wator {
  dsoar_heap* heap;
  Sea a;
  StepGraphs graphs;
};

namespace {

int wator_one_step(dsoar_wator* w, uint32_t flags, hipStream_t st) {
  dsoar_heap* h = w->heap;
  const uint32_t base = flags & DSOAR_DO_PLAIN, reuse = base | DSOAR_DO_REUSE_ENUM;
  // Decide creates and deletes nothing, so Move reuses its list; the newborns
  // of a Move are not visited by it (snapshot semantics).
  int rc = launch_doall<FishDecide>(h, kFish, w->a, base, st);
  if (!rc) rc = launch_doall<FishMove>(h, kFish, w->a, reuse, st);
  if (!rc) rc = launch_doall<SharkDecide>(h, kShark, w->a, base, st);
  if (!rc) rc = launch_doall<SharkMove>(h, kShark, w->a, reuse, st);
  if (!rc) rc = launch_doall<FishEaten>(h, kFish, w->a, base, st);
  if (rc) return rc;
  launch_timed(w->heap, kKindWatorTick, tick_kernel, dim3(1), dim3(1), st, w->a);
  DSOAR_LAUNCHED(h);
  return DSOAR_OK;
}

size_t round256(uint64_t b) { return (size_t)((b + 255) / 256 * 256); }

}  // namespace

extern "C" {

size_t dsoar_wator_bytes(uint32_t side) {
  const uint64_t n = (uint64_t)side * side;
  if (side == 0 || n > (1ull << 30)) return 0;
  return 256 + round256(n) + round256(n * 8);
}

int dsoar_wator_create(dsoar_heap* heap, uint32_t side, const dsoar_wator_rules* rules, void* dev_mem,
                       size_t dev_bytes, dsoar_wator** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !wator_heap_ok(heap) || !rules || !dev_mem || ((uintptr_t)dev_mem & 255u) ||
      rules->fish_breed < 1 || rules->shark_breed < 1 || rules->starve < 1)
    return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_wator_bytes(side);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_wator* w = new (std::nothrow) dsoar_wator;
  if (!w) return DSOAR_ERR_INVALID_ARG;
  memset(w, 0, sizeof(*w));
  const uint64_t n = (uint64_t)side * side;
  uint8_t* b = (uint8_t*)dev_mem;
  w->heap = heap;
  w->a.step = (uint32_t*)b;
  w->a.kind = b + 256;
  w->a.req = (uint64_t*)(b + 256 + round256(n));
  w->a.side = side;
  w->a.seed = rules->seed;
  w->a.fish_breed = rules->fish_breed;
  w->a.shark_breed = rules->shark_breed;
  w->a.starve = rules->starve;
  *out = w;
  return DSOAR_OK;
}

int dsoar_wator_destroy(dsoar_wator* w) {
  if (!w) return DSOAR_ERR_INVALID_ARG;
  step_graphs_clear(w->graphs);
  delete w;
  return DSOAR_OK;
}

int dsoar_wator_init(dsoar_wator* w, const int32_t* kind_dev, const int32_t* age_dev, const int32_t* energy_dev,
                     uint32_t step0, void* stream) {
  if (!w || !kind_dev || !age_dev || !energy_dev) return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)w->a.side * w->a.side;
  with_width(w->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    launch_timed(w->heap, kKindWatorInit, wator_init_kernel<kLG>, dim3((uint32_t)((n + 255) / 256)), dim3(256), (hipStream_t)stream,
                     DevHeapW<kLG>(w->heap->dev), w->a, kind_dev, age_dev, energy_dev, step0);
  });
  DSOAR_LAUNCHED(w->heap);
  return DSOAR_OK;
}

int dsoar_wator_step(dsoar_wator* w, uint32_t steps, uint32_t flags, void* stream) {
  if (!w) return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  dsoar_heap* h = w->heap;
  if (flags & DSOAR_GRAPH) {
    if (flags & DSOAR_DO_PLAIN) return DSOAR_ERR_INVALID_ARG;
    return step_graphs_run(h, w->graphs, steps, st, [&](hipStream_t gs) { return wator_one_step(w, 0, gs); });
  }
  for (uint32_t i = 0; i < steps; ++i) {
    const int rc = wator_one_step(w, flags, st);
    if (rc) return rc;
  }
  return DSOAR_OK;
}

int dsoar_wator_read(dsoar_wator* w, int32_t* kind_dev, int32_t* age_dev, int32_t* energy_dev, void* stream) {
  if (!w || !kind_dev || !age_dev || !energy_dev) return DSOAR_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t n = (uint64_t)w->a.side * w->a.side;
  hipLaunchKernelGGL(wator_read_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, w->a, kind_dev,
                     age_dev, energy_dev);
  DSOAR_LAUNCHED(w->heap);
  const ReadArgs r{age_dev, energy_dev};
  int rc = launch_doall<FishRead>(w->heap, kFish, r, DSOAR_DO_PERSISTENT, st);
  if (!rc) rc = launch_doall<SharkRead>(w->heap, kShark, r, DSOAR_DO_PERSISTENT, st);
  return rc;
}

}  // extern "C"
