// Game of Life as objects (B3/S23 on square tori), for one world or many
// worlds sharing one heap.
//
// Types: Cell {alive} is created once per grid position and found through a
// position -> handle index (a plane of live bits beside it copies the flags
// for the neighbour reads); Alive {cell, world, action} exists for every live
// cell; Candidate {cell, world, action} exists during a generation for every
// dead cell next to a live one.  One generation is four do-alls:
//   1 Alive:     count live neighbours -> action (die unless 2 or 3); create
//                the Candidate of each dead neighbour whose first live
//                neighbour (in a fixed direction order) is this cell, so
//                that every such cell gets exactly one, without atomics.
//   2 Candidate: action = born iff exactly 3 live neighbours.
//   3 Alive:     dying ones clear their Cell's alive flag and delete themselves.
//   4 Candidate: born ones set their Cell's alive flag and create an Alive;
//                every Candidate deletes itself.
// Live flags are only read in phases 1-2 and only written in 3-4, so the
// kernel boundaries make the update synchronous.
#include <string.h>

#include <new>

#include "internal.hpp"

namespace dsoar {
namespace {

enum : uint32_t { kCell = 0, kAlive = 1, kCand = 2 };
enum : uint32_t { kCAlive = 0 };
enum : uint32_t { kACell = 0, kAWorld = 1, kAAction = 2 };
constexpr uint32_t kKindGolUpdate = 35;  // timing id of the fused phases 3 and 4

// Beside the position -> Cell handle index, a live-bit plane holds a copy of
// every Cell's live flag, one bit per cell in the index's order (bit g % 32
// of word g / 32; a cell whose Cell is missing, only after an out-of-memory
// init, reads dead).  The neighbourhood reads of phases 1 and 2 load it: a
// row's five cells are one pair of dword loads, and the plane of all 256
// batched worlds (48.8 M cells) is 6 MB, so the rows that the neighbourhoods
// of a wavefront's scattered cells touch are few cache lines, many of them
// shared with other wavefronts.  Phases 3 and 4 (which read no neighbours)
// flip the bits of the cells that die or are born with atomic AND / OR.
struct World {
  const uint32_t* cells;  // global cell index -> Cell handle (kNull if missing)
  const uint32_t* bits;   // live bits
  const uint32_t* off;    // world -> first global cell index (num_worlds + 1 entries)
  const uint32_t* side;   // world -> side length
};

// Sets the live state of the Cell at global index g, whose handle is wd
// (its field and its bit); only the cell's own Alive or Candidate does this.
// False if the Cell is missing (after an out-of-memory init).
template <class H>
__device__ __forceinline__ bool set_cell_live(const H& h, const World& w, uint32_t g, uint32_t wd, uint32_t live) {
  if (wd == kNull) return false;
  *field_ptr<uint32_t>(h, wd, kCell, kCAlive) = live;
  uint32_t* word = const_cast<uint32_t*>(w.bits) + (g >> 5);
  const uint32_t bit = 1u << (g & 31u);
  if (live)
    __hip_atomic_fetch_or(word, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    __hip_atomic_fetch_and(word, ~bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Writes the live bits of a run of consecutive cells held by the lanes of a
// wavefront in order (lane l: cell g of lane 0 plus l; lanes past the run's
// end pass in = false): the lane at the head of each 32-bit word's part of
// the run clears that part (if `clear`) and sets the bits of its live cells,
// so that runs of other wavefronts or worlds that share the word stay intact.
__device__ __forceinline__ void write_live_run(uint32_t* bits, uint32_t g, bool in, bool live, bool clear) {
  const uint32_t lane = lane_id();
  const uint64_t inm = __ballot(in), lm = __ballot(in && live);
  const uint32_t sh = g & 31u;
  if (!in || (lane != 0 && sh != 0)) return;
  const uint32_t cnt = 32u - sh < 64u - lane ? 32u - sh : 64u - lane;  // lanes of this word, <= 32
  const uint64_t run = ((1ull << cnt) - 1ull) << lane;
  const uint32_t rm = (uint32_t)((inm & run) >> lane) << sh;
  const uint32_t lv = (uint32_t)((lm & run) >> lane) << sh;
  uint32_t* word = bits + (g >> 5);
  if (clear) __hip_atomic_fetch_and(word, ~rm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (lv) __hip_atomic_fetch_or(word, lv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global index of neighbour d (0..7: the row above, left and right, the row
// below) of cell (x, y) of a world at offset `off` with side `side`.
__device__ __forceinline__ uint32_t neighbour(uint32_t off, uint32_t side, uint32_t x, uint32_t y, uint32_t d) {
  const uint32_t ddx = (0x9224u >> (2 * d)) & 3u;  // dx + 1 for d = 0..7: 0 1 2 0 2 0 1 2
  const uint32_t ddy = (0xA940u >> (2 * d)) & 3u;  // dy + 1 for d = 0..7: 0 0 0 1 1 2 2 2
  uint32_t nx = x + ddx, ny = y + ddy;              // shifted by +1, wrap below
  nx = nx == 0 ? side - 1 : (nx - 1 == side ? 0 : nx - 1);
  ny = ny == 0 ? side - 1 : (ny - 1 == side ? 0 : ny - 1);
  return off + ny * side + nx;
}

// The 5 x 5 neighbourhood of a cell: bit (dy + 2) * 5 + (dx + 2) for the
// cell at offset (dx, dy).  Directions d = 0..7 in the order of neighbour();
// direction 7 - d is the opposite of direction d.
constexpr int kDirX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
constexpr int kDirY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
constexpr uint32_t nb_bit(int dx, int dy) { return (uint32_t)((dy + 2) * 5 + dx + 2); }

// A dead cell's Candidate is created by the first of its live neighbours in
// direction order.  The dead neighbour in direction d sees this cell in
// direction 7 - d, so this cell creates it iff none of the dead cell's
// neighbours in the directions before 7 - d is alive; owner_mask(d) holds
// those cells.  On a torus smaller than 5 x 5 several offsets name one cell:
// each offset is loaded from the cell it names, so the rule still picks one
// creator per dead cell.
constexpr uint32_t owner_mask(uint32_t d) {
  uint32_t m = 0;
  for (uint32_t e = 0; e + d < 7; ++e) m |= 1u << nb_bit(kDirX[d] + kDirX[e], kDirY[d] + kDirY[e]);
  return m;
}
constexpr uint32_t ring_mask() {
  uint32_t m = 0;
  for (uint32_t d = 0; d < 8; ++d) m |= 1u << nb_bit(kDirX[d], kDirY[d]);
  return m;
}

// x + dx on a torus of side `side`, dx in -2..2 (any side >= 1).
__device__ __forceinline__ uint32_t torus_add(uint32_t x, int dx, uint32_t side) {
  int v = (int)x + dx;
  const int s = (int)side;
  v = v < 0 ? v + s : v;
  v = v < 0 ? v + s : v;
  v = v >= s ? v - s : v;
  v = v >= s ? v - s : v;
  return (uint32_t)v;
}

// The (2R + 1) x (2R + 1) neighbourhood of cell (x, y) of the world at `off`
// with side `side`, from the live-bit plane: bit (dy + R) * (2R + 1) + (dx +
// R) is set for a live cell at offset (dx, dy); the centre is left out.  A
// row whose window does not wrap around the torus is one pair of dword loads
// shifted into place (the bit plane is padded, so a read past the last cell
// stays in the buffer); a row that wraps loads its cells one by one.
template <int R>
__device__ __forceinline__ uint32_t neighbourhood(const uint32_t* bits, uint32_t off, uint32_t side, uint32_t x,
                                                  uint32_t y) {
  constexpr int D = 2 * R + 1;
  const bool inside = x >= (uint32_t)R && x + R < side;
  uint32_t al = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const uint32_t rb = off + torus_add(y, i - R, side) * side;  // bit index of the row's first cell
    uint32_t v = 0;
    if (inside) {
      const uint32_t a = rb + x - R;
      const uint32_t* p = bits + (a >> 5);
      v = (uint32_t)((((uint64_t)p[1] << 32) | p[0]) >> (a & 31u));
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const uint32_t c = rb + torus_add(x, j - R, side);
        v |= ((bits[c >> 5] >> (c & 31u)) & 1u) << j;
      }
    }
    al |= (v & ((1u << D) - 1u)) << (i * D);
  }
  return al & ~(1u << (R * D + R));
}

// A listed object's cell position.  The do-all methods take two blocks per
// wavefront pass (run_pair): each lane reads both of its slots' fields and
// then both positions' neighbourhoods before it uses any of them (a
// wavefront whose second block is absent skips its reads).  A slot that is
// not live reads as world 0's corner (side 1 stands in when the world
// table's slot 0 is empty), so no index is ever formed from its fields.
struct CellPos {
  uint32_t wid, off, side, x, y;
};
__device__ __forceinline__ CellPos cell_pos(const World& w, uint32_t g, uint32_t wid, bool live) {
  const uint32_t wi = live ? wid : 0u;
  const uint32_t o = w.off[wi], sd = w.side[wi];
  CellPos p;
  p.wid = wi;
  p.off = live ? o : 0u;
  p.side = live ? sd : 1u;
  const uint32_t local = live ? g - p.off : 0u;
  p.y = local / p.side;
  p.x = local - p.y * p.side;
  return p;
}

struct AlivePrep {
  static constexpr uint32_t kKind = 30;
  using Args = World;
  template <class H>
  static __device__ __forceinline__ void run_pair(const H& h, uint32_t type, uint32_t s0, bool l0, uint32_t s1,
                                                  bool l1, const Args& w, bool& d0, bool& d1) {
    const uint32_t self[2] = {s0, s1};
    const bool lv[2] = {l0, l1};
    const uint32_t n = __ballot(l1) ? 2u : 1u;  // objects this wavefront holds per lane
    uint32_t g[2] = {0, 0}, wid[2] = {0, 0};
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      g[u] = *field_ptr<uint32_t>(h, self[u], type, kACell);
      wid[u] = *field_ptr<uint32_t>(h, self[u], type, kAWorld);
    }
    CellPos p[2];
    uint32_t alive[2] = {0, 0};
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) p[u] = cell_pos(w, g[u], wid[u], lv[u] && u < n);
    // Live states of the 24 surrounding cells.  (A cell whose Cell is
    // missing reads as dead; its Candidate never becomes an Alive.)
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      alive[u] = neighbourhood<2>(w.bits, p[u].off, p[u].side, p[u].x, p[u].y);
    }
    uint32_t claim[2];
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      claim[u] = 0;
#pragma unroll
      for (uint32_t d = 0; d < 8; ++d) {
        const uint32_t b = nb_bit(kDirX[d], kDirY[d]);
        const bool dead = (~alive[u] >> b) & 1u;
        if (dead && !(alive[u] & owner_mask(d))) claim[u] |= 1u << d;
      }
      if (!lv[u]) claim[u] = 0;
    }
    // One coalesced allocation for the new Candidates of both blocks.
    const uint32_t k0 = (uint32_t)__popc(claim[0]);
    new_many(h, kCand, k0 + (uint32_t)__popc(claim[1]), [&](uint32_t j, uint32_t o) {
      if (o == kNull) return;
      const uint32_t u = j < k0 ? 0u : 1u;
      const CellPos& q = u ? p[1] : p[0];
      const uint32_t n = neighbour(q.off, q.side, q.x, q.y, nth_set_bit(claim[u], u ? j - k0 : j));
      *field_ptr<uint32_t>(h, o, kCand, kACell) = n;
      *field_ptr<uint32_t>(h, o, kCand, kAWorld) = q.wid;
      *field_ptr<uint32_t>(h, o, kCand, kAAction) = 0;
    });
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      const uint32_t live = (uint32_t)__popc(alive[u] & ring_mask());
      if (lv[u]) *field_ptr<uint32_t>(h, self[u], type, kAAction) = (live == 2 || live == 3) ? 0u : 1u;
    }
    d0 = d1 = false;
  }
  template <class H>
  static __device__ __forceinline__ bool run(const H& h, uint32_t type, uint32_t self, const Args& w) {
    const uint32_t g = *field_ptr<uint32_t>(h, self, type, kACell);
    const uint32_t wid = *field_ptr<uint32_t>(h, self, type, kAWorld);
    const uint32_t off = w.off[wid], side = w.side[wid];
    const uint32_t local = g - off;
    const uint32_t y = local / side, x = local - y * side;
    const uint32_t alive = neighbourhood<2>(w.bits, off, side, x, y);
    uint32_t claim = 0;
#pragma unroll
    for (uint32_t d = 0; d < 8; ++d) {
      const uint32_t b = nb_bit(kDirX[d], kDirY[d]);
      const bool dead = (~alive >> b) & 1u;
      if (dead && !(alive & owner_mask(d))) claim |= 1u << d;
    }
    const uint32_t live = (uint32_t)__popc(alive & ring_mask());
    new_many(h, kCand, (uint32_t)__popc(claim), [&](uint32_t j, uint32_t o) {
      if (o == kNull) return;
      const uint32_t n = neighbour(off, side, x, y, nth_set_bit(claim, j));
      *field_ptr<uint32_t>(h, o, kCand, kACell) = n;
      *field_ptr<uint32_t>(h, o, kCand, kAWorld) = wid;
      *field_ptr<uint32_t>(h, o, kCand, kAAction) = 0;
    });
    *field_ptr<uint32_t>(h, self, type, kAAction) = (live == 2 || live == 3) ? 0u : 1u;
    return false;
  }
};

struct CandPrep {
  static constexpr uint32_t kKind = 31;
  using Args = World;
  template <class H>
  static __device__ __forceinline__ void run_pair(const H& h, uint32_t type, uint32_t s0, bool l0, uint32_t s1,
                                                  bool l1, const Args& w, bool& d0, bool& d1) {
    const uint32_t self[2] = {s0, s1};
    const bool lv[2] = {l0, l1};
    const uint32_t n = __ballot(l1) ? 2u : 1u;
    uint32_t g[2] = {0, 0}, wid[2] = {0, 0}, alive[2] = {0, 0};
    CellPos p[2];
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      g[u] = *field_ptr<uint32_t>(h, self[u], type, kACell);
      wid[u] = *field_ptr<uint32_t>(h, self[u], type, kAWorld);
    }
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) p[u] = cell_pos(w, g[u], wid[u], lv[u] && u < n);
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      alive[u] = neighbourhood<1>(w.bits, p[u].off, p[u].side, p[u].x, p[u].y);
    }
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u)
      if (lv[u]) *field_ptr<uint32_t>(h, self[u], type, kAAction) = __popc(alive[u]) == 3 ? 1u : 0u;
    d0 = d1 = false;
  }
  template <class H>
  static __device__ __forceinline__ bool run(const H& h, uint32_t type, uint32_t self, const Args& w) {
    const uint32_t g = *field_ptr<uint32_t>(h, self, type, kACell);
    const uint32_t wid = *field_ptr<uint32_t>(h, self, type, kAWorld);
    const uint32_t off = w.off[wid], side = w.side[wid];
    const uint32_t local = g - off;
    const uint32_t y = local / side, x = local - y * side;
    const uint32_t alive = neighbourhood<1>(w.bits, off, side, x, y);
    *field_ptr<uint32_t>(h, self, type, kAAction) = __popc(alive) == 3 ? 1u : 0u;
    return false;
  }
};

// Phases 3 and 4 (the Cells of dying and born cells; each object deletes
// itself only): loads of both slots first, then the Cells' handles of both.
struct AliveUpdate {
  static constexpr uint32_t kKind = 32;
  static constexpr uint32_t kMinWaves = 8;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = World;
  template <class H>
  static __device__ __forceinline__ void run_pair(const H& h, uint32_t type, uint32_t s0, bool l0, uint32_t s1,
                                                  bool l1, const Args& w, bool& d0, bool& d1) {
    const uint32_t self[2] = {s0, s1};
    const bool lv[2] = {l0, l1};
    const uint32_t n = __ballot(l1) ? 2u : 1u;
    bool dying[2] = {false, false};
    uint32_t g[2] = {0, 0}, wd[2];
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      dying[u] = lv[u] && *field_ptr<uint32_t>(h, self[u], type, kAAction) != 0;
      g[u] = *field_ptr<uint32_t>(h, self[u], type, kACell);
    }
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) wd[u] = u < n ? w.cells[dying[u] ? g[u] : 0u] : kNull;
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u)
      if (dying[u]) set_cell_live(h, w, g[u], wd[u], 0);
    d0 = dying[0];
    d1 = dying[1];
  }
  template <class H>
  static __device__ __forceinline__ bool run(const H& h, uint32_t type, uint32_t self, const Args& w) {
    if (*field_ptr<uint32_t>(h, self, type, kAAction) == 0) return false;
    const uint32_t g = *field_ptr<uint32_t>(h, self, type, kACell);
    set_cell_live(h, w, g, w.cells[g], 0);
    return true;
  }
};

struct CandUpdate {
  static constexpr uint32_t kKind = 33;
  static constexpr uint32_t kMinWaves = 8;
  static constexpr bool kDeletesOnlyThis = true;
  using Args = World;
  template <class H>
  static __device__ __forceinline__ void run_pair(const H& h, uint32_t type, uint32_t s0, bool l0, uint32_t s1,
                                                  bool l1, const Args& w, bool& d0, bool& d1) {
    const uint32_t self[2] = {s0, s1};
    const bool lv[2] = {l0, l1};
    const uint32_t n = __ballot(l1) ? 2u : 1u;
    bool born[2] = {false, false};
    uint32_t g[2] = {0, 0}, wid[2] = {0, 0}, wd[2];
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      if (u >= n) break;
      g[u] = *field_ptr<uint32_t>(h, self[u], type, kACell);
      wid[u] = *field_ptr<uint32_t>(h, self[u], type, kAWorld);
      born[u] = lv[u] && *field_ptr<uint32_t>(h, self[u], type, kAAction) != 0;
    }
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) wd[u] = u < n ? w.cells[born[u] ? g[u] : 0u] : kNull;
    uint32_t nb = 0;  // bit u: cell u is born and has its Cell
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u)
      if (born[u] && set_cell_live(h, w, g[u], wd[u], 1)) nb |= 1u << u;
    // One allocation for the Alive objects of both blocks' births.
    new_many(h, kAlive, (uint32_t)__popc(nb), [&](uint32_t j, uint32_t o) {
      if (o == kNull) return;
      const uint32_t u = nth_set_bit(nb, j);
      *field_ptr<uint32_t>(h, o, kAlive, kACell) = u ? g[1] : g[0];
      *field_ptr<uint32_t>(h, o, kAlive, kAWorld) = u ? wid[1] : wid[0];
      *field_ptr<uint32_t>(h, o, kAlive, kAAction) = 0;
    });
    d0 = l0;
    d1 = l1;
  }
  template <class H>
  static __device__ __forceinline__ bool run(const H& h, uint32_t type, uint32_t self, const Args& w) {
    const uint32_t g = *field_ptr<uint32_t>(h, self, type, kACell);
    const uint32_t wid = *field_ptr<uint32_t>(h, self, type, kAWorld);
    const bool born = *field_ptr<uint32_t>(h, self, type, kAAction) != 0;
    if (born && set_cell_live(h, w, g, w.cells[g], 1)) {
      const uint32_t o = dsoar_new(h, kAlive);
      if (o != kNull) {
        *field_ptr<uint32_t>(h, o, kAlive, kACell) = g;
        *field_ptr<uint32_t>(h, o, kAlive, kAWorld) = wid;
        *field_ptr<uint32_t>(h, o, kAlive, kAAction) = 0;
      }
    }
    return true;
  }
};

__device__ __forceinline__ uint32_t world_of(const uint32_t* off, uint32_t num_worlds, uint32_t g) {
  uint32_t lo = 0, hi = num_worlds;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Creates the Cells of cells first + i, i < n (grid byte i nonzero: live),
// and an Alive for every live one.  A wavefront takes 64 * PL consecutive
// cells, lane l the PL from l * PL on, so a lane's Cells are one block of
// consecutive positions when PL is 64 (the wavefront's request of 64 blocks
// is one atomic on the free bitmap), and its live cells' Alive objects are
// one request more.  Large creations use 64 cells per lane and open the
// Alive objects' own blocks (the heap copy they run with has the fresh
// policy for Alive): thousands of wavefronts asking for a few dozen Alive
// objects each at once would otherwise all look up the same few active
// blocks, which took 5.2 of the 5.5 ms that 48.8 M cells took.  Below 2^22
// cells one cell per lane is kept: on a 1024 x 1024 world the objects laid
// out 64 positions per block made every later generation's update 13 %
// slower, for an init 20 us shorter.
constexpr uint32_t kCellsWideMin = 1u << 22;  // from this many cells, 64 per lane

// Live bits of cells g0 .. g0 + cnt - 1 (bit j of v: cell g0 + j), cnt <= 64:
// words wholly inside the range are stored, the others updated with atomic
// AND / OR under the range's mask, so that bits of other lanes and worlds
// in a shared word stay intact.
__device__ __forceinline__ void write_live_range(uint32_t* bits, uint32_t g0, uint32_t cnt, uint64_t v) {
  uint32_t done = 0;
  while (done < cnt) {
    const uint32_t g = g0 + done, sh = g & 31u;
    const uint32_t take = 32u - sh < cnt - done ? 32u - sh : cnt - done;
    const uint32_t m = (take == 32u ? ~0u : ((1u << take) - 1u)) << sh;
    const uint32_t x = ((uint32_t)(v >> done) << sh) & m;
    uint32_t* word = bits + (g >> 5);
    if (m == ~0u) {
      *word = x;
    } else {
      __hip_atomic_fetch_and(word, ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (x) __hip_atomic_fetch_or(word, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    done += take;
  }
}

template <uint32_t PL, class H, class WorldOf>
__device__ __forceinline__ void create_cells(const H& h, const World& w, uint32_t first, uint32_t n,
                                             const uint8_t* grid, WorldOf world_of_cell) {
  static_assert(PL == 1 || PL == 64, "one or 64 cells per lane");
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t base = (wave * 64u + lane_id()) * PL;  // this lane's first cell, relative to `first`
  const uint32_t k = base < n ? (uint32_t)(n - base < PL ? n - base : PL) : 0u;
  uint64_t live = 0;
  if constexpr (PL == 64) {
    if (k == 64 && ((uintptr_t)(grid + base) & 15u) == 0) {
      const uint4* q = reinterpret_cast<const uint4*>(grid + base);
#pragma unroll
      for (uint32_t c = 0; c < 4; ++c) {
        const uint4 t = q[c];
        const uint32_t d[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
#pragma unroll
          for (uint32_t b = 0; b < 4; ++b)
            live |= (uint64_t)(((d[e] >> (8 * b)) & 0xFFu) != 0) << (16 * c + 4 * e + b);
      }
    } else {
      for (uint32_t j = 0; j < k; ++j) live |= (uint64_t)(grid[base + j] != 0) << j;
    }
  } else {
    live = k && grid[base] ? 1ull : 0ull;
  }
  uint64_t made = 0;  // bit j: cell j got its Cell
  new_many(h, kCell, k, [&](uint32_t j, uint32_t o) {
    if (o != kNull) {
      *field_ptr<uint32_t>(h, o, kCell, kCAlive) = (uint32_t)(live >> j) & 1u;
      made |= 1ull << j;
    }
    const_cast<uint32_t*>(w.cells)[first + (uint32_t)(base + j)] = o;
  });
  if constexpr (PL == 64) {
    if (k) write_live_range(const_cast<uint32_t*>(w.bits), first + (uint32_t)base, k, live & made);
  } else {
    write_live_run(const_cast<uint32_t*>(w.bits), first + (uint32_t)base, k != 0, (live & made) != 0, true);
  }
  new_many(h, kAlive, (uint32_t)__popcll(live), [&](uint32_t r, uint32_t o) {
    if (o == kNull) return;
    const uint32_t g = first + (uint32_t)(base + nth_set_bit(live, r));
    *field_ptr<uint32_t>(h, o, kAlive, kACell) = g;
    *field_ptr<uint32_t>(h, o, kAlive, kAWorld) = world_of_cell(g);
    *field_ptr<uint32_t>(h, o, kAlive, kAAction) = 0;
  });
}

uint32_t cells_per_lane(uint64_t n) { return n >= kCellsWideMin ? 64u : 1u; }

// The heap as the creation kernels see it: with 64 cells per lane, the Alive
// objects a wavefront creates open blocks of their own.
template <uint32_t LG>
DevHeapW<LG> creation_heap(const dsoar_heap* heap, uint32_t per_lane) {
  DevHeapW<LG> d(heap->dev);
  if (per_lane > 1) d.fresh_types |= 1u << kAlive;
  return d;
}

// Creates every Cell (in position order) and an Alive for every live cell.
template <uint32_t LG, uint32_t PL>
__global__ void gol_init_kernel(DevHeapW<LG> h, World w, uint32_t num_worlds, uint32_t total, const uint8_t* grid) {
  // A lane's cells lie in at most two worlds (a world has at least 64 * 64
  // cells when PL is 64): the world of the first is looked up once.
  const uint64_t c0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64u * PL + lane_id() * PL;
  const uint32_t w0 = c0 < total ? world_of(w.off, num_worlds, (uint32_t)c0) : 0u;
  create_cells<PL>(h, w, 0u, total, grid, [&](uint32_t g) {
    return g >= w.off[w0] && g < w.off[w0 + 1] ? w0 : world_of(w.off, num_worlds, g);
  });
}

__global__ void gol_read_kernel(DevHeap h, World w, uint32_t off, uint32_t n, uint8_t* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t wd = w.cells[off + i];
  out[i] = wd == kNull ? 0xFF : (uint8_t)*field_ptr<uint32_t>(h, wd, kCell, kCAlive);
}

// Records world slot's cell range in the world table.
__global__ void gol_set_slot_kernel(World w, uint32_t slot, uint32_t off, uint32_t side) {
  const_cast<uint32_t*>(w.off)[slot] = off;
  const_cast<uint32_t*>(w.side)[slot] = side;
}

// Creates the objects of one world admitted into slot `slot`.
template <uint32_t LG, uint32_t PL>
__global__ void gol_admit_kernel(DevHeapW<LG> h, World w, uint32_t slot, uint32_t off, uint32_t n,
                                 const uint8_t* grid) {
  create_cells<PL>(h, w, off, n, grid, [&](uint32_t) { return slot; });
}

// Deletes the Cells of one world (the Alive objects go with GolDeleteWorld).
template <uint32_t LG>
__global__ void gol_retire_cells_kernel(DevHeapW<LG> h, World w, uint32_t off, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t* c = const_cast<uint32_t*>(w.cells) + off + i;
  if (*c != kNull) dsoar_delete(h, *c);
  *c = kNull;
  write_live_run(const_cast<uint32_t*>(w.bits), off + i, true, false, true);
}

struct GolDeleteWorld {
  static constexpr uint32_t kKind = 34;
  struct Args { uint32_t slot; };
  template <class H>
  static __device__ bool run(const H& h, uint32_t type, uint32_t self, const Args& a) {
    return *field_ptr<uint32_t>(h, self, type, kAWorld) == a.slot;
  }
};

bool gol_heap_ok(const dsoar_heap* h) {
  if (h->desc.num_types < 3) return false;
  const uint32_t want[3] = {1, 3, 3};
  for (uint32_t t = 0; t < 3; ++t) {
    const dsoar_type_layout& L = h->desc.types[t];
    if (L.num_fields < want[t]) return false;
    for (uint32_t f = 0; f < want[t]; ++f)
      if (L.field_bytes[f] != 4) return false;
  }
  return true;
}

// Device buffer of a world set: the world table (offsets and sides), the
// cell index (4 bytes per cell) and the live-bit plane (padded by two words,
// so that a window's second dword load past the last cell stays inside).
uint64_t table_head(uint32_t num_worlds) { return ((uint64_t)(2 * num_worlds + 1) * 4 + 255) / 256 * 256; }
uint64_t index_bytes(uint64_t cells) { return (cells * 4 + 255) / 256 * 256; }
uint64_t bits_bytes(uint64_t cells) { return (((cells + 31) / 32 + 2) * 4 + 255) / 256 * 256; }
uint64_t world_set_bytes(uint32_t num_worlds, uint64_t cells) {
  return table_head(num_worlds) + index_bytes(cells) + bits_bytes(cells);
}

void carve(World& w, uint8_t* dev_mem, uint32_t num_worlds, uint64_t cells) {
  uint32_t* tab = (uint32_t*)dev_mem;
  w.off = tab;
  w.side = tab + num_worlds + 1;
  w.cells = (const uint32_t*)(dev_mem + table_head(num_worlds));
  w.bits = (const uint32_t*)(dev_mem + table_head(num_worlds) + index_bytes(cells));
}

uint64_t gol_total_cells(uint32_t num_worlds, const uint32_t* sides) {
  uint64_t t = 0;
  for (uint32_t i = 0; i < num_worlds; ++i) t += (uint64_t)sides[i] * sides[i];
  return t;
}

}  // namespace
}  // namespace dsoar

using namespace dsoar;

struct dsoar_gol {
  dsoar_heap* heap;
  World w;
  uint32_t num_worlds;   // world slots
  uint32_t total;        // cells of the cell index (the arena)
  uint32_t* h_off;       // host copy of each slot's cell range (pool mode)
  uint32_t* h_side;
  uint8_t* live;         // slot holds a world (pool mode)
  StepGraphs graphs;
};

namespace {

int gol_generation(dsoar_gol* g, uint32_t flags, hipStream_t s) {
  dsoar_heap* h = g->heap;
  const uint32_t base = flags & DSOAR_DO_PLAIN;
  int rc = launch_doall<AlivePrep>(h, kAlive, g->w, base, s);
  if (!rc) rc = launch_doall<CandPrep>(h, kCand, g->w, base, s);
  // Phase 2 creates and deletes nothing, phase 3 touches only Alive objects:
  // phases 3 and 4 reuse the enumerations of phases 1 and 2.
  if (base & DSOAR_DO_PLAIN) {
    if (!rc) rc = launch_doall<AliveUpdate>(h, kAlive, g->w, base | DSOAR_DO_REUSE_ENUM, s);
    if (!rc) rc = launch_doall<CandUpdate>(h, kCand, g->w, base | DSOAR_DO_REUSE_ENUM, s);
  } else if (!rc) {
    // Phases 3 and 4 touch disjoint cells (dying ones, born ones) and each
    // object only its own: one launch over both lists.
    rc = launch_doall2<AliveUpdate, CandUpdate>(h, kAlive, g->w, kCand, g->w, kKindGolUpdate, s);
  }
  return rc;
}

}  // namespace

extern "C" {

size_t dsoar_gol_bytes(uint32_t num_worlds, const uint32_t* sides) {
  if (num_worlds == 0 || !sides) return 0;
  for (uint32_t i = 0; i < num_worlds; ++i)
    if (sides[i] < 1 || sides[i] > 65535) return 0;
  const uint64_t total = gol_total_cells(num_worlds, sides);
  if (total >= (1ull << 32)) return 0;
  return (size_t)world_set_bytes(num_worlds, total);
}

int dsoar_gol_create(dsoar_heap* heap, uint32_t num_worlds, const uint32_t* sides, void* dev_mem, size_t dev_bytes,
                     void* stream, dsoar_gol** out) {
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !gol_heap_ok(heap) || !dev_mem || ((uintptr_t)dev_mem & 255u)) return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_gol_bytes(num_worlds, sides);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_gol* g = new (std::nothrow) dsoar_gol;
  if (!g) return DSOAR_ERR_INVALID_ARG;
  memset(g, 0, sizeof(*g));
  g->heap = heap;
  g->num_worlds = num_worlds;
  g->total = (uint32_t)gol_total_cells(num_worlds, sides);
  carve(g->w, (uint8_t*)dev_mem, num_worlds, g->total);
  uint32_t* tab = (uint32_t*)dev_mem;
  uint32_t* host = (uint32_t*)malloc((size_t)(2 * num_worlds + 1) * 4);
  if (!host) {
    delete g;
    return DSOAR_ERR_INVALID_ARG;
  }
  uint32_t acc = 0;
  for (uint32_t i = 0; i < num_worlds; ++i) {
    host[i] = acc;
    host[num_worlds + 1 + i] = sides[i];
    acc += sides[i] * sides[i];
  }
  host[num_worlds] = acc;
  hipError_t e = hipMemcpyAsync(tab, host, (size_t)(2 * num_worlds + 1) * 4, hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  free(host);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(heap, e);
  }
  *out = g;
  return DSOAR_OK;
}

int dsoar_gol_destroy(dsoar_gol* g) {
  if (!g) return DSOAR_ERR_INVALID_ARG;
  free(g->h_off);
  free(g->h_side);
  free(g->live);
  step_graphs_clear(g->graphs);
  delete g;
  return DSOAR_OK;
}

int dsoar_gol_init(dsoar_gol* g, const uint8_t* grid_dev, void* stream) {
  if (!g || !grid_dev) return DSOAR_ERR_INVALID_ARG;
  with_width(g->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    const uint32_t per_lane = cells_per_lane(g->total);
    const uint64_t per_wg = 256ull * per_lane;
    const dim3 grid((uint32_t)((g->total + per_wg - 1) / per_wg));
    if (per_lane == 64)
      launch_timed(g->heap, kKindGolInit, gol_init_kernel<kLG, 64>, grid, dim3(256), (hipStream_t)stream,
                   creation_heap<kLG>(g->heap, per_lane), g->w, g->num_worlds, g->total, grid_dev);
    else
      launch_timed(g->heap, kKindGolInit, gol_init_kernel<kLG, 1>, grid, dim3(256), (hipStream_t)stream,
                   creation_heap<kLG>(g->heap, per_lane), g->w, g->num_worlds, g->total, grid_dev);
  });
  DSOAR_LAUNCHED(g->heap);
  return DSOAR_OK;
}

int dsoar_gol_step(dsoar_gol* g, uint32_t generations, uint32_t flags, void* stream) {
  if (!g) return DSOAR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  dsoar_heap* h = g->heap;
  if (flags & DSOAR_GOL_GRAPH) {
    if (flags & DSOAR_DO_PLAIN) return DSOAR_ERR_INVALID_ARG;  // plain mode synchronises
    return step_graphs_run(h, g->graphs, generations, s, [&](hipStream_t gs) { return gol_generation(g, 0, gs); });
  }
  for (uint32_t i = 0; i < generations; ++i) {
    const int rc = gol_generation(g, flags, s);
    if (rc) return rc;
  }
  return DSOAR_OK;
}

int dsoar_gol_read(dsoar_gol* g, uint8_t* grid_dev, void* stream) {
  if (!g || !grid_dev) return DSOAR_ERR_INVALID_ARG;
  hipLaunchKernelGGL(gol_read_kernel, dim3((uint32_t)(((uint64_t)g->total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, g->heap->dev,
                     g->w, 0u, g->total, grid_dev);
  DSOAR_LAUNCHED(g->heap);
  return DSOAR_OK;
}

uint32_t dsoar_gol_total_cells(const dsoar_gol* g) { return g ? g->total : 0; }

// ------------------------------------------------------------- world pool

size_t dsoar_golpool_bytes(uint32_t max_worlds, uint32_t arena_cells) {
  if (max_worlds == 0 || max_worlds > (1u << 20) || arena_cells == 0) return 0;
  return (size_t)world_set_bytes(max_worlds, arena_cells);
}

int dsoar_golpool_create(dsoar_heap* heap, uint32_t max_worlds, uint32_t arena_cells, void* dev_mem,
                         size_t dev_bytes, void* stream, dsoar_gol** out) {
  (void)stream;
  if (!out) return DSOAR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!heap_ok(heap) || !gol_heap_ok(heap) || !dev_mem || ((uintptr_t)dev_mem & 255u)) return DSOAR_ERR_INVALID_ARG;
  const size_t need = dsoar_golpool_bytes(max_worlds, arena_cells);
  if (need == 0) return DSOAR_ERR_INVALID_ARG;
  if (dev_bytes < need) return DSOAR_ERR_TOO_SMALL;
  dsoar_gol* g = new (std::nothrow) dsoar_gol;
  if (!g) return DSOAR_ERR_INVALID_ARG;
  memset(g, 0, sizeof(*g));
  g->heap = heap;
  g->num_worlds = max_worlds;
  g->total = arena_cells;
  g->h_off = (uint32_t*)calloc(max_worlds, 4);
  g->h_side = (uint32_t*)calloc(max_worlds, 4);
  g->live = (uint8_t*)calloc(max_worlds, 1);
  if (!g->h_off || !g->h_side || !g->live) {
    dsoar_gol_destroy(g);
    return DSOAR_ERR_INVALID_ARG;
  }
  carve(g->w, (uint8_t*)dev_mem, max_worlds, arena_cells);
  *out = g;
  return DSOAR_OK;
}

int dsoar_gol_admit(dsoar_gol* g, uint32_t slot, uint32_t cell_offset, uint32_t side, const uint8_t* grid_dev,
                    void* stream) {
  if (!g || !g->live || slot >= g->num_worlds || g->live[slot] || side == 0 || side > 65535 || !grid_dev)
    return DSOAR_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)side * side;
  if ((uint64_t)cell_offset + n > g->total) return DSOAR_ERR_INVALID_ARG;
  for (uint32_t k = 0; k < g->num_worlds; ++k)  // cell ranges of resident worlds must not overlap
    if (g->live[k] && cell_offset < g->h_off[k] + g->h_side[k] * g->h_side[k] && g->h_off[k] < cell_offset + n)
      return DSOAR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(gol_set_slot_kernel, dim3(1), dim3(1), 0, s, g->w, slot, cell_offset, side);
  DSOAR_LAUNCHED(g->heap);
  with_width(g->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    const uint32_t per_lane = cells_per_lane(n);
    const uint64_t per_wg = 256ull * per_lane;
    const dim3 grid((uint32_t)((n + per_wg - 1) / per_wg));
    if (per_lane == 64)
      launch_timed(g->heap, kKindGolAdmit, gol_admit_kernel<kLG, 64>, grid, dim3(256), s,
                   creation_heap<kLG>(g->heap, per_lane), g->w, slot, cell_offset, (uint32_t)n, grid_dev);
    else
      launch_timed(g->heap, kKindGolAdmit, gol_admit_kernel<kLG, 1>, grid, dim3(256), s,
                   creation_heap<kLG>(g->heap, per_lane), g->w, slot, cell_offset, (uint32_t)n, grid_dev);
  });
  DSOAR_LAUNCHED(g->heap);
  g->h_off[slot] = cell_offset;
  g->h_side[slot] = side;
  g->live[slot] = 1;
  return DSOAR_OK;
}

int dsoar_gol_retire(dsoar_gol* g, uint32_t slot, void* stream) {
  if (!g || !g->live || slot >= g->num_worlds || !g->live[slot]) return DSOAR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  int rc = launch_doall<GolDeleteWorld>(g->heap, kAlive, GolDeleteWorld::Args{slot}, 0, s);
  if (rc) return rc;
  const uint32_t n = g->h_side[slot] * g->h_side[slot];
  with_width(g->heap, [&](auto w_) {
    constexpr uint32_t kLG = decltype(w_)::value;
    hipLaunchKernelGGL(gol_retire_cells_kernel<kLG>, dim3((uint32_t)(((uint64_t)n + 255) / 256)), dim3(256), 0, s, DevHeapW<kLG>(g->heap->dev), g->w,
                     g->h_off[slot], n);
  });
  DSOAR_LAUNCHED(g->heap);
  g->live[slot] = 0;
  return DSOAR_OK;
}

int dsoar_gol_read_world(dsoar_gol* g, uint32_t slot, uint8_t* grid_dev, void* stream) {
  if (!g || !g->live || slot >= g->num_worlds || !g->live[slot] || !grid_dev) return DSOAR_ERR_INVALID_ARG;
  const uint32_t n = g->h_side[slot] * g->h_side[slot];
  hipLaunchKernelGGL(gol_read_kernel, dim3((uint32_t)(((uint64_t)n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, g->heap->dev, g->w,
                     g->h_off[slot], n, grid_dev);
  DSOAR_LAUNCHED(g->heap);
  return DSOAR_OK;
}

}  // extern "C"
