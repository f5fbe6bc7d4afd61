/*
 * CPU oracle for the SMMO object heap and parallel do-all
 * (DynaSOAr, arXiv 1809.07444).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Sequential, plain C,
 * built with -O2 -ffp-contract=off and no fast-math.  Shares no source with
 * the device code.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ====================================================================== RNG
 * SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014), written out from its
 * published definition, and the workload hash built on it:
 *   hash(seed, stream, a, b) = mix(mix(mix(seed ^ stream*golden) ^ a) ^ b). */
uint64_t orc_mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

uint64_t orc_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  uint64_t h = orc_mix64(seed ^ (stream * 0x9E3779B97F4A7C15ull));
  h = orc_mix64(h ^ a);
  return orc_mix64(h ^ b);
}

/* U{lo..hi} from the top 32 bits of h: lo + floor(top32 * span / 2^32). */
int32_t orc_uniform_int(uint64_t h, int32_t lo, int32_t hi) {
  uint64_t span = (uint64_t)(hi - lo + 1);
  return lo + (int32_t)(((h >> 32) * span) >> 32);
}

/* ======================================================= hierarchical bitmap
 * Sec. 3 ("Data Structure"): a bitmap of N bits is ceil(N/w) containers of w
 * bits, plus a nested bitmap of ceil(N/w) bits when N > w.  Bit i of the
 * nested bitmap is the OR of container i (container consistency). */

static int popc64(uint64_t x) { return __builtin_popcountll(x); }

int orc_bm_init(orc_bitmap *b, int64_t nbits, int width, int all_set) {
  memset(b, 0, sizeof(*b));
  if (nbits < 1 || width < 2 || width > 64) return -1;
  b->width = width;
  int64_t n = nbits;
  int l = 0;
  for (;;) {
    if (l >= ORC_MAX_LEVELS) return -1;
    b->nbits[l] = n;
    b->nwords[l] = (n + width - 1) / width;
    b->words[l] = (uint64_t *)calloc((size_t)b->nwords[l], sizeof(uint64_t));
    if (!b->words[l]) return -1;
    l++;
    if (n <= width) break; /* no nested bitmap */
    n = (n + width - 1) / width;
  }
  b->nlevels = l;
  if (all_set) {
    /* Set every bit at level 0, then every level is the OR of the one below. */
    for (int64_t pos = 0; pos < b->nbits[0]; pos++) b->words[0][pos / width] |= 1ull << (pos % width);
    for (int lv = 1; lv < b->nlevels; lv++)
      for (int64_t i = 0; i < b->nbits[lv]; i++)
        if (b->words[lv - 1][i]) b->words[lv][i / width] |= 1ull << (i % width);
  }
  return 0;
}

void orc_bm_free(orc_bitmap *b) {
  for (int l = 0; l < b->nlevels; l++) free(b->words[l]);
  free(b->trace);
  memset(b, 0, sizeof(*b));
}

int orc_bm_get(const orc_bitmap *b, int level, int64_t pos) {
  return (int)((b->words[level][pos / b->width] >> (pos % b->width)) & 1u);
}

static void trace_push(orc_bitmap *b, int level, int64_t pos) {
  if (b->ntrace == b->trace_cap) {
    int64_t cap = b->trace_cap ? 2 * b->trace_cap : 64;
    int64_t *t = (int64_t *)realloc(b->trace, (size_t)cap * sizeof(int64_t));
    if (!t) return;
    b->trace = t;
    b->trace_cap = cap;
  }
  b->trace[b->ntrace++] = ((int64_t)level << 40) + pos;
}

/* Alg. 2: clear the bit with an atomic AND (sequential here); it succeeded if
 * the bit was set.  If it succeeded and the container had exactly one bit
 * set before, the container is now empty and this call owns clearing the
 * container's bit in the nested bitmap (with the retrying clear()). */
int orc_bm_try_clear(orc_bitmap *b, int level, int64_t pos) {
  int64_t cid = pos / b->width;
  uint64_t mask = 1ull << (pos % b->width);
  uint64_t prev = b->words[level][cid];
  b->words[level][cid] = prev & ~mask;
  int success = (prev & mask) != 0;
  if (success) trace_push(b, level, pos);
  if (success && level + 1 < b->nlevels && popc64(prev) == 1) orc_bm_clear(b, level + 1, cid);
  return success;
}

/* Sec. 2.1, "similarly": set with an atomic OR; success if the bit was clear.
 * The container's nested bit is set by the call that made the container
 * non-empty (prev == 0). */
int orc_bm_try_set(orc_bitmap *b, int level, int64_t pos) {
  int64_t cid = pos / b->width;
  uint64_t mask = 1ull << (pos % b->width);
  uint64_t prev = b->words[level][cid];
  b->words[level][cid] = prev | mask;
  int success = (prev & mask) == 0;
  if (success && level + 1 < b->nlevels && prev == 0) orc_bm_set(b, level + 1, cid);
  return success;
}

/* clear(pos) = retry try_clear until it succeeds.  Sequentially, a retry can
 * never succeed once the first attempt failed (nobody else sets the bit), so
 * the model reports the would-be livelock as an error instead of spinning. */
int orc_bm_clear(orc_bitmap *b, int level, int64_t pos) {
  return orc_bm_try_clear(b, level, pos) ? 0 : -1;
}

int orc_bm_set(orc_bitmap *b, int level, int64_t pos) {
  return orc_bm_try_set(b, level, pos) ? 0 : -1;
}

/* try_find_set(): descend from the top container, picking the lowest set bit
 * at every level.  An empty container on the way down means the bitmap is
 * inconsistent; the operation then reports FAIL. */
int64_t orc_bm_try_find_set(const orc_bitmap *b) {
  int64_t idx = 0;
  for (int l = b->nlevels - 1; l >= 0; l--) {
    uint64_t w = b->words[l][idx];
    if (w == 0) return ORC_FAIL;
    idx = idx * b->width + __builtin_ctzll(w);
  }
  return idx < b->nbits[0] ? idx : ORC_FAIL;
}

/* clear(): find a set bit and clear it, repeating until the clear succeeds
 * (the intent of Sec. 2.1; see the readings list).  FAIL if the bitmap is
 * empty. */
int64_t orc_bm_find_clear(orc_bitmap *b) {
  for (;;) {
    int64_t i = orc_bm_try_find_set(b);
    if (i == ORC_FAIL) return ORC_FAIL;
    if (orc_bm_try_clear(b, 0, i)) return i;
  }
}

/* Number of bits violating container consistency, plus any set bit beyond a
 * level's size. */
int64_t orc_bm_consistency_violations(const orc_bitmap *b) {
  int64_t bad = 0;
  for (int l = 0; l < b->nlevels; l++) {
    for (int64_t p = b->nbits[l]; p < b->nwords[l] * b->width; p++)
      if (orc_bm_get(b, l, p)) bad++;
    if (l + 1 < b->nlevels)
      for (int64_t i = 0; i < b->nwords[l]; i++)
        if ((b->words[l][i] != 0) != (orc_bm_get(b, l + 1, i) != 0)) bad++;
  }
  return bad;
}

void *orc_bm_new(int64_t nbits, int width, int all_set) {
  orc_bitmap *b = (orc_bitmap *)calloc(1, sizeof(orc_bitmap));
  if (!b) return NULL;
  if (orc_bm_init(b, nbits, width, all_set) != 0) {
    orc_bm_free(b);
    free(b);
    return NULL;
  }
  return b;
}

void orc_bm_delete(void *b) {
  if (!b) return;
  orc_bm_free((orc_bitmap *)b);
  free(b);
}

int orc_bm_nlevels(void *b) { return ((orc_bitmap *)b)->nlevels; }
int64_t orc_bm_nwords(void *b, int level) { return ((orc_bitmap *)b)->nwords[level]; }

void orc_bm_words(void *b, int level, uint64_t *out) {
  orc_bitmap *bm = (orc_bitmap *)b;
  memcpy(out, bm->words[level], (size_t)bm->nwords[level] * sizeof(uint64_t));
}

int64_t orc_bm_trace(void *b, int64_t *out, int64_t cap) {
  orc_bitmap *bm = (orc_bitmap *)b;
  int64_t n = bm->ntrace < cap ? bm->ntrace : cap;
  if (out && n) memcpy(out, bm->trace, (size_t)n * sizeof(int64_t));
  return bm->ntrace;
}

/* op: 0 try_set, 1 try_clear, 2 set, 3 clear, 4 try_find_set, 5 find_clear,
 * 6 get.  All act on level 0 (the user-visible bitmap). */
int orc_bm_op(void *b, int op, int64_t pos, int64_t *result) {
  orc_bitmap *bm = (orc_bitmap *)b;
  if (op <= 3 || op == 6) {
    if (pos < 0 || pos >= bm->nbits[0]) return -1;
  }
  switch (op) {
    case 0: *result = orc_bm_try_set(bm, 0, pos); return 0;
    case 1: *result = orc_bm_try_clear(bm, 0, pos); return 0;
    case 2: *result = orc_bm_set(bm, 0, pos); return 0;
    case 3: *result = orc_bm_clear(bm, 0, pos); return 0;
    case 4: *result = orc_bm_try_find_set(bm); return 0;
    case 5: *result = orc_bm_find_clear(bm); return 0;
    case 6: *result = orc_bm_get(bm, 0, pos); return 0;
    default: return -1;
  }
}

/* ======================================================== block capacities
 * Sec. 2 ("Blocks of the smallest type always have a capacity of 64 ... other
 * types may have a smaller capacity"): the block holds 64 objects of the
 * smallest type; a type gets the largest power-of-two number of its objects
 * whose bytes do not exceed that (powers of two keep a block's slots one
 * aligned group of a 64-bit object bitmap), and never fewer than one. */
int32_t orc_type_capacity(const int32_t *sizes, int32_t ntypes, int32_t t) {
  int64_t smallest = sizes[0];
  for (int32_t i = 1; i < ntypes; i++)
    if (sizes[i] < smallest) smallest = sizes[i];
  const int64_t block_bytes = 64 * smallest;
  int32_t best = 1;
  for (int32_t c = 1; c <= 64; c *= 2)
    if ((int64_t)c * sizes[t] <= block_bytes) best = c;
  return best;
}

/* Sec. 1.2: a do-all over type t visits the objects of t and of every type
 * that inherits from t.  Type u inherits from t when the chain of parent
 * links starting at u reaches t; the chain is followed one link at a time,
 * and a chain longer than the number of types has a cycle. */
uint32_t orc_visit_types(const int32_t *parent, int32_t ntypes, int32_t t) {
  if (ntypes < 1 || ntypes > 32 || t < 0 || t >= ntypes) return 0;
  /* A forest: every chain ends (at -1) within ntypes links. */
  for (int32_t u = 0; u < ntypes; u++) {
    int32_t a = u, steps = 0;
    while (a != -1) {
      if (a < 0 || a >= ntypes || ++steps > ntypes) return 0;
      a = parent[a];
    }
  }
  uint32_t mask = 0;
  for (int32_t u = 0; u < ntypes; u++) {
    int32_t a = u;
    while (a != -1 && a != t) a = parent[a];
    if (a == t) mask |= 1u << u;
  }
  return mask;
}

/* ================================================================ heap model
 * Sec. 2: M blocks of `capacity` object slots, each holding objects of one
 * type; a 64-bit object allocation bitmap per block; block states free,
 * allocated[T], active[T], each indexed by a hierarchical bitmap.
 * Sec. 2.2, Alg. 1: allocate in an active block of T when one exists,
 * otherwise take a free block, initialise it and mark it allocated and active;
 * reserve a slot, and clear active[T] when the reservation took the last slot.
 * Deterministic choices: lowest active block, lowest free slot, lowest free
 * block.  Deletion: clear the slot bit; a block that was full becomes active
 * again.  Empty blocks return to free only in orc_heap_reclaim (quiescence). */

#define ORC_TYPE_NONE (-1)

typedef struct {
  int32_t M, c, ntypes;
  uint64_t cap_mask;
  uint64_t *objbm;
  int32_t *btype;
  orc_bitmap freebm, alloc[ORC_MAX_TYPES], active[ORC_MAX_TYPES];
  int64_t allocs[ORC_MAX_TYPES], frees[ORC_MAX_TYPES];
  int64_t errors;
} orc_heap;

void *orc_heap_new(int32_t num_blocks, int32_t capacity, int32_t num_types) {
  if (num_blocks < 1 || capacity < 1 || capacity > 64 || num_types < 1 || num_types > ORC_MAX_TYPES)
    return NULL;
  orc_heap *h = (orc_heap *)calloc(1, sizeof(orc_heap));
  if (!h) return NULL;
  h->M = num_blocks;
  h->c = capacity;
  h->ntypes = num_types;
  h->cap_mask = capacity == 64 ? ~0ull : ((1ull << capacity) - 1);
  h->objbm = (uint64_t *)calloc((size_t)num_blocks, sizeof(uint64_t));
  h->btype = (int32_t *)malloc((size_t)num_blocks * sizeof(int32_t));
  for (int32_t i = 0; i < num_blocks; i++) h->btype[i] = ORC_TYPE_NONE;
  orc_bm_init(&h->freebm, num_blocks, 64, 1);
  for (int t = 0; t < num_types; t++) {
    orc_bm_init(&h->alloc[t], num_blocks, 64, 0);
    orc_bm_init(&h->active[t], num_blocks, 64, 0);
  }
  return h;
}

void orc_heap_delete(void *hv) {
  orc_heap *h = (orc_heap *)hv;
  if (!h) return;
  free(h->objbm);
  free(h->btype);
  orc_bm_free(&h->freebm);
  for (int t = 0; t < h->ntypes; t++) {
    orc_bm_free(&h->alloc[t]);
    orc_bm_free(&h->active[t]);
  }
  free(h);
}

int64_t orc_heap_alloc(void *hv, int32_t type) {
  orc_heap *h = (orc_heap *)hv;
  if (type < 0 || type >= h->ntypes) return -2;
  for (;;) {
    int64_t bid = orc_bm_try_find_set(&h->active[type]);
    if (bid == ORC_FAIL) { /* slow path */
      bid = orc_bm_find_clear(&h->freebm);
      if (bid == ORC_FAIL) return -1; /* out of memory */
      h->btype[bid] = type;
      h->objbm[bid] = 0;
      orc_bm_set(&h->alloc[type], 0, bid);
      orc_bm_set(&h->active[type], 0, bid);
    }
    uint64_t freebits = ~h->objbm[bid] & h->cap_mask;
    if (freebits == 0) { /* cannot happen sequentially: full blocks are never active */
      h->errors++;
      return -3;
    }
    int slot = __builtin_ctzll(freebits);
    h->objbm[bid] |= 1ull << slot;
    if ((h->objbm[bid] & h->cap_mask) == h->cap_mask) orc_bm_clear(&h->active[type], 0, bid);
    h->allocs[type]++;
    return bid * 64 + slot;
  }
}

int orc_heap_free(void *hv, int64_t handle) {
  orc_heap *h = (orc_heap *)hv;
  int64_t bid = handle / 64;
  int slot = (int)(handle % 64);
  if (handle < 0 || bid >= h->M || slot >= h->c) return -1;
  int32_t t = h->btype[bid];
  if (t == ORC_TYPE_NONE || !((h->objbm[bid] >> slot) & 1)) return -1;
  int was_full = (h->objbm[bid] & h->cap_mask) == h->cap_mask;
  h->objbm[bid] &= ~(1ull << slot);
  if (was_full) orc_bm_set(&h->active[t], 0, bid);
  h->frees[t]++;
  return 0;
}

/* Return every empty typed block to the free state. */
int64_t orc_heap_reclaim(void *hv) {
  orc_heap *h = (orc_heap *)hv;
  int64_t n = 0;
  for (int32_t b = 0; b < h->M; b++) {
    int32_t t = h->btype[b];
    if (t == ORC_TYPE_NONE || h->objbm[b] != 0) continue;
    orc_bm_clear(&h->alloc[t], 0, b);
    if (orc_bm_get(&h->active[t], 0, b)) orc_bm_clear(&h->active[t], 0, b);
    h->btype[b] = ORC_TYPE_NONE;
    orc_bm_set(&h->freebm, 0, b);
    n++;
  }
  return n;
}

/* Block-state invariants at quiescence after reclaim.  Returns a bit set:
 * bit 1 I2 allocated[T] <=> type T and non-empty; bit 2 I3 active[T] <=>
 * allocated[T] and not full; bit 3 I4 active => allocated; bit 4 I5 free <=>
 * untyped and empty, and states of different types disjoint; bit 5 I6
 * container consistency of every bitmap; bit 6 I7 live == allocs - frees. */
int64_t orc_heap_check(void *hv) {
  orc_heap *h = (orc_heap *)hv;
  int64_t bad = 0;
  int64_t live[ORC_MAX_TYPES] = {0};
  for (int32_t b = 0; b < h->M; b++) {
    int32_t t = h->btype[b];
    uint64_t ob = h->objbm[b] & h->cap_mask;
    if (h->objbm[b] & ~h->cap_mask) bad |= 1 << 1;
    int isfree = orc_bm_get(&h->freebm, 0, b);
    if (isfree != (t == ORC_TYPE_NONE && ob == 0)) bad |= 1 << 4;
    for (int u = 0; u < h->ntypes; u++) {
      int al = orc_bm_get(&h->alloc[u], 0, b);
      int ac = orc_bm_get(&h->active[u], 0, b);
      if (al != (t == u && ob != 0)) bad |= 1 << 1;
      if (ac != (al && ob != h->cap_mask)) bad |= 1 << 2;
      if (ac && !al) bad |= 1 << 3;
      if ((al || ac) && isfree) bad |= 1 << 4;
    }
    if (t != ORC_TYPE_NONE) live[t] += popc64(ob);
  }
  if (orc_bm_consistency_violations(&h->freebm)) bad |= 1 << 5;
  for (int u = 0; u < h->ntypes; u++) {
    if (orc_bm_consistency_violations(&h->alloc[u])) bad |= 1 << 5;
    if (orc_bm_consistency_violations(&h->active[u])) bad |= 1 << 5;
    if (live[u] != h->allocs[u] - h->frees[u]) bad |= 1 << 6;
  }
  return bad;
}

/* out: [free_blocks, then per type (allocated_blocks, active_blocks, live,
 * allocs, frees)] for ORC_MAX_TYPES types. */
void orc_heap_counts(void *hv, int64_t *out) {
  orc_heap *h = (orc_heap *)hv;
  memset(out, 0, sizeof(int64_t) * (1 + 5 * ORC_MAX_TYPES));
  for (int32_t b = 0; b < h->M; b++) {
    out[0] += orc_bm_get(&h->freebm, 0, b);
    for (int u = 0; u < h->ntypes; u++) {
      out[1 + 5 * u] += orc_bm_get(&h->alloc[u], 0, b);
      out[2 + 5 * u] += orc_bm_get(&h->active[u], 0, b);
    }
    if (h->btype[b] != ORC_TYPE_NONE) out[3 + 5 * h->btype[b]] += popc64(h->objbm[b]);
  }
  for (int u = 0; u < h->ntypes; u++) {
    out[4 + 5 * u] = h->allocs[u];
    out[5 + 5 * u] = h->frees[u];
  }
}

void orc_heap_dump(void *hv, uint64_t *obj_bitmap, int32_t *block_type) {
  orc_heap *h = (orc_heap *)hv;
  memcpy(obj_bitmap, h->objbm, (size_t)h->M * sizeof(uint64_t));
  memcpy(block_type, h->btype, (size_t)h->M * sizeof(int32_t));
}

/* ===================================================== alloc/do-all micro
 * Objects {id, x, v}.  Start with ids 0..n_init-1.  Each step: every live
 * object does x = fma(0.01f, v, x) (one rounding); then every object with
 * id % 3 == 0 is deleted; then ids 3k (k < n_renew) are created again with
 * the step's inputs.  The state is a map id -> (x, v); here a dense array. */
int orc_micro_run(int32_t n_init, int32_t steps, int32_t n_renew,
                  const float *x0, const float *v0,
                  const float *xs, const float *vs,
                  float *out_x, float *out_v, uint8_t *out_present,
                  int64_t *counts) {
  if (n_init < 0 || steps < 0 || n_renew < 0 || 3ll * (n_renew - 1) >= n_init) return -1;
  int64_t allocs = 0, frees = 0;
  for (int32_t id = 0; id < n_init; id++) {
    out_x[id] = x0[id];
    out_v[id] = v0[id];
    out_present[id] = 1;
    allocs++;
  }
  const float k = 0.01f;
  for (int32_t s = 0; s < steps; s++) {
    for (int32_t id = 0; id < n_init; id++)
      if (out_present[id]) out_x[id] = fmaf(k, out_v[id], out_x[id]);
    for (int32_t id = 0; id < n_init; id++)
      if (out_present[id] && id % 3 == 0) {
        out_present[id] = 0;
        frees++;
      }
    for (int32_t j = 0; j < n_renew; j++) {
      int32_t id = 3 * j;
      out_present[id] = 1;
      out_x[id] = xs[(int64_t)s * n_renew + j];
      out_v[id] = vs[(int64_t)s * n_renew + j];
      allocs++;
    }
  }
  counts[0] = allocs;
  counts[1] = frees;
  return 0;
}

/* ============================================================ Game of Life
 * B3/S23 on a width x height torus, one synchronous generation.
 * counts (optional, 4 entries): dead cells with at least one live neighbour
 * (the candidates an object implementation creates), births, deaths, and the
 * live population after the step. */
int orc_gol_step(int32_t width, int32_t height, const uint8_t *in, uint8_t *out,
                 int64_t *counts) {
  int64_t cand = 0, births = 0, deaths = 0, pop = 0;
  for (int32_t y = 0; y < height; y++) {
    for (int32_t x = 0; x < width; x++) {
      int n = 0;
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          if (dx == 0 && dy == 0) continue;
          int32_t xx = (x + dx + width) % width;
          int32_t yy = (y + dy + height) % height;
          n += in[(int64_t)yy * width + xx] ? 1 : 0;
        }
      uint8_t alive = in[(int64_t)y * width + x] ? 1 : 0;
      uint8_t next;
      if (alive) {
        next = (n == 2 || n == 3) ? 1 : 0;
        if (!next) deaths++;
      } else {
        next = (n == 3) ? 1 : 0;
        if (n > 0) cand++;
        if (next) births++;
      }
      out[(int64_t)y * width + x] = next;
      pop += next;
    }
  }
  if (counts) {
    counts[0] = cand;
    counts[1] = births;
    counts[2] = deaths;
    counts[3] = pop;
  }
  return 0;
}

/* Runs `generations` steps in place; per_generation_counts (optional) gets 4
 * entries per generation, as orc_gol_step. */
int orc_gol_run(int32_t width, int32_t height, int32_t generations,
                uint8_t *grid, int64_t *per_generation_counts) {
  if (width < 1 || height < 1 || generations < 0) return -1;
  size_t n = (size_t)width * (size_t)height;
  uint8_t *tmp = (uint8_t *)malloc(n);
  if (!tmp) return -1;
  for (int32_t g = 0; g < generations; g++) {
    orc_gol_step(width, height, grid, tmp, per_generation_counts ? per_generation_counts + 4 * (int64_t)g : NULL);
    memcpy(grid, tmp, n);
  }
  free(tmp);
  return 0;
}

/* ============================================================== Sugarscape
 * Synchronous, deterministic Sugarscape-style model on a side x side torus
 * (the paper names the application but not its rules; these are the rules
 * adopted here, stated in full).  One step t:
 *  1 regrow: sugar[c] = min(sugar[c] + 1, cap[c]) everywhere.
 *  2 choose: each agent at p looks at its own cell and at the cells 1..vision
 *    steps away in the four axis directions; among its own cell and the cells
 *    unoccupied at the start of the phase it picks the most sugar, then the
 *    smallest distance, then the lowest cell index.  Target != p is a move
 *    request; the lowest requesting cell index wins each target.
 *  3 move: winners move; losers stay.
 *  4 eat: sugar += cell sugar; cell sugar = 0; sugar -= metabolism; age += 1;
 *    the agent dies if sugar <= 0 or age >= max_age.
 *  5 reproduce: an agent with sugar >= repro_min and fertile_min <= age <=
 *    fertile_max requests the lowest-index empty von Neumann neighbour; the
 *    lowest requesting cell index wins it.
 *  6 birth: the winner's child gets floor(sugar / 2) (the parent keeps the
 *    rest), metabolism U{1..4} from hash(seed, 10, t, n), vision U{1..6} from
 *    hash(seed, 11, t, n), age 0, at cell n.
 * Agents are stored by cell (at most one per cell).
 * Pins: hand-worked one- and two-agent cases, the tie-breaks, the birth and
 * death rules and run invariants (at most one agent per cell, 0 <= sugar <=
 * cap, population ledger), all derived from the rules above.  The paper fixes
 * none of these rules, so with respect to the paper this function is parity
 * unpinned. */

#define SUG_STREAM_CHILD_METAB 10
#define SUG_STREAM_CHILD_VISION 11

static int64_t wrap_cell(int32_t side, int32_t x, int32_t y) {
  x = ((x % side) + side) % side;
  y = ((y % side) + side) % side;
  return (int64_t)y * side + x;
}

int orc_sugar_run(int32_t side, int32_t steps, int32_t step0, uint64_t seed,
                  const orc_sugar_rules *rules, int32_t *sugar, const int32_t *cap,
                  uint8_t *occ, int32_t *a_sugar, int32_t *a_metab,
                  int32_t *a_vision, int32_t *a_age, int64_t *counts) {
  if (side < 1 || steps < 0) return -1;
  const int64_t n = (int64_t)side * side;
  int64_t *target = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *req = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  uint8_t *snap = (uint8_t *)malloc((size_t)n);
  if (!target || !req || !snap) {
    free(target); free(req); free(snap);
    return -1;
  }
  const int dx[4] = {1, -1, 0, 0};
  const int dy[4] = {0, 0, 1, -1};
  for (int32_t s = 0; s < steps; s++) {
    const uint64_t t = (uint64_t)(step0 + s);
    /* 1 regrow */
    for (int64_t c = 0; c < n; c++) sugar[c] = sugar[c] + 1 < cap[c] ? sugar[c] + 1 : cap[c];
    /* 2 choose, against the occupancy at the start of the phase */
    memcpy(snap, occ, (size_t)n);
    for (int64_t c = 0; c < n; c++) req[c] = INT64_MAX;
    for (int64_t p = 0; p < n; p++) {
      if (!snap[p]) continue;
      int32_t px = (int32_t)(p % side), py = (int32_t)(p / side);
      int64_t best = p;
      int32_t best_sugar = sugar[p], best_dist = 0;
      for (int d = 0; d < 4; d++)
        for (int32_t k = 1; k <= a_vision[p]; k++) {
          int64_t q = wrap_cell(side, px + dx[d] * k, py + dy[d] * k);
          if (snap[q]) continue;
          int better = sugar[q] > best_sugar ||
                       (sugar[q] == best_sugar && (k < best_dist || (k == best_dist && q < best)));
          if (better) {
            best = q;
            best_sugar = sugar[q];
            best_dist = k;
          }
        }
      target[p] = best;
      if (best != p && p < req[best]) req[best] = p;
    }
    /* 3 move: sources were occupied and targets empty in the snapshot, so the
     * moves are disjoint and can be applied in any order. */
    for (int64_t p = 0; p < n; p++) {
      if (!snap[p] || target[p] == p || req[target[p]] != p) continue;
      int64_t q = target[p];
      occ[q] = 1;
      a_sugar[q] = a_sugar[p];
      a_metab[q] = a_metab[p];
      a_vision[q] = a_vision[p];
      a_age[q] = a_age[p];
      occ[p] = 0;
      if (counts) counts[2]++;
    }
    /* 4 eat, metabolise, age, die */
    for (int64_t c = 0; c < n; c++) {
      if (!occ[c]) continue;
      a_sugar[c] += sugar[c];
      sugar[c] = 0;
      a_sugar[c] -= a_metab[c];
      a_age[c] += 1;
      if (a_sugar[c] <= 0 || a_age[c] >= rules->max_age) {
        occ[c] = 0;
        if (counts) counts[1]++;
      }
    }
    /* 5 reproduce-request, against the occupancy after phase 4 */
    memcpy(snap, occ, (size_t)n);
    for (int64_t c = 0; c < n; c++) req[c] = INT64_MAX;
    for (int64_t p = 0; p < n; p++) {
      target[p] = -1;
      if (!snap[p]) continue;
      if (a_sugar[p] < rules->repro_min || a_age[p] < rules->fertile_min || a_age[p] > rules->fertile_max)
        continue;
      int32_t px = (int32_t)(p % side), py = (int32_t)(p / side);
      int64_t best = -1;
      for (int d = 0; d < 4; d++) {
        int64_t q = wrap_cell(side, px + dx[d], py + dy[d]);
        if (!snap[q] && (best < 0 || q < best)) best = q;
      }
      if (best < 0) continue;
      target[p] = best;
      if (p < req[best]) req[best] = p;
    }
    /* 6 birth */
    for (int64_t p = 0; p < n; p++) {
      if (!snap[p] || target[p] < 0 || req[target[p]] != p) continue;
      int64_t q = target[p];
      int32_t give = a_sugar[p] / 2;
      a_sugar[p] -= give;
      occ[q] = 1;
      a_sugar[q] = give;
      a_metab[q] = orc_uniform_int(orc_hash(seed, SUG_STREAM_CHILD_METAB, t, (uint64_t)q), 1, 4);
      a_vision[q] = orc_uniform_int(orc_hash(seed, SUG_STREAM_CHILD_VISION, t, (uint64_t)q), 1, 6);
      a_age[q] = 0;
      if (counts) counts[0]++;
    }
  }
  free(target);
  free(req);
  free(snap);
  return 0;
}

/* =============================================================== traffic
 * Nagel-Schreckenberg cellular traffic (the paper's "traffic" application
 * names the model; its rules are the published ones), on open single-lane
 * roads.  One step t, for every car at cell i of road r with speed v, all
 * decisions taken on the state at the start of the step:
 *  1 accelerate: v = min(v + 1, vmax);
 *  2 brake: v = min(v, gap), gap = the empty cells directly ahead of the car
 *    (cells past the road's end count as empty: the exit);
 *  3 dawdle: if v > 0 and Bernoulli(p_slow) from hash(seed, 32, r*length + i, t),
 *    v = v - 1;
 *  4 move: the car advances v cells; one that passes the last cell leaves.
 * Then on every road whose first cell is empty, a car enters there at speed 0
 * when Bernoulli(p_in) from hash(seed, 33, r, t).
 * Moves never collide: a car ends before the old cell of the car ahead. */

#define TRAFFIC_STREAM_SLOW 32
#define TRAFFIC_STREAM_IN 33

int orc_traffic_run(int32_t roads, int32_t length, int32_t steps, int32_t step0, uint64_t seed,
                    int32_t vmax, uint32_t p_slow24, uint32_t p_in24, int32_t *vel, int64_t *counts) {
  if (roads < 1 || length < 1 || steps < 0 || vmax < 1) return -1;
  const int64_t n = (int64_t)roads * length;
  int32_t *next = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!next) return -1;
  for (int32_t s = 0; s < steps; s++) {
    const uint64_t t = (uint64_t)(step0 + s);
    for (int64_t c = 0; c < n; c++) next[c] = -1;
    for (int32_t r = 0; r < roads; r++) {
      const int32_t *road = vel + (int64_t)r * length;
      for (int32_t i = 0; i < length; i++) {
        if (road[i] < 0) continue;
        int32_t v = road[i] + 1 < vmax ? road[i] + 1 : vmax;
        int32_t gap = 0;
        while (gap < v && (i + gap + 1 >= length || road[i + gap + 1] < 0)) gap++;
        if (gap < v) v = gap;
        const uint64_t h = orc_hash(seed, TRAFFIC_STREAM_SLOW, (uint64_t)r * (uint64_t)length + (uint64_t)i, t);
        if (v > 0 && (uint32_t)(h >> 40) < p_slow24) v--;
        if (i + v >= length) {
          counts[1]++;
        } else {
          next[(int64_t)r * length + i + v] = v;
        }
      }
    }
    for (int32_t r = 0; r < roads; r++) {
      const uint64_t h = orc_hash(seed, TRAFFIC_STREAM_IN, (uint64_t)r, t);
      if (next[(int64_t)r * length] < 0 && (uint32_t)(h >> 40) < p_in24) {
        next[(int64_t)r * length] = 0;
        counts[0]++;
      }
    }
    memcpy(vel, next, (size_t)n * sizeof(int32_t));
  }
  free(next);
  return 0;
}

/* ============================================================ collisions
 * Bodies in the plane under mutual attraction, merging when they come close
 * (the paper names the application; the rules here are the ones adopted,
 * written out in full).  G is folded into the masses.  One step:
 *  1 acceleration of every live body i, summed over all ids j in increasing
 *    order (j = i and merged bodies contribute exactly 0):
 *      dx = x_j - x_i, dy = y_j - y_i, r2 = fma(dx, dx, fma(dy, dy, eps2)),
 *      s = m_j / (r2 * sqrt(r2)), ax = fma(s, dx, ax), ay = fma(s, dy, ay)
 *  2 move: vx = fma(dt, ax, vx), x = fma(dt, vx, x) (and y)
 *  3 roots: a live body is a root if no live body of lower id lies within
 *    the merge radius: d2 = fma(dx, dx, dy * dy) < r2_merge
 *  4 targets: a live non-root body merges into the lowest-id root within the
 *    merge radius, if there is one
 *  5 merge: a root that absorbs bodies takes, in increasing id order of the
 *    absorbed, M = M + m_i, P = fma(m_i, v_i, P) and C = fma(m_i, x_i, C),
 *    starting from M = m_j, P = m_j * v_j, C = m_j * x_j; then v = P / M,
 *    x = C / M, m = M.  Roots that absorb nothing are unchanged.
 *  6 the absorbed bodies are removed (m = 0).
 * Every operation is IEEE single precision with one rounding; fma and sqrt
 * are correctly rounded. */

int orc_collide_run(int32_t n, int32_t steps, const orc_collide_params *p, float *x, float *y, float *vx,
                    float *vy, float *m, int64_t *counts) {
  if (n < 1 || steps < 0) return -1;
  float *ax = (float *)malloc((size_t)n * sizeof(float));
  float *ay = (float *)malloc((size_t)n * sizeof(float));
  int32_t *target = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  uint8_t *root = (uint8_t *)malloc((size_t)n);
  if (!ax || !ay || !target || !root) {
    free(ax); free(ay); free(target); free(root);
    return -1;
  }
  for (int32_t s = 0; s < steps; s++) {
    for (int32_t i = 0; i < n; i++) {
      float sx = 0.0f, sy = 0.0f;
      if (m[i] > 0.0f) {
        for (int32_t j = 0; j < n; j++) {
          const float dx = x[j] - x[i], dy = y[j] - y[i];
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, p->eps2));
          const float sc = m[j] / (r2 * sqrtf(r2));
          sx = fmaf(sc, dx, sx);
          sy = fmaf(sc, dy, sy);
        }
      }
      ax[i] = sx;
      ay[i] = sy;
    }
    for (int32_t i = 0; i < n; i++) {
      if (!(m[i] > 0.0f)) continue;
      vx[i] = fmaf(p->dt, ax[i], vx[i]);
      vy[i] = fmaf(p->dt, ay[i], vy[i]);
      x[i] = fmaf(p->dt, vx[i], x[i]);
      y[i] = fmaf(p->dt, vy[i], y[i]);
    }
    for (int32_t i = 0; i < n; i++) {
      root[i] = 0;
      if (!(m[i] > 0.0f)) continue;
      int near_lower = 0;
      for (int32_t j = 0; j < i && !near_lower; j++) {
        if (!(m[j] > 0.0f)) continue;
        const float dx = x[j] - x[i], dy = y[j] - y[i];
        if (fmaf(dx, dx, dy * dy) < p->r2_merge) near_lower = 1;
      }
      root[i] = (uint8_t)!near_lower;
    }
    for (int32_t i = 0; i < n; i++) {
      target[i] = -1;
      if (!(m[i] > 0.0f) || root[i]) continue;
      for (int32_t j = 0; j < n; j++) {
        if (!root[j]) continue;
        const float dx = x[j] - x[i], dy = y[j] - y[i];
        if (fmaf(dx, dx, dy * dy) < p->r2_merge) {
          target[i] = j;
          break;
        }
      }
    }
    for (int32_t j = 0; j < n; j++) {
      if (!root[j]) continue;
      float M = m[j], px = m[j] * vx[j], py = m[j] * vy[j], cx = m[j] * x[j], cy = m[j] * y[j];
      int absorbed = 0;
      for (int32_t i = 0; i < n; i++) {
        if (target[i] != j) continue;
        M = M + m[i];
        px = fmaf(m[i], vx[i], px);
        py = fmaf(m[i], vy[i], py);
        cx = fmaf(m[i], x[i], cx);
        cy = fmaf(m[i], y[i], cy);
        absorbed++;
      }
      if (!absorbed) continue;
      vx[j] = px / M;
      vy[j] = py / M;
      x[j] = cx / M;
      y[j] = cy / M;
      m[j] = M;
    }
    for (int32_t i = 0; i < n; i++)
      if (target[i] >= 0) {
        m[i] = 0.0f;
        counts[0]++;
      }
  }
  free(ax); free(ay); free(target); free(root);
  return 0;
}


/* ================================================================= wa-tor
 * Fish and sharks on a square torus (the paper names the application; the
 * rules are Dewdney's published ones in a synchronous reading, written out in
 * full).  kind[c]: 0 empty, 1 fish, 2 shark; age[c] for both, energy[c] for
 * sharks.  Neighbours of a cell in the order up, right, down, left (torus).
 * One step t:
 *  Fish: on the grid at the start of the phase, a fish picks one of its empty
 *    neighbours, the k-th in neighbour order with k = U{0..n-1} from
 *    hash(seed, 40, c, t), n = number of empty neighbours.  A target cell
 *    requested by several fish goes to the lowest requesting cell.  Every
 *    fish ages by one; a fish that moves with age >= fish_breed leaves a
 *    newborn fish (age 0) in the cell it left and its own age becomes 0.
 *  Sharks: on the grid after the fish phase, a shark picks one of its fish
 *    neighbours (k from hash(seed, 41, c, t) over them) or, if it has none
 *    and its energy is above 1, one of its empty neighbours (same draw).  The
 *    lowest requesting cell wins a target.  A shark that moves onto a fish
 *    eats it and its energy becomes `starve`; any other shark loses one unit
 *    and dies where it stands when it reaches 0.  Sharks age and breed as
 *    fish do (shark_breed; a newborn shark has energy `starve`).
 * After each step empty cells hold age 0 and energy 0, and fish energy 0.
 * counts[0..3] += fish born, sharks born, fish eaten, sharks starved. */

#define WATOR_STREAM_FISH 40
#define WATOR_STREAM_SHARK 41

static int64_t wator_nb(int32_t side, int64_t c, int d) {
  const int64_t x = c % side, y = c / side;
  int64_t nx = x, ny = y;
  if (d == 0) ny = y == 0 ? side - 1 : y - 1;
  if (d == 1) nx = x + 1 == side ? 0 : x + 1;
  if (d == 2) ny = y + 1 == side ? 0 : y + 1;
  if (d == 3) nx = x == 0 ? side - 1 : x - 1;
  return ny * side + nx;
}

/* Lowest requesting cell per target: win[target] = min over requesters. */
static void wator_resolve(int64_t n, const int64_t *target, int64_t *win) {
  for (int64_t c = 0; c < n; c++) win[c] = -1;
  for (int64_t c = 0; c < n; c++) {
    const int64_t t = target[c];
    if (t >= 0 && (win[t] < 0 || c < win[t])) win[t] = c;
  }
}

int orc_wator_run(int32_t side, int32_t steps, int32_t step0, uint64_t seed, int32_t fish_breed,
                  int32_t shark_breed, int32_t starve, int32_t *kind, int32_t *age, int32_t *energy,
                  int64_t *counts) {
  if (side < 1 || steps < 0 || fish_breed < 1 || shark_breed < 1 || starve < 1) return -1;
  const int64_t n = (int64_t)side * side;
  int64_t *target = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *win = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int32_t *k0 = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!target || !win || !k0) {
    free(target);
    free(win);
    free(k0);
    return -1;
  }
  for (int32_t s = 0; s < steps; s++) {
    const uint64_t t = (uint64_t)(step0 + s);
    /* fish phase */
    memcpy(k0, kind, (size_t)n * sizeof(int32_t));
    for (int64_t c = 0; c < n; c++) {
      target[c] = -1;
      if (k0[c] != 1) continue;
      int64_t opt[4];
      int m = 0;
      for (int d = 0; d < 4; d++) {
        const int64_t q = wator_nb(side, c, d);
        if (k0[q] == 0) opt[m++] = q;
      }
      if (m > 0) target[c] = opt[orc_uniform_int(orc_hash(seed, WATOR_STREAM_FISH, (uint64_t)c, t), 0, m - 1)];
    }
    wator_resolve(n, target, win);
    for (int64_t c = 0; c < n; c++) {
      if (k0[c] != 1) continue;
      const int32_t a = age[c] + 1;
      const int64_t q = target[c];
      if (q >= 0 && win[q] == c) {
        kind[q] = 1;
        if (a >= fish_breed) {
          age[q] = 0;
          age[c] = 0; /* the newborn stays in the old cell */
          counts[0]++;
        } else {
          age[q] = a;
          kind[c] = 0;
        }
      } else {
        age[c] = a;
      }
    }
    /* shark phase */
    memcpy(k0, kind, (size_t)n * sizeof(int32_t));
    for (int64_t c = 0; c < n; c++) {
      target[c] = -1;
      if (k0[c] != 2) continue;
      int64_t fish[4], empty[4];
      int nf = 0, ne = 0;
      for (int d = 0; d < 4; d++) {
        const int64_t q = wator_nb(side, c, d);
        if (k0[q] == 1) fish[nf++] = q;
        if (k0[q] == 0) empty[ne++] = q;
      }
      const uint64_t h = orc_hash(seed, WATOR_STREAM_SHARK, (uint64_t)c, t);
      if (nf > 0)
        target[c] = fish[orc_uniform_int(h, 0, nf - 1)];
      else if (ne > 0 && energy[c] > 1)
        target[c] = empty[orc_uniform_int(h, 0, ne - 1)];
    }
    wator_resolve(n, target, win);
    for (int64_t c = 0; c < n; c++) {
      if (k0[c] != 2) continue;
      const int64_t q = target[c];
      const int won = q >= 0 && win[q] == c;
      const int ate = won && k0[q] == 1;
      const int32_t e = ate ? starve : energy[c] - 1;
      const int32_t a = age[c] + 1;
      if (e <= 0) {
        kind[c] = 0;
        counts[3]++;
      } else if (won) {
        if (ate) counts[2]++;
        kind[q] = 2;
        energy[q] = e;
        if (a >= shark_breed) {
          age[q] = 0;
          age[c] = 0;
          energy[c] = starve;
          counts[1]++;
        } else {
          age[q] = a;
          kind[c] = 0;
        }
      } else {
        energy[c] = e;
        age[c] = a;
      }
    }
    /* Canonical sea: empty cells carry age 0 and energy 0, fish energy 0. */
    for (int64_t c = 0; c < n; c++) {
      if (kind[c] == 0) age[c] = 0;
      if (kind[c] != 2) energy[c] = 0;
    }
  }
  free(target);
  free(win);
  free(k0);
  return 0;
}
