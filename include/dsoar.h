/*
 * dsoar.h - C ABI of the MI355X object heap and parallel do-all.
 *
 * The method is DynaSOAr's (arXiv 1809.07444): a device-side heap of
 * equal-size blocks, each holding objects of one type in an SOA layout
 * (Sec. 2, "heap layout" figure), block states indexed by lock-free
 * hierarchical bitmaps (Sec. 2 "Block States", Sec. 3, Alg. 2), allocation
 * by Alg. 1 (Sec. 2.2) with wavefront request coalescing (Sec. 2.4), and a
 * parallel do-all that compacts the allocated blocks of a type and assigns
 * one wavefront lane per object slot (Sec. 2.3, "thread assignment" figure).
 *
 * Conventions for every entry point:
 *  - Return value: DSOAR_OK (0) or a negative dsoar_status.  Nothing throws.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous and stream-ordered unless stated otherwise; every
 *    call that touches one heap must be issued on one stream (the heap relies
 *    on stream order for quiescence between kernels).
 *  - Pointers named *_dev are device pointers; all others are host pointers.
 *  - The caller owns all memory it passes in.  The heap never allocates device
 *    memory: it lives inside the caller's buffer, which must stay allocated
 *    until dsoar_heap_destroy.  Host metadata is owned by the heap handle.
 *  - A heap handle must not be used from two host threads at once.
 *
 * Device-side `new` and `delete` are C++ device functions (dsoar_new,
 * dsoar_delete in the package's device header) called inside kernels; the
 * do-all methods and workload kernels listed below use them.
 */
#ifndef DSOAR_H
#define DSOAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSOAR_MAX_TYPES 8
#define DSOAR_MAX_FIELDS 8
#define DSOAR_NULL 0xFFFFFFFFu /* the null object handle */
#define DSOAR_ABI_VERSION 2

typedef enum {
  DSOAR_OK = 0,
  DSOAR_ERR_INVALID_ARG = -1,  /* bad size, type, field or pointer */
  DSOAR_ERR_OOM = -2,          /* a device new found no free block (sticky) */
  DSOAR_ERR_RETRY_LIMIT = -3,  /* a bounded device retry loop gave up (sticky) */
  DSOAR_ERR_HIP = -4,          /* a HIP runtime call failed */
  DSOAR_ERR_DOUBLE_FREE = -5,  /* delete of a slot that was not allocated (sticky) */
  DSOAR_ERR_TOO_SMALL = -6,    /* the caller's buffer is smaller than required */
  DSOAR_ERR_UNSUPPORTED = -7   /* method/type combination not available */
} dsoar_status;

/* Object handle: (block << 6) | slot.  DSOAR_NULL on failure. */
typedef uint32_t dsoar_obj;

typedef struct dsoar_heap dsoar_heap;

/* Per-type field layout (Sec. 2: one SOA array per field inside a block).
 * field_bytes[i] is 4 or 8.  parent: 0 for a type of its own, else 1 + the
 * index of its parent type (Sec. 1.2: class inheritance without wasted
 * memory).  A subclass is declared after its parent and begins with the
 * parent's fields (same count and widths), followed by its own; its blocks
 * hold only its own objects, in its own SOA layout, so neither type carries
 * the other's fields.  A do-all over a type visits the objects of the type
 * and of all its subclasses, its method reading the inherited fields by the
 * parent's field indices. */
typedef struct {
  uint32_t num_fields;
  uint32_t field_bytes[DSOAR_MAX_FIELDS];
  uint32_t parent;
} dsoar_type_layout;

/* Heap geometry.  num_blocks = M (1 .. 2^26 - 1: in a heap of 2^26 blocks
 * slot 63 of the last block would have the handle DSOAR_NULL).  block_capacity = slots per
 * block of every type, 64 (one wavefront per block, the paper's capacity for
 * the smallest type) or 32 (two blocks per wavefront; Sec. 2 notes capacities
 * of at least 32 keep 4-byte SOA arrays at 128 bytes), or 0 for the byte-size
 * rule of Sec. 2: the smallest type has 64 slots and fixes the block size (64
 * of its objects), every other type the largest power of two of slots that
 * fits a block (64 / c blocks per wavefront in a do-all).  All types are
 * declared up front (Sec. 2, footnote on pre-declared types). */
typedef struct {
  uint32_t num_blocks;
  uint32_t block_capacity;
  uint32_t num_types;
  uint32_t bitmap_width; /* bits per container of the block-state bitmaps (Sec. 3):
                            64 (or 0) or 32.  It fixes the fan-out of every level
                            and so the number of levels, ceil(log_width M) */
  dsoar_type_layout types[DSOAR_MAX_TYPES];
} dsoar_heap_desc;

/* Byte offsets of the heap's regions inside the caller's buffer, for tests
 * and tools that inspect device memory directly. */
typedef struct {
  uint64_t total_bytes;
  uint64_t data_offset;       /* block b, field f of type t at data_offset +
                                 b*block_stride + field_offset[t][f] + slot*width */
  uint64_t block_stride;
  uint64_t obj_bitmap_offset; /* uint64 per block: bit s = slot s allocated */
  uint64_t block_type_offset; /* uint32 per block: type in the low 8 bits (0xFF =
                                 free), times the block was freed above them */
  uint64_t bitmaps_offset;    /* (1 + 2*num_types) hierarchical bitmaps:
                                 0 = free, 1+2t = allocated[t], 2+2t = active[t] */
  uint64_t bitmap_stride;     /* bytes between consecutive bitmaps */
  uint32_t bitmap_width;      /* container width in bits (32 or 64) */
  uint32_t num_levels;        /* levels per bitmap (level 0 = one bit per block) */
  uint32_t level_word_offset[8]; /* per level: offset in containers from the bitmap's start */
  uint32_t level_words[8];       /* per level: containers (level bit j is bit j % 32 of the
                                    32-bit unit j / 32 of the level at either width) */
  uint32_t field_offset[DSOAR_MAX_TYPES][DSOAR_MAX_FIELDS];
  uint32_t type_capacity[DSOAR_MAX_TYPES]; /* slots per block of each type */
} dsoar_heap_layout;

/* Quiescent statistics, filled by dsoar_heap_stats. */
typedef struct {
  uint64_t allocs[DSOAR_MAX_TYPES];       /* successful device news */
  uint64_t frees[DSOAR_MAX_TYPES];        /* successful device deletes */
  uint64_t live_objects[DSOAR_MAX_TYPES]; /* popcount of the object bitmaps */
  uint64_t visits[DSOAR_MAX_TYPES];       /* objects visited by do-all methods */
  uint32_t allocated_blocks[DSOAR_MAX_TYPES];
  uint32_t active_blocks[DSOAR_MAX_TYPES];
  uint32_t typed_blocks[DSOAR_MAX_TYPES]; /* blocks whose type word is t */
  uint64_t reserve_retries;               /* reservations that gained fewer bits than tried */
  uint64_t slow_paths;                    /* free blocks taken (Alg. 1 slow path) */
  uint64_t find_fails;                    /* try_find_set FAILs on active[T] */
  uint64_t method_atomics;                /* atomic RMWs do-all methods issued on their own data */
  uint64_t online_releases;               /* blocks freed by the delete that emptied them */
  uint64_t blocks_taken;                  /* free-block count: blocks taken from the free bitmap */
  uint64_t blocks_returned;               /* and returned to it; num_blocks + returned - taken
                                             blocks are free or being opened (a request is out of
                                             memory only when this reads 0, Sec. 2.2) */
  uint32_t free_blocks;
  uint32_t num_blocks;
  uint32_t oom;                           /* sticky flags */
  uint32_t retry_limit_hit;
  uint32_t double_free;
  uint32_t reserved;
} dsoar_stats;

/* Invariant codes reported by dsoar_heap_check (counts per code). */
enum {
  DSOAR_INV_BITMAP_RANGE = 0, /* object bits set at or above the capacity */
  DSOAR_INV_ALLOCATED = 1,    /* allocated[T] <=> type T and non-empty */
  DSOAR_INV_ACTIVE = 2,       /* active[T] <=> allocated[T] and not full */
  DSOAR_INV_ACTIVE_IMPLIES_ALLOCATED = 3,
  DSOAR_INV_FREE = 4,         /* free <=> untyped and empty; states disjoint */
  DSOAR_INV_CONTAINER = 5,    /* nested bit = OR of its container (Sec. 3) */
  DSOAR_INV_LIVE_COUNT = 6,   /* live = allocs - frees, per type */
  DSOAR_INV_FREE_COUNT = 7,   /* free blocks = num_blocks + returned - taken */
  DSOAR_INV_COUNT = 8
};

/* ------------------------------------------------------------------ heap -- */

/* Device bytes a heap of this geometry needs (0 if the descriptor is invalid). */
size_t dsoar_heap_bytes(const dsoar_heap_desc* desc);

/* Creates a heap inside dev_mem (device, >= dsoar_heap_bytes, 256-byte
 * aligned) and initialises it on `stream`: every block free (Sec. 2, "block
 * states" figure: initially every block is free), all other bitmaps empty.
 * *out receives the host handle.  Errors: INVALID_ARG, TOO_SMALL, HIP. */
int dsoar_heap_create(const dsoar_heap_desc* desc, void* dev_mem, size_t dev_bytes,
                      void* stream, dsoar_heap** out);

/* Frees the host handle.  Never touches dev_mem. */
int dsoar_heap_destroy(dsoar_heap* heap);

/* Returns the heap to its initial (all free) state, clears the counters and
 * the sticky flags. */
int dsoar_heap_reset(dsoar_heap* heap, void* stream);

int dsoar_heap_get_layout(const dsoar_heap* heap, dsoar_heap_layout* out);

/* Launch shape of do-all kernels: workgroups of wg_threads (64..1024, a
 * multiple of 64) and, for persistent launches, wgs_per_cu workgroups per
 * compute unit (1..64).  Defaults 256 and 8. */
int dsoar_heap_set_launch(dsoar_heap* heap, uint32_t wg_threads, uint32_t wgs_per_cu);

/* Allocation policy.  By default (bulk_min = 0xFFFFFFFF) a wavefront fills
 * active blocks of the type first (Sec. 2.2) and takes free blocks only when
 * it finds none, whole ones while it still needs at least a block's worth.
 * A wavefront whose outstanding requests number at least bulk_min instead
 * takes whole free blocks directly, without the active lookup (fewer atomics,
 * more partially filled blocks).  Values below the block capacity mean the
 * capacity. */
int dsoar_heap_set_policy(dsoar_heap* heap, uint32_t bulk_min);

/* Per-type allocation policy.  DSOAR_POLICY_DENSE (the default for every
 * type) is the dense policy above.  With DSOAR_POLICY_FRESH a request of the
 * type skips the active lookup: a wavefront opens free blocks of its own
 * (whole ones while it needs at least a block's worth, then one block for the
 * rest, which stays active like any other partly filled block).  Meant for
 * types whose objects all die within one phase, so that dense packing buys
 * nothing and the lookup is pure latency (the Game of Life's Candidates).
 * DSOAR_POLICY_BOUNDED is the dense policy with at most two passes over
 * active blocks per request; what is still missing then comes from a free
 * block: for types whose active blocks hold only a slot or two each, where
 * filling every hole costs many passes.  Under FRESH and BOUNDED a request
 * that finds no free block goes back to the active blocks, so the heap is
 * still out of memory only when it is full.  The slot placement differs, the
 * results do not.  type >= the heap's number of types or another policy
 * value: DSOAR_ERR_INVALID_ARG. */
enum { DSOAR_POLICY_DENSE = 0, DSOAR_POLICY_FRESH = 1, DSOAR_POLICY_BOUNDED = 2 };
int dsoar_heap_set_type_policy(dsoar_heap* heap, uint32_t type, uint32_t policy);

/* Where the bitmap searches of a wavefront start (any set bit may be
 * returned, Sec. 2.1; results never depend on it).  DSOAR_SEARCH_HASHED (the
 * default): a hash of the wavefront's index, spreading concurrent searches
 * over the whole bitmap.  DSOAR_SEARCH_LOWEST: the lowest set bit at every
 * level (and the lowest free slots of a block), the sequential choice.
 * DSOAR_SEARCH_XCD: the hash, with the top level's choice narrowed to the
 * eighth of the top container that the wavefront's XCD owns, so that the
 * eight XCDs mostly work in disjoint parts of the heap.  Other values:
 * DSOAR_ERR_INVALID_ARG. */
enum { DSOAR_SEARCH_HASHED = 0, DSOAR_SEARCH_LOWEST = 1, DSOAR_SEARCH_XCD = 2 };
int dsoar_heap_set_search(dsoar_heap* heap, uint32_t policy);

/* Block reclamation.  By default (online = 0) a block emptied by deletes
 * stays allocated to its type until the next enumeration of that type or
 * dsoar_reclaim returns it to the free bitmap, at a point where no kernel of
 * the heap runs.  With online = 1 the delete that empties a block frees it at
 * once (Sec. 2 block states: free = holds no object), so other types can take
 * it within the same kernel; allocations then pin a block while reserving in
 * it (two more atomics per reservation).  Results do not depend on it. */
int dsoar_heap_set_reclaim(dsoar_heap* heap, int online);

/* Blocks per wavefront pass for do-all methods that split into a load phase
 * and an apply phase (at block capacity 64): 1, 2, 4 (the default) or 8.  The
 * loads of all blocks of a pass are issued before any is used, which keeps
 * more memory traffic in flight (Sec. 2.3: the do-all is bound by memory
 * access).  Used only when every wavefront of the launch gets that many
 * blocks; results do not depend on it.  Other values: DSOAR_ERR_INVALID_ARG. */
int dsoar_heap_set_unroll(dsoar_heap* heap, uint32_t blocks_per_pass);

/* Per-launch timing: when enabled, every enumeration, do-all and
 * object-creating launch of this heap is bracketed by a pair of HIP events
 * on its stream (at most 8192 launches are recorded between reports).
 * dsoar_heap_timing synchronises on the last event, aggregates the recorded
 * launches by kernel kind into kinds/counts/total_ms, and clears the records.
 * Kinds: 1 enumeration; do-alls 10 visit count, 11 delete-if-mod, 12 gather,
 * 20/21 micro update/cull, 30..33 Game of Life phases 1..4 (35: phases 3 and
 * 4 in one launch, 34 world deletion), 40..45 Sugarscape phases and world
 * deletion, 50/51 traffic decide/drive, 60..65 collisions, 70..76 wa-tor;
 * other kernels 22 micro creation, 36/37 Game of Life initial cells and
 * admission, 46/47 Sugarscape regrow and admission, 52/53 traffic entry and
 * initial cars, 66 collisions initial bodies, 77/78 wa-tor initial sea and
 * step tick. */
int dsoar_heap_set_timing(dsoar_heap* heap, int enable);
int dsoar_heap_timing(dsoar_heap* heap, uint32_t* kinds, uint32_t* counts, double* total_ms,
                      uint32_t max_kinds, uint32_t* num_kinds);

/* The HIP error code of the last failed HIP call made for this heap. */
int dsoar_last_hip_error(const dsoar_heap* heap);

/* Parallel enumeration (Sec. 2.3, two steps): compacts the set bits of
 * allocated[type] into the heap's index array R (ascending block ids) with a
 * snapshot S of each block's object bitmap, and the count, all on the device.
 * Blocks of `type` that are empty are first returned to the free state
 * (quiescent reclamation).  Must be ordered after every kernel that mutates
 * the heap. */
int dsoar_enumerate(dsoar_heap* heap, uint32_t type, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the enumeration
 * of dsoar_enumerate, block reclamation included, written to the caller's
 * R_dev (uint32, at least num_blocks entries), S_dev (uint64, as many) and
 * count_dev (one uint32), with the scan's ticket, epoch and look-back words
 * in a fixed scratch array of the library (about 128 KiB per GPU, held until
 * the process ends) instead of the heap's buffer; allocates nothing.  Covers
 * heaps of up to 2^26 - 1 blocks, the largest dsoar_heap_create accepts;
 * other arguments out of range: DSOAR_ERR_INVALID_ARG.  Every call on one GPU
 * shares that GPU's scratch (each call clears what it needs first), so calls
 * that overlap on one GPU, on different streams or from different threads,
 * race and must be ordered by the caller. */
int dsoar_enumerate_noalloc(dsoar_heap* heap, uint32_t type, uint32_t* R_dev, uint64_t* S_dev,
                            uint32_t* count_dev, void* stream);

/* Reads back the count of the last enumeration of `type` (synchronises). */
int dsoar_enum_count(dsoar_heap* heap, uint32_t type, uint32_t* count, void* stream);

/* Device addresses of the enumeration arrays of `type`: R (uint32 block ids)
 * and S (uint64 object-bitmap snapshots), valid until the heap is destroyed. */
int dsoar_enum_arrays(dsoar_heap* heap, uint32_t type, uint64_t* R_dev, uint64_t* S_dev);

/* Returns every empty typed block, of every type, to the free state. */
int dsoar_reclaim(dsoar_heap* heap, void* stream);

/* Do-all flags. */
#define DSOAR_DO_PERSISTENT 0u  /* fixed grid, loops over the device count (graph-safe) */
#define DSOAR_DO_PLAIN 1u       /* reads the count back (synchronises) and launches
                                   exactly count*capacity/64 wavefronts */
#define DSOAR_DO_REUSE_ENUM 2u  /* skip enumeration: reuse R/S/count of the last
                                   dsoar_enumerate of this type (valid only if no
                                   object of the type was created or deleted since) */

/* Built-in do-all methods. */
enum {
  DSOAR_METHOD_VISIT_COUNT = 1,  /* args: dsoar_visit_args.  counts_dev[obj] += 1 */
  DSOAR_METHOD_DELETE_IF_MOD = 2,/* args: dsoar_mod_args.  delete this if the
                                    int32 field % modulus == residue */
  DSOAR_METHOD_MICRO_UPDATE = 3, /* args: none.  x = fma(0.01f, v, x) on the
                                    microbenchmark type {int32 id, f32 x, f32 v} */
  DSOAR_METHOD_MICRO_CULL = 4,   /* args: none.  delete this if id % 3 == 0 */
  DSOAR_METHOD_FIELD_GATHER = 5  /* args: dsoar_gather_args.  out_dev[key] = field */
};

typedef struct { uint32_t* counts_dev; } dsoar_visit_args;            /* num_blocks*64 entries */
typedef struct { uint32_t field; int32_t modulus; int32_t residue; } dsoar_mod_args;
typedef struct { uint32_t key_field; uint32_t field; uint32_t num_keys; uint32_t reserved;
                 void* out_dev; uint8_t* present_dev; } dsoar_gather_args;

/* Runs `method` once for every object of `type`, and of every type that
 * inherits from it (Sec. 1.2), that is live when the enumeration runs (Sec.
 * 2.3: c consecutive lanes per allocated block, lane tid % c handles slot
 * tid % c when that slot is allocated).  The lists of all those types are
 * enumerated before any method runs; field indices in `args` name fields of
 * `type`, which its subclasses inherit.  Objects created during the do-all
 * are not visited; a method may delete only `this`, which takes effect when
 * its wavefront finishes the block.  Errors: INVALID_ARG, UNSUPPORTED
 * (unknown method), HIP. */
int dsoar_parallel_do(dsoar_heap* heap, uint32_t type, uint32_t method,
                      const void* args, size_t args_bytes, uint32_t flags, void* stream);

/* Counters, sticky flags and block/object counts (Sec. 2, "Block States":
 * free, allocated[T] and active[T] blocks counted from their bitmaps, live
 * objects from the object allocation bitmaps).  Synchronises `stream`.
 * Returns OOM / RETRY_LIMIT / DOUBLE_FREE if the matching sticky flag is set
 * (the struct is filled in either way). */
int dsoar_heap_stats(dsoar_heap* heap, dsoar_stats* out, void* stream);

/* Reclaims all empty blocks, then checks the block-state invariants at
 * quiescence: the state rules of Sec. 2 ("Block States": allocated[T] iff the
 * block holds objects of T, active[T] implies allocated[T], free iff empty)
 * and the container consistency of Sec. 3 (each nested bit is the OR of its
 * container), which holds once every operation has completed.
 * violations[DSOAR_INV_COUNT] receives the number of violations per code.
 * Synchronises `stream`. */
int dsoar_heap_check(dsoar_heap* heap, uint32_t* violations, void* stream);

/* Device entry points for callers without their own kernels: for each of n
 * entries (0 <= n <= 2^32 - 1, taken by wavefronts 64 consecutive entries at
 * a time) a lane calls device new (out_dev[i] = handle or DSOAR_NULL), or
 * device delete of objs_dev[i] (DSOAR_NULL entries are skipped; a handle
 * outside the heap or of a free slot sets the sticky DOUBLE_FREE flag). */
int dsoar_alloc_n(dsoar_heap* heap, uint32_t type, uint32_t n, dsoar_obj* out_dev, void* stream);
int dsoar_free_n(dsoar_heap* heap, const dsoar_obj* objs_dev, uint32_t n, void* stream);

/* Concurrency stress of new/delete (tests): n lanes run `rounds` rounds; in
 * round r each wavefront creates one object per lane of type (spread *
 * wavefront + r) mod num_types, writes the handle into the object's field 0 (4 bytes in
 * every type), and deletes it at once unless a hash of (seed, lane, round)
 * is 0 mod keep; kept handles go to out_dev[lane * rounds + r] (DSOAR_NULL
 * otherwise).  errors_dev[0] (device, zeroed by the caller) counts fields
 * found overwritten, i.e. slots handed out twice.  INVALID_ARG unless
 * 1 <= n <= 2^31 and n * rounds <= 2^32. */
int dsoar_stress_churn(dsoar_heap* heap, uint32_t n, uint32_t rounds, uint32_t keep, uint32_t spread,
                       uint32_t seed, dsoar_obj* out_dev, uint32_t* errors_dev, void* stream);

/* Copies a 4-byte field of n objects to/from a dense device array.
 * DSOAR_NULL and handles outside the heap (block >= num_blocks, or slot >=
 * the type's capacity) are skipped: their array entries are left as they are. */
int dsoar_field_read(dsoar_heap* heap, uint32_t type, uint32_t field, const dsoar_obj* objs_dev,
                     uint32_t n, uint32_t* out_dev, void* stream);
int dsoar_field_write(dsoar_heap* heap, uint32_t type, uint32_t field, const dsoar_obj* objs_dev,
                      uint32_t n, const uint32_t* in_dev, void* stream);

const char* dsoar_error_string(int status);
int dsoar_abi_version(void);

/* ------------------------------------------------------- hierarchical bitmap
 * A stand-alone device bitmap with the heap's operations (Sec. 2.1, Sec. 3,
 * Alg. 2), for testing them in isolation.  Each op runs on its own
 * wavefront, all ops of one call concurrently. */
enum {
  DSOAR_BM_TRY_SET = 0, DSOAR_BM_TRY_CLEAR = 1, DSOAR_BM_SET = 2, DSOAR_BM_CLEAR = 3,
  DSOAR_BM_TRY_FIND_SET = 4, DSOAR_BM_FIND_CLEAR = 5
};
/* Bytes for a bitmap of nbits bits (all levels) with containers of `width`
 * bits (32 or 64).  0 if nbits is 0 or > 2^30, or for another width. */
size_t dsoar_bitmap_bytes(uint32_t nbits, uint32_t width);
/* Initialises all levels: every bit clear (all_set = 0) or every bit < nbits set. */
int dsoar_bitmap_init(void* bm_dev, uint32_t nbits, uint32_t width, int all_set, void* stream);
/* ops_dev: n pairs (kind, pos).  results_dev[i]: 1/0 for try_*, 0 for set/clear
 * (-3 if the retry limit was hit), the position found or -1 (FAIL) for the
 * finds.  start_dev (optional, n entries) gives each find's rotation start. */
int dsoar_bitmap_run(void* bm_dev, uint32_t nbits, uint32_t width, const uint32_t* ops_dev, uint32_t n,
                     const uint32_t* start_dev, int32_t* results_dev, void* stream);

/* --------------------------------------------- microbenchmark workload ----
 * Type {int32 id, float32 x, float32 v} (fields 0, 1, 2). */
/* n lanes each create one object: id = lane, x = x0_dev[id], v = v0_dev[id]. */
int dsoar_micro_init(dsoar_heap* heap, uint32_t type, uint32_t n, const float* x0_dev,
                     const float* v0_dev, void* stream);
/* One step: do-all x = fma(0.01f, v, x); do-all delete id % 3 == 0; then
 * n_renew lanes create id = 3k with x = xs_dev[k], v = vs_dev[k]. */
int dsoar_micro_step(dsoar_heap* heap, uint32_t type, uint32_t n_renew, const float* xs_dev,
                     const float* vs_dev, uint32_t flags, void* stream);

/* ------------------------------------------------------------------ probes
 * Ceilings the heap is measured against (AMD publishes no atomic peak).
 * dsoar_probe_atomics: `waves` wavefronts, one lane each, do `iters` agent-
 * scope 64-bit atomic ORs: mode 0 each on its own 64-byte line (throughput),
 * 1 the same as a dependent chain (latency), 2 all on one word (contention);
 * mode 3 is a chain of dependent agent-scope loads.  buf_dev: >= 16 words,
 * 64-byte aligned, scratch (overwritten).  dsoar_probe_copy: a plain 16-byte
 * vector copy kernel (bytes a multiple of 16). */
int dsoar_probe_atomics(void* buf_dev, uint32_t words, uint32_t mode, uint32_t iters, uint32_t waves,
                        void* stream);
int dsoar_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/* ------------------------------------------------- Game of Life as objects
 * The paper's game-of-life application (Sec. 4, applications figure) on
 * square tori, one or many worlds in one heap.  The heap must declare, in
 * this order, Cell {int32 alive}, Alive {int32 cell, int32 world, int32
 * action} and Candidate {int32 cell, int32 world, int32 action}.  One
 * generation is four do-alls (Alive, Candidate, Alive, Candidate); Candidate
 * and Alive objects are created and deleted with device new/delete. */
typedef struct dsoar_gol dsoar_gol;
#define DSOAR_GRAPH 0x100u     /* capture one generation (step) once into a HIP graph
                                  and replay it (needs a non-default stream) */
#define DSOAR_GOL_GRAPH DSOAR_GRAPH
/* Device bytes for the world table and the cell index (0 if invalid).  sides:
 * host array of num_worlds side lengths (1..65535, total cells < 2^32). */
size_t dsoar_gol_bytes(uint32_t num_worlds, const uint32_t* sides);
/* World w's cell (x, y) has global index off[w] + y*side[w] + x, off being
 * the prefix sum of side^2.  dev_mem: >= dsoar_gol_bytes, 256-byte aligned,
 * caller-owned.  Synchronises `stream` once (uploads the world table). */
int dsoar_gol_create(dsoar_heap* heap, uint32_t num_worlds, const uint32_t* sides, void* dev_mem,
                     size_t dev_bytes, void* stream, dsoar_gol** out);
int dsoar_gol_destroy(dsoar_gol* gol);
/* Creates the objects of the initial state: grid_dev[g] != 0 means cell g is
 * alive (uint8 per global cell).  The heap should be freshly reset. */
int dsoar_gol_init(dsoar_gol* gol, const uint8_t* grid_dev, void* stream);
/* Advances every world by `generations` synchronous B3/S23 generations.
 * flags: DSOAR_DO_PLAIN or DSOAR_DO_PERSISTENT, optionally | DSOAR_GOL_GRAPH
 * (persistent only). */
int dsoar_gol_step(dsoar_gol* gol, uint32_t generations, uint32_t flags, void* stream);
/* grid_dev[g] = 1 if cell g is alive, else 0 (uint8 per global cell). */
int dsoar_gol_read(dsoar_gol* gol, uint8_t* grid_dev, void* stream);
uint32_t dsoar_gol_total_cells(const dsoar_gol* gol);

/* World pool (continuous batching): max_worlds slots over a cell index of
 * arena_cells cells.  Worlds are admitted into free slots and retired between
 * generations; dsoar_gol_step advances every resident world by one
 * generation per call (graph replay works across admissions).  A world's
 * evolution depends only on its own cells, so it is the same alone or with
 * others. */
size_t dsoar_golpool_bytes(uint32_t max_worlds, uint32_t arena_cells);
int dsoar_golpool_create(dsoar_heap* heap, uint32_t max_worlds, uint32_t arena_cells, void* dev_mem,
                         size_t dev_bytes, void* stream, dsoar_gol** out);
/* Admits a side x side world (grid_dev: uint8 per cell, row-major) into a free
 * slot at cell index range [cell_offset, cell_offset + side^2), which must not
 * overlap a resident world. */
int dsoar_gol_admit(dsoar_gol* gol, uint32_t slot, uint32_t cell_offset, uint32_t side,
                    const uint8_t* grid_dev, void* stream);
/* Deletes the objects of the world in `slot` (between generations) and frees it. */
int dsoar_gol_retire(dsoar_gol* gol, uint32_t slot, void* stream);
/* grid_dev[i] = 1 if cell i of the world in `slot` is alive, else 0. */
int dsoar_gol_read_world(dsoar_gol* gol, uint32_t slot, uint8_t* grid_dev, void* stream);

/* ------------------------------------------------- Sugarscape-style agents
 * The paper's sugarscape application (Sec. 4, applications figure) with a
 * synchronous, deterministic rule set on side x side tori.  The heap's type 0
 * must be Agent {int32 sugar, metabolism, vision, age, pos, target, world}.
 * One step: regrow (sugar = min(sugar + 1, cap)); choose the best visible
 * cell (most sugar, then nearest, then lowest index, among the own cell and
 * unoccupied cells up to `vision` along the four axes); move (the lowest
 * requesting cell index wins a target); eat, metabolise, age, and die (delete)
 * at sugar <= 0 or age >= max_age; fertile agents (fertile_min <= age <=
 * fertile_max) with sugar >= repro_min request their lowest-index empty von
 * Neumann neighbour, and the lowest requesting cell index creates a child
 * there (new) with half of its sugar, metabolism U{1..4} and vision U{1..6}
 * drawn from hash(seed, 10 or 11, step, cell), age 0. */
typedef struct dsoar_sugar dsoar_sugar;
typedef struct {
  int32_t max_age, repro_min, fertile_min, fertile_max;
  uint64_t seed; /* seed of the single-world interface */
} dsoar_sugar_rules;

/* World pool (continuous batching): up to max_worlds worlds, each in its own
 * range of an arena of arena_cells cells, stepped together by
 * dsoar_sugar_step.  A world's evolution depends only on its own state, seed
 * and step index, so it is the same alone or with others. */
size_t dsoar_sugarpool_bytes(uint32_t max_worlds, uint32_t arena_cells);
int dsoar_sugarpool_create(dsoar_heap* heap, uint32_t max_worlds, uint32_t arena_cells,
                           const dsoar_sugar_rules* rules, void* dev_mem, size_t dev_bytes,
                           dsoar_sugar** out);
/* Admits a side x side world into a free slot at arena cells [cell_offset,
 * cell_offset + side^2) (must not overlap a resident world), from per-cell
 * device arrays as in dsoar_sugar_init; seed and step0 key its random draws.
 * Checks every cell's sugar and capacity on the device first and synchronises
 * the stream for the result: a value outside 0..127 returns
 * DSOAR_ERR_INVALID_ARG and leaves the pool unchanged. */
int dsoar_sugar_admit(dsoar_sugar* sugar, uint32_t slot, uint32_t cell_offset, uint32_t side, uint64_t seed,
                      uint32_t step0, const int32_t* sugar_dev, const int32_t* cap_dev,
                      const uint8_t* occ_dev, const int32_t* a_sugar_dev, const int32_t* a_metab_dev,
                      const int32_t* a_vision_dev, const int32_t* a_age_dev, void* stream);
/* Deletes every agent of the world in `slot` and frees the slot. */
int dsoar_sugar_retire(dsoar_sugar* sugar, uint32_t slot, void* stream);
/* Canonical state of one resident world (as dsoar_sugar_read). */
int dsoar_sugar_read_world(dsoar_sugar* sugar, uint32_t slot, int32_t* sugar_dev, uint8_t* occ_dev,
                           int32_t* a_sugar_dev, int32_t* a_metab_dev, int32_t* a_vision_dev,
                           int32_t* a_age_dev, uint64_t* moves, void* stream);

/* Single-world interface: a pool of one slot covering a side x side arena.
 * Device bytes for it (0 if invalid). */
size_t dsoar_sugar_bytes(uint32_t side);
int dsoar_sugar_create(dsoar_heap* heap, uint32_t side, const dsoar_sugar_rules* rules, void* dev_mem,
                       size_t dev_bytes, dsoar_sugar** out);
int dsoar_sugar_destroy(dsoar_sugar* sugar);
/* Initial state from per-cell device arrays (side*side each): sugar and cap
 * (int32, 0..127: a cell keeps its sugar in one byte beside its occupancy
 * bit; a value outside returns DSOAR_ERR_INVALID_ARG, checked on the device
 * before anything changes, which synchronises the stream), occ (uint8, 1 = an agent
 * starts here) and the agents' sugar, metabolism, vision and age (int32, read
 * where occ).  Vision is 1..6 (the choose phase looks at most 6 cells along
 * each axis).  step0 = index of the first step (it keys the random draws).
 * The heap should be freshly reset. */
int dsoar_sugar_init(dsoar_sugar* sugar, const int32_t* sugar_dev, const int32_t* cap_dev,
                     const uint8_t* occ_dev, const int32_t* a_sugar_dev, const int32_t* a_metab_dev,
                     const int32_t* a_vision_dev, const int32_t* a_age_dev, uint32_t step0, void* stream);
/* Advances `steps` steps.  flags: DSOAR_DO_PLAIN or DSOAR_DO_PERSISTENT,
 * optionally | DSOAR_GRAPH (persistent only). */
int dsoar_sugar_step(dsoar_sugar* sugar, uint32_t steps, uint32_t flags, void* stream);
/* Canonical state per cell (device arrays, side*side each); agent fields are 0
 * where no agent is.  *moves (host, optional) receives the moves made since
 * init and synchronises the stream. */
int dsoar_sugar_read(dsoar_sugar* sugar, int32_t* sugar_dev, uint8_t* occ_dev, int32_t* a_sugar_dev,
                     int32_t* a_metab_dev, int32_t* a_vision_dev, int32_t* a_age_dev, uint32_t* moves,
                     void* stream);

/* ------------------------------------------------------------------ traffic
 * Nagel-Schreckenberg traffic (the paper's "traffic" application, Fig. 6) on
 * `roads` open single-lane roads of `length` cells: Car objects {cell, speed,
 * next speed} (type 0 of the heap: at least three 4-byte fields) advance by
 * the model's rules; cars enter at a road's first cell and are deleted when
 * they pass its last cell.  Per step: a do-all decides every car's speed
 * (accelerate, brake to the empty cells ahead, dawdle with probability
 * p_slow24 / 2^24 from hash(seed, 32, cell, t)), a second do-all moves the
 * cars, then a car enters each empty first cell with probability p_in24 /
 * 2^24 from hash(seed, 33, road, t) (the hash of the workload generator). */
typedef struct dsoar_traffic dsoar_traffic;
typedef struct {
  int32_t vmax;      /* top speed, 1 .. 8 */
  uint32_t p_slow24; /* dawdling probability * 2^24 (<= 2^24) */
  uint32_t p_in24;   /* entry probability * 2^24 (<= 2^24) */
  uint32_t reserved;
  uint64_t seed;
} dsoar_traffic_rules;
/* Device bytes for the road state (0 if roads * length is 0 or above 2^30). */
size_t dsoar_traffic_bytes(uint32_t roads, uint32_t length);
/* dev_mem: caller-owned, 256-byte aligned, at least dsoar_traffic_bytes. */
int dsoar_traffic_create(dsoar_heap* heap, uint32_t roads, uint32_t length, const dsoar_traffic_rules* rules,
                         void* dev_mem, size_t dev_bytes, dsoar_traffic** out);
int dsoar_traffic_destroy(dsoar_traffic* traffic);
/* Initial state: vel_dev[r*length + i] (int32, device) is the speed (0 ..
 * vmax) of the car in cell i of road r, or -1 for an empty cell.  step0 keys
 * the random draws of the first step.  The heap should be freshly reset. */
int dsoar_traffic_init(dsoar_traffic* traffic, const int32_t* vel_dev, uint32_t step0, void* stream);
/* Advances `steps` steps.  flags: DSOAR_DO_PLAIN or DSOAR_DO_PERSISTENT,
 * optionally | DSOAR_GRAPH (persistent only). */
int dsoar_traffic_step(dsoar_traffic* traffic, uint32_t steps, uint32_t flags, void* stream);
/* Speed per cell (-1 = empty) into vel_dev (int32, roads*length, device). */
int dsoar_traffic_read(dsoar_traffic* traffic, int32_t* vel_dev, void* stream);

/* --------------------------------------------------------------- collisions
 * Merging bodies in the plane (the paper's "collisions" application, Fig.
 * 6b): Body objects {x, y, vx, vy, ax, ay, m, id} (type 0 of the heap: at
 * least eight 4-byte fields).  Per step six do-alls: accelerations summed
 * over all ids in increasing order (m_j (p_j - p) / (r2 sqrt(r2)), r2 = |p_j -
 * p|^2 + eps2), Euler move (v += dt a, p += dt v), roots (no live body of
 * lower id within the merge radius), targets (a non-root merges into the
 * lowest-id root within the radius), merges (mass, momentum and mass-weighted
 * position added in increasing id order), removal of the merged bodies
 * (delete).  Single-precision operations, one rounding each, in that order.
 * With r2_merge = 0 no body ever merges and a step is the first two do-alls
 * only: the paper's "nbody" application (Fig. 6d). */
typedef struct dsoar_collide dsoar_collide;
typedef struct {
  float dt;       /* time step */
  float eps2;     /* softening, > 0 */
  float r2_merge; /* merge radius squared, >= 0 */
  uint32_t reserved;
} dsoar_collide_params;
/* Device bytes for n body ids (0 if n is 0 or above 2^24). */
size_t dsoar_collide_bytes(uint32_t n);
int dsoar_collide_create(dsoar_heap* heap, uint32_t n, const dsoar_collide_params* params, void* dev_mem,
                         size_t dev_bytes, dsoar_collide** out);
int dsoar_collide_destroy(dsoar_collide* collide);
/* Bodies by id from device float arrays of n entries; a body exists where
 * m_dev[id] > 0.  The heap should be freshly reset. */
int dsoar_collide_init(dsoar_collide* collide, const float* x_dev, const float* y_dev, const float* vx_dev,
                       const float* vy_dev, const float* m_dev, void* stream);
/* Advances `steps` steps.  flags: DSOAR_DO_PLAIN or DSOAR_DO_PERSISTENT,
 * optionally | DSOAR_GRAPH (persistent only). */
int dsoar_collide_step(dsoar_collide* collide, uint32_t steps, uint32_t flags, void* stream);
/* State by id into device float arrays of n entries; m = 0 for a body that
 * merged away (its other entries keep their last values). */
int dsoar_collide_read(dsoar_collide* collide, float* x_dev, float* y_dev, float* vx_dev, float* vy_dev,
                       float* m_dev, void* stream);

/* ------------------------------------------------------------------- wa-tor
 * Fish and sharks on a side x side torus (the paper's "wator" application,
 * Fig. 6h; Dewdney's rules as a synchronous step).  The heap must declare
 * Fish {int32 pos, int32 age, int32 target} as type 0 and Shark {int32 pos,
 * int32 age, int32 energy, int32 target} as type 1.  One step: fish pick an
 * empty neighbour (up, right, down, left; the k-th, k = U{0..n-1} from
 * hash(seed, 40, cell, t)), the lowest requesting cell wins, movers of age >=
 * fish_breed leave a newborn fish (new); sharks pick a neighbouring fish, or
 * with none and energy above 1 an empty neighbour (hash(seed, 41, cell, t)),
 * the lowest requesting cell wins, a shark landing on a fish eats it (energy
 * = starve) and any other loses one unit and deletes itself at 0, breeding as
 * fish do; eaten fish delete themselves.  The step index lives on the device
 * (a captured step replays correctly). */
typedef struct dsoar_wator dsoar_wator;
typedef struct {
  int32_t fish_breed;  /* >= 1 */
  int32_t shark_breed; /* >= 1 */
  int32_t starve;      /* a shark's full energy, >= 1 */
  uint32_t reserved;
  uint64_t seed;
} dsoar_wator_rules;
/* Device bytes for the sea (0 if side is 0 or side^2 above 2^30). */
size_t dsoar_wator_bytes(uint32_t side);
/* dev_mem: caller-owned, 256-byte aligned, at least dsoar_wator_bytes. */
int dsoar_wator_create(dsoar_heap* heap, uint32_t side, const dsoar_wator_rules* rules, void* dev_mem,
                       size_t dev_bytes, dsoar_wator** out);
int dsoar_wator_destroy(dsoar_wator* wator);
/* Initial sea from device int32 arrays of side^2 cells (row-major): kind (0
 * empty, 1 fish, 2 shark), age, energy (sharks, 1 .. starve).  step0 keys the
 * draws of the first step.  The heap should be freshly reset. */
int dsoar_wator_init(dsoar_wator* wator, const int32_t* kind_dev, const int32_t* age_dev, const int32_t* energy_dev,
                     uint32_t step0, void* stream);
/* Advances `steps` steps.  flags: DSOAR_DO_PLAIN or DSOAR_DO_PERSISTENT,
 * optionally | DSOAR_GRAPH (persistent only). */
int dsoar_wator_step(dsoar_wator* wator, uint32_t steps, uint32_t flags, void* stream);
/* The sea into device int32 arrays of side^2 cells: kind, age (0 where empty)
 * and energy (0 except for sharks). */
int dsoar_wator_read(dsoar_wator* wator, int32_t* kind_dev, int32_t* age_dev, int32_t* energy_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DSOAR_H */
