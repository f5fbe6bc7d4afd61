/*
 * CPU oracle for the SMMO object heap and parallel do-all
 * (DynaSOAr, arXiv 1809.07444).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential statement of
 * what the device path must compute.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * links, imports or calls it, and it shares no source with the device code.
 *
 * Parts:
 *   - hierarchical bitmap model (paper Sec. 3, Alg. 2; operations of Sec. 2.1),
 *     with a configurable container width so the paper's width-4 example
 *     (Fig. "bitmap clear example") can be replayed exactly;
 *   - sequential heap model (Sec. 2: block states; Sec. 2.2, Alg. 1), which
 *     gives the ideal (fully dense) block usage and checks state invariants;
 *   - workload references: the alloc/do-all microbenchmark, Game of Life
 *     (dense B3/S23 torus), and the Sugarscape-style agent model.
 */
#ifndef DSOAR_ORACLE_H
#define DSOAR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVELS 12
#define ORC_MAX_TYPES 8
#define ORC_FAIL (-1)

/* ------------------------------------------------------------------ RNG -- */
uint64_t orc_mix64(uint64_t z);
uint64_t orc_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b);
int32_t orc_uniform_int(uint64_t h, int32_t lo, int32_t hi);

/* ------------------------------------------------------ hierarchical bitmap */
typedef struct {
  int width;                        /* bits per container (64 in the heap) */
  int nlevels;                      /* level 0 = the bitmap itself */
  int64_t nbits[ORC_MAX_LEVELS];
  int64_t nwords[ORC_MAX_LEVELS];
  uint64_t *words[ORC_MAX_LEVELS];
  /* Every successful clear, as level * 2^40 + position, in order. */
  int64_t *trace;
  int64_t ntrace, trace_cap;
} orc_bitmap;

int orc_bm_init(orc_bitmap *b, int64_t nbits, int width, int all_set);
void orc_bm_free(orc_bitmap *b);
int orc_bm_get(const orc_bitmap *b, int level, int64_t pos);
int orc_bm_try_clear(orc_bitmap *b, int level, int64_t pos);
int orc_bm_try_set(orc_bitmap *b, int level, int64_t pos);
int orc_bm_clear(orc_bitmap *b, int level, int64_t pos);
int orc_bm_set(orc_bitmap *b, int level, int64_t pos);
int64_t orc_bm_try_find_set(const orc_bitmap *b);
int64_t orc_bm_find_clear(orc_bitmap *b);
int64_t orc_bm_consistency_violations(const orc_bitmap *b);

/* Flat handle-based wrappers for ctypes. */
void *orc_bm_new(int64_t nbits, int width, int all_set);
void orc_bm_delete(void *b);
int orc_bm_nlevels(void *b);
int64_t orc_bm_nwords(void *b, int level);
void orc_bm_words(void *b, int level, uint64_t *out);
int64_t orc_bm_trace(void *b, int64_t *out, int64_t cap);
int orc_bm_op(void *b, int op, int64_t pos, int64_t *result);

/* --------------------------------------------------- block capacities --- */
/* Sec. 2: slots per block of type t among ntypes types of sizes[] bytes.  The
 * smallest type has 64 and fixes the block size (64 of its objects); another
 * type gets the largest power of two of its objects that fits in that size,
 * at least 1. */
int32_t orc_type_capacity(const int32_t *sizes, int32_t ntypes, int32_t t);

/* ---------------------------------------------------------- subclasses --- */
/* Sec. 1.2 (class inheritance): parent[u] is the index of type u's parent, or
 * -1.  A do-all over type t runs its method on every object whose type is t
 * or inherits from t through any number of parent links.  Returns that set
 * of types as a bit mask (bit u = type u), or 0 if the parent links are not
 * a forest (a link out of range, or a cycle). */
uint32_t orc_visit_types(const int32_t *parent, int32_t ntypes, int32_t t);

/* ---------------------------------------------------------- heap model --- */
void *orc_heap_new(int32_t num_blocks, int32_t capacity, int32_t num_types);
void orc_heap_delete(void *h);
int64_t orc_heap_alloc(void *h, int32_t type);
int orc_heap_free(void *h, int64_t handle);
int64_t orc_heap_reclaim(void *h);
int64_t orc_heap_check(void *h);
void orc_heap_counts(void *h, int64_t *out);
void orc_heap_dump(void *h, uint64_t *obj_bitmap, int32_t *block_type);

/* ------------------------------------------------------------- micro ----- */
int orc_micro_run(int32_t n_init, int32_t steps, int32_t n_renew,
                  const float *x0, const float *v0,
                  const float *xs, const float *vs,
                  float *out_x, float *out_v, uint8_t *out_present,
                  int64_t *counts);

/* ------------------------------------------------------- game of life ---- */
int orc_gol_step(int32_t width, int32_t height, const uint8_t *in, uint8_t *out,
                 int64_t *counts);
int orc_gol_run(int32_t width, int32_t height, int32_t generations,
                uint8_t *grid, int64_t *per_generation_counts);

/* ---------------------------------------------------------- sugarscape --- */
typedef struct {
  int32_t max_age;
  int32_t repro_min;
  int32_t fertile_min;
  int32_t fertile_max;
} orc_sugar_rules;

/* Grids are side*side, row-major; agent arrays are indexed by cell and valid
 * where occ[cell] != 0.  counts: [births, deaths, moves] accumulated. */
int orc_sugar_run(int32_t side, int32_t steps, int32_t step0, uint64_t seed,
                  const orc_sugar_rules *rules, int32_t *sugar, const int32_t *cap,
                  uint8_t *occ, int32_t *a_sugar, int32_t *a_metab,
                  int32_t *a_vision, int32_t *a_age, int64_t *counts);

#ifdef __cplusplus
}
#endif

/* ----------------------------------------------------------- traffic ----- */
/* Nagel-Schreckenberg traffic on `roads` open roads of `length` cells, for
 * `steps` steps starting at step index step0.  vel[r*length + i] is the speed
 * of the car in cell i of road r, or -1 for an empty cell (updated in place).
 * counts[0] += cars that entered, counts[1] += cars that left. */
int orc_traffic_run(int32_t roads, int32_t length, int32_t steps, int32_t step0, uint64_t seed,
                    int32_t vmax, uint32_t p_slow24, uint32_t p_in24, int32_t *vel, int64_t *counts);


/* --------------------------------------------------------- collisions ---- */
/* Particle system with merging bodies in the plane (the paper's "collisions"
 * application, Fig. 6b).  Bodies are indexed by id; m[id] == 0 marks a body
 * that merged into another (its other entries keep their last values).
 * Updates x, y, vx, vy, m in place for `steps` steps; counts[0] += merges. */
typedef struct {
  float dt, eps2, r2_merge;
} orc_collide_params;
int orc_collide_run(int32_t n, int32_t steps, const orc_collide_params *p, float *x, float *y, float *vx,
                    float *vy, float *m, int64_t *counts);

/* ------------------------------------------------------------ wa-tor ---- */
/* Fish and sharks on a side x side torus (the paper's "wator" application,
 * Fig. 6h; Dewdney's rules in a synchronous reading).  kind[c] 0 empty, 1
 * fish, 2 shark; age[c]; energy[c] (sharks).  Updated in place for `steps`
 * steps from step index step0; counts[0..3] += fish born, sharks born, fish
 * eaten, sharks starved. */
int orc_wator_run(int32_t side, int32_t steps, int32_t step0, uint64_t seed, int32_t fish_breed,
                  int32_t shark_breed, int32_t starve, int32_t *kind, int32_t *age, int32_t *energy,
                  int64_t *counts);

#endif
