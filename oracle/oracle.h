/*
 * CPU oracle for thread-parallel anisotropic mesh adaptation
 * (Rokos, Gorman, Jensen, Kelly, "Thread Parallelism for Highly Irregular
 * Computation in Anisotropic Mesh Adaptation", arXiv:1505.04694).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, serial FP64 definition of
 * what the adaptation path computes, used by the tests, by the smoke check and
 * by the benchmark's CPU-baseline leg. The product path never loads it, and it
 * shares no code with the HIP library.
 *
 * Every operation runs the paper's round structure literally: colour the
 * active vertices (Section 3.2), take the colour classes one after another as
 * independent sets, apply each member's operation (Section 2.4), and make the
 * adjacency lists reflect every change before the next class starts (the
 * deferred update of Section 3.3, which in a serial program is an immediate
 * update). Worklists for the next round collect the touched vertices
 * (Section 2.4.5, Section 3.4).
 *
 * Parity notes: results are sets (rows are sorted id sets, elements are
 * stored counter-clockwise with the smallest id first), so the order in which
 * a class's members are applied does not change the result; the orc_* calls
 * take a permutation seed to test exactly that.
 */
#ifndef PM_ORACLE_H
#define PM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_mesh orc_mesh;

/* element quality functionals (Sec. 2.2): the mean ratio
 * q = 4 sqrt(3) sqrt(det M) A / sum of squared metric edge lengths, and
 * Vasilevskii's functional with its size factor */
enum { ORC_QUALITY_MEAN_RATIO = 0, ORC_QUALITY_VASILEVSKII = 1 };

/* Algorithm 1's phases (loop state of orc_adapt) */
enum { ORC_PHASE_COARSEN = 1, ORC_PHASE_SWAP = 2, ORC_PHASE_REFINE = 3, ORC_PHASE_SMOOTH = 4, ORC_PHASE_DONE = 5 };

/* stats slots written by the phase calls (int64[ORC_NSTATS]) */
enum {
  ORC_ROUNDS = 0,      /* rounds (coarsen/swap), passes (refine), sweeps (smooth) */
  ORC_COLOURED = 1,    /* vertices coloured, summed over colourings           */
  ORC_EVALUATED = 2,   /* members evaluated (after re-validation)              */
  ORC_DEFERRED = 3,    /* members deferred by re-validation                    */
  ORC_COMMITTED = 4,   /* collapses / splits / flips / accepted moves          */
  ORC_COLOURS = 5,     /* colours used, summed over colourings                 */
  ORC_EDGES = 6,       /* edges tested by refinement                           */
  ORC_CONVERGED = 7,   /* 1 if the phase stopped because no work was left      */
  ORC_NEWV = 8,        /* vertices created                                     */
  ORC_NEWT = 9,        /* elements created                                     */
  ORC_NSTATS = 16
};

/* Copies the inputs. tags may be NULL (unit-square tags from exact
 * coordinates). Returns NULL on invalid input. */
orc_mesh* orc_create(int64_t V, int64_t T, const double* xy, const int32_t* tri,
                     const double* metric, const uint8_t* tags, uint64_t seed);
void orc_destroy(orc_mesh* m);
/* the functional every decision, smoothing step and orc_quality uses (the
 * mean ratio by default); returns -1 for an unknown kind */
int32_t orc_set_quality(orc_mesh* m, int32_t kind);
/* slot counts (dead slots included until compaction) */
void orc_sizes(const orc_mesh* m, int64_t* V, int64_t* T);
/* raw export of all slots; any pointer may be NULL */
void orc_export(const orc_mesh* m, double* xy, int32_t* tri, double* metric, uint8_t* tags,
                uint8_t* valive, uint8_t* talive);
/* total row lengths, then rows as CSR (off has V+1 entries) */
void orc_row_totals(const orc_mesh* m, int64_t* nn_total, int64_t* ne_total);
void orc_export_rows(const orc_mesh* m, int64_t* nn_off, int32_t* nn, int64_t* ne_off, int32_t* ne);
void orc_set_xy(orc_mesh* m, int32_t v, double x, double y);
void orc_set_metric(orc_mesh* m, int32_t v, double a, double b, double c);

/* SplitMix64 (Steele, Lea, Flood 2014): the i-th output of the generator
 * seeded with s, and the uint32 vertex priority built from it. */
uint64_t orc_splitmix(uint64_t s, uint64_t i);
uint32_t orc_prio(uint64_t seed, uint32_t ctx, uint32_t id);

/* Colour the subgraph induced by the active vertices (NULL = all live).
 * colour_out: V slots, -1 for inactive. Returns the number of colours. */
int32_t orc_colour(orc_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out);

/* Per-class hook for property tests: phase, round (sweep for smoothing),
 * class, stage (0 = before the class's operations, 1 = after their commit). */
typedef void (*orc_hook)(void* user, int32_t phase, int32_t round, int32_t cls, int32_t stage);
void orc_set_hook(orc_mesh* m, orc_hook hook, void* user);
/* members of the class the hook is called for (after re-validation);
 * returns the count, writes at most cap ids */
int64_t orc_class_members(const orc_mesh* m, int32_t* out, int64_t cap);
/* the same class before re-validation (ascending ids) */
int64_t orc_class_whole(const orc_mesh* m, int32_t* out, int64_t cap);
/* 0 = members in ascending id; otherwise a seeded shuffle of each class */
void orc_set_order_seed(orc_mesh* m, uint64_t order_seed);

/* Phases. Return 0 on success, 1 when a round/pass cap was hit, <0 on error. */
int32_t orc_coarsen(orc_mesh* m, int32_t sweep, double L_low2, double q_min,
                    int32_t max_rounds, int64_t* stats);
int32_t orc_refine(orc_mesh* m, double L_up2, int32_t max_passes, int64_t* stats);
int32_t orc_swap(orc_mesh* m, int32_t sweep, int32_t max_rounds, int64_t* stats);
/* kind 0 = Laplacian in metric, 1 = gradient of the quality functional,
 * 2 = min-max: ascent on the patch's worst quality */
int32_t orc_smooth(orc_mesh* m, int32_t sweep, int32_t kind, int32_t sweeps, int64_t* stats);
/* stable renumbering of live vertices and elements */
void orc_compact(orc_mesh* m);

/* Algorithm 1 (Sec. 2.3): repeat coarsen, swap, refine until an iteration
 * changes nothing or max_iterations have run, then smooth once. Iteration i
 * uses sweep index i, the final smoothing sweep index 0. The loop state is
 * kept in the mesh: with max_phases > 0 at most that many phases run and the
 * call returns 2 at a resume point; 0 when the procedure has finished. Stats:
 * the phases' counters summed, ORC_ROUNDS = iterations completed,
 * ORC_CONVERGED = 1 if an iteration changed nothing. */
int32_t orc_adapt(orc_mesh* m, int32_t max_iterations, int32_t max_phases, int32_t smooth_kind,
                  int32_t smooth_sweeps, double L_low2, double L_up2, double q_min, int32_t coarsen_rounds,
                  int32_t swap_rounds, int32_t refine_passes, int64_t* stats);
void orc_get_context(const orc_mesh* m, int32_t* iteration, int32_t* phase, int32_t* changed);
void orc_set_context(orc_mesh* m, int32_t iteration, int32_t phase, int32_t changed);

/* Quality functional Q = sum of mean-ratio qualities; optional adjoint.
 * dQdx: V x 2, dQdM: V x 3 (stored entries m00, m01, m11). */
void orc_quality(const orc_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM);
/* per-element quality (T slots, 0 for dead) */
void orc_element_quality(const orc_mesh* m, double* q);
/* Q_v: sum of q over the elements around v */
double orc_patch_quality(const orc_mesh* m, int32_t v);

/* ---- tetrahedral meshes of the unit cube (Sec. 4's extrusion to 3D) ----------
 * Coarsening, refinement and Laplacian smoothing in the metric; no swaps.
 * xyz: V x 3; tet: T x 4 ids, positively oriented; metric: V x 6 entries
 * (m00, m01, m02, m11, m12, m22); tags: 6 bits (x = 0, x = 1, y = 0, y = 1,
 * z = 0, z = 1) or NULL to derive them from exact coordinates. */
typedef struct orc3_mesh orc3_mesh;
orc3_mesh* orc3_create(int64_t V, int64_t T, const double* xyz, const int32_t* tet, const double* metric,
                       const uint8_t* tags, uint64_t seed);
void orc3_destroy(orc3_mesh* m);
void orc3_sizes(const orc3_mesh* m, int64_t* V, int64_t* T);
void orc3_export(const orc3_mesh* m, double* xyz, int32_t* tet, double* metric, uint8_t* tags, uint8_t* valive,
                 uint8_t* talive);
void orc3_row_totals(const orc3_mesh* m, int64_t* nn_total, int64_t* ne_total);
void orc3_export_rows(const orc3_mesh* m, int64_t* nn_off, int32_t* nn, int64_t* ne_off, int32_t* ne);
void orc3_set_xyz(orc3_mesh* m, int32_t v, double x, double y, double z);
void orc3_set_hook(orc3_mesh* m, orc_hook hook, void* user);
int64_t orc3_class_members(const orc3_mesh* m, int32_t* out, int64_t cap);
int64_t orc3_class_whole(const orc3_mesh* m, int32_t* out, int64_t cap);
int32_t orc3_colour(orc3_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out);
int32_t orc3_coarsen(orc3_mesh* m, int32_t sweep, double L_low2, double q_min, int32_t max_rounds, int64_t* stats);
int32_t orc3_refine(orc3_mesh* m, double L_up2, int32_t max_passes, int64_t* stats);
int32_t orc3_smooth(orc3_mesh* m, int32_t sweep, int32_t sweeps, int64_t* stats);
/* sum and minimum of the element quality (live elements) */
void orc3_quality(const orc3_mesh* m, double* Q, double* qmin);
void orc3_element_quality(const orc3_mesh* m, double* q);

#ifdef __cplusplus
}
#endif
#endif
