/*
 * pmesh: thread-parallel anisotropic mesh adaptation on one MI355X (gfx950).
 *
 * C ABI of the adaptation hot path after Rokos, Gorman, Jensen and Kelly,
 * "Thread Parallelism for Highly Irregular Computation in Anisotropic Mesh
 * Adaptation" (arXiv:1505.04694). The problem statement is Algorithm 1 of
 * Sec. 2.3: a piecewise-linear triangle mesh M and a node-wise metric tensor
 * field S go in, an adapted mesh comes out, through coarsening, refinement,
 * swapping and smoothing (Sec. 2.4). Each kernel runs in rounds of
 * independent sets from a vertex colouring (Sec. 3.2) and commits adjacency
 * changes with a deferred update (Sec. 3.3).
 *
 * Conventions
 *  - Every call returns a pm_status. No C++ exception crosses this boundary.
 *  - Mesh storage lives in device memory owned by the handle. Input arrays
 *    are copied; the caller keeps ownership of everything it passes.
 *  - All device work is ordered on the stream given at creation (a
 *    hipStream_t passed as void*, NULL = the null stream). A call returns
 *    after its work is complete whenever it reports host-side results
 *    (stats, Q, counts); pm_quality's gradient outputs are written on the
 *    stream and complete when the call returns.
 *  - One handle is not thread-safe; distinct handles are independent.
 *  - After an error other than PM_E_DEVICE the handle stays usable and
 *    pm_last_error() describes the failure.
 *  - Vertex data layout: xy is V x 2 doubles (x, y); metric is V x 3 doubles
 *    (m00, m01, m11) of the symmetric tensor [[m00, m01], [m01, m11]];
 *    tri is T x 3 int32 vertex ids, counter-clockwise; tags is V bytes with
 *    bit 1: x = 0, 2: x = 1, 4: y = 0, 8: y = 1 (the unit square's sides).
 */
#ifndef PMESH_PM_H
#define PMESH_PM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PM_OK = 0,
  PM_E_ARG = 1,      /* bad argument (null pointer, size, option range)        */
  PM_E_MESH = 2,     /* invalid mesh: orientation, manifoldness, ids, metric   */
  PM_E_NOMEM = 3,    /* device allocation failed                               */
  PM_E_DEVICE = 4,   /* HIP runtime error; the handle should be destroyed      */
  PM_W_NOT_CONVERGED = 5, /* round/pass cap reached; the mesh is valid         */
  PM_W_PAUSED = 6    /* pm_adapt stopped at a resume point (o->max_phases)     */
} pm_status;

enum { PM_MEM_HOST = 0, PM_MEM_DEVICE = 1 };
/* Element quality functionals (Sec. 2.2), both 1 exactly for the equilateral
 * triangle with unit edges in the metric, computed with the element's tensor
 * M = the mean of its three vertex tensors and A its Euclidean area:
 *  PM_QUALITY_MEAN_RATIO: q = 4 sqrt(3) sqrt(det M) A / (sum of the squared
 *    metric edge lengths); invariant under M -> cM, so it measures shape only;
 *  PM_QUALITY_VASILEVSKII: Vasilevskii's functional with its size factor,
 *    Q = 12 sqrt(3) sqrt(det M) A / P^2 * F(P / 3), P the metric perimeter,
 *    F(x) = (m (2 - m))^3 with m = min(x, 1/x).
 * Decisions compare the square of the value (q^2, or Q * Q rounded once) with
 * q_min^2. */
enum { PM_QUALITY_MEAN_RATIO = 0, PM_QUALITY_VASILEVSKII = 1 };

/* smoothing kinds: the Laplacian in the metric; a gradient step on the patch's
 * quality sum; min-max, an ascent step on the patch's worst quality */
enum { PM_SMOOTH_LAPLACE = 0, PM_SMOOTH_GRADIENT = 1, PM_SMOOTH_MINMAX = 2 };
/* phases of Algorithm 1 (pm_adapt's loop state, see pm_context) */
enum { PM_PHASE_COARSEN = 1, PM_PHASE_SWAP = 2, PM_PHASE_REFINE = 3, PM_PHASE_SMOOTH = 4, PM_PHASE_DONE = 5 };

typedef struct {
  const double* xy;      /* V x 2 */
  const int32_t* tri;    /* T x 3, counter-clockwise */
  const double* metric;  /* V x 3 (m00, m01, m11), symmetric positive definite */
  const uint8_t* tags;   /* V, or NULL: derived from exact coordinates 0 and 1 */
  int64_t V, T;
  int32_t mem_kind;      /* PM_MEM_HOST or PM_MEM_DEVICE for all four arrays */
} pm_mesh_desc;

/* Kernel shapes. Every choice gives bit-identical results (the tests check
 * this); they trade occupancy, latency and launch count against each other,
 * and the package's autotuner (autotune.py) picks them by measurement.
 * Zero means the default. */
typedef struct {
  int32_t op_lanes;      /* lanes per member in collapse and flip classes: 0 = 16;
                            1 (one thread per member), 8 or 16                   */
  int32_t smooth_lanes;  /* lanes per vertex in smoothing classes: 0 = 8; 1 or 8  */
  int32_t commit_chunk;  /* class members per commit work-group: 0 = by class size
                            (16, 64 or 128); 16, 32, 64 or 128                   */
  int32_t small_work;    /* 0: lists of up to 8192 vertices are coloured by one
                            work-group, and classes of up to 32 members run with
                            their commit in one launch; 1: always the grid-wide
                            kernels                                              */
  int32_t class_colours; /* colours counted by the first pass that cuts a
                            colouring into class lists: 0 = 32; 4, 8, 16, 32,
                            64, 128 or 256 (a colouring with more colours is
                            cut again from the full table)                       */
  int32_t commit_order;  /* 0: the commit of a class of at least V/64 members
                            walks the rows in vertex order, smaller classes from
                            their members; 1: always from the members; 2:
                            always in vertex order                              */
  int32_t host_rounds;   /* 0: rounds whose list is coloured by one work-group
                            and whose classes have at most 32 members run
                            device-driven (each kernel takes its sizes from
                            device counters, the host reads back every four
                            rounds); 2: the same, two rounds captured as a
                            graph that the handle keeps and replays while its
                            launch arguments are unchanged; 1: the host drives
                            every round                                         */
  int32_t reserved;      /* 0 */
} pm_tuning;

/* Device memory provider for a handle (optional: pm_options.allocator, read
 * at creation). Every device buffer the handle holds comes from
 * alloc(bytes, stream, user) and goes back through release(ptr, bytes,
 * stream, user) with the byte count it was allocated with; both are called
 * from the calling host thread with the handle's stream. Releases are stream
 * ordered: work already queued on the stream may still use a released block,
 * so the provider may hand it out again only to later work on that stream
 * (the semantics of stream-ordered caching allocators such as torch's). alloc
 * returns NULL when it cannot serve a request, and the call then fails with
 * PM_E_NOMEM. The provider must outlive the handle. Without one, the library
 * keeps its own stream-ordered block cache over hipMalloc. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*release)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} pm_allocator;

/* Thresholds are squared metric lengths. Defaults (pm_default_options):
 * L_low2 = 0.5, L_up2 = 2.0, q_min = 0.1, seed = 0, sweep = 0,
 * coarsen_rounds = 200, swap_rounds = 100, refine_passes = 32,
 * smooth_kind = PM_SMOOTH_LAPLACE, smooth_sweeps = 1, slack = 2.0,
 * pool_headroom = 3.0, max_iterations = 8, max_phases = 0, tune = zeros,
 * quality = PM_QUALITY_MEAN_RATIO, allocator = NULL. */
typedef struct {
  double L_low2;          /* collapse an edge when L^2 < L_low2                 */
  double L_up2;           /* split an edge when L^2 > L_up2                     */
  double q_min;           /* a collapse may not create an element with q < q_min */
  uint64_t seed;          /* priority seed (fixed at creation; see pm_mesh_create) */
  int32_t sweep;          /* outer sweep index, part of the priority context    */
  int32_t coarsen_rounds; /* round cap of pm_coarsen                            */
  int32_t swap_rounds;    /* round cap of pm_swap                               */
  int32_t refine_passes;  /* pass cap of pm_refine                              */
  int32_t smooth_kind;    /* PM_SMOOTH_LAPLACE or PM_SMOOTH_GRADIENT            */
  int32_t smooth_sweeps;  /* coloured sweeps of pm_smooth                       */
  double slack;           /* adjacency row capacity factor (>= 1), at creation  */
  double pool_headroom;   /* free room kept in the adjacency pools and the
                             commit's staging area, as a multiple of the live
                             entries (>= 1), at creation. A round that runs out
                             has its rows rebuilt from the element list with
                             twice the room and goes on, so results do not
                             depend on it; less room uses less device memory
                             and costs rebuilds.                                */
  int32_t max_iterations; /* pm_adapt: cap on Algorithm 1's outer iterations    */
  int32_t max_phases;     /* pm_adapt: phases to run in this call before
                             returning at a resume point; 0 = no limit          */
  pm_tuning tune;         /* kernel shapes                                      */
  int32_t quality;        /* element functional of every decision and of
                             pm_quality, fixed at creation: PM_QUALITY_MEAN_RATIO
                             or PM_QUALITY_VASILEVSKII                          */
  int32_t reserved;       /* 0                                                  */
  const pm_allocator* allocator; /* device memory provider, at creation; NULL =
                                    the library's own block cache             */
} pm_options;

/* Per-phase counters, all integers:
 * v[0] rounds (coarsen, swap), passes (refine), sweeps (smooth)
 * v[1] vertices coloured, summed over colourings
 * v[2] members evaluated after re-validation
 * v[3] members deferred by re-validation
 * v[4] committed operations: collapses, split edges, flips, accepted moves
 * v[5] colours used, summed over colourings
 * v[6] edges tested by refinement
 * v[7] 1 when the phase ran out of work (converged)
 * v[8] vertices created, v[9] elements created
 * v[10] deferred-update records committed
 * v[11] adjacency rows relocated by the commit
 * v[12] JP colouring iterations
 * v[13] rounds whose rows were rebuilt after the pools or the staging area
 *       ran out of room
 * pm_adapt sums its phases' counters, with v[0] = outer iterations run. */
typedef struct {
  int64_t v[16];
} pm_stats;
/* slots of pm_stats.v */
enum {
  PM_S_ROUNDS = 0, PM_S_COLOURED = 1, PM_S_EVALUATED = 2, PM_S_DEFERRED = 3, PM_S_COMMITTED = 4,
  PM_S_COLOURS = 5, PM_S_EDGES = 6, PM_S_CONVERGED = 7, PM_S_NEWV = 8, PM_S_NEWT = 9
};

typedef struct pm_mesh pm_mesh;

/* Fills o with the defaults listed above. */
pm_status pm_default_options(pm_options* o);

/* Builds the device store (Sec. 3.1: per-vertex adjacency lists of vertices
 * and elements) from a triangle list: slack-padded rows, each a sorted id set.
 * Validates ids, orientation (every triangle counter-clockwise with positive
 * area), manifoldness (no directed edge used twice), finite SPD metric.
 * o may be NULL (defaults); o->seed becomes the handle's priority seed.
 * stream: hipStream_t as void*. On success *out owns all device memory. */
pm_status pm_mesh_create(const pm_mesh_desc* d, const pm_options* o, void* stream, pm_mesh** out);

/* Frees the handle and all its device memory. NULL is accepted. */
pm_status pm_mesh_destroy(pm_mesh* m);

/* Current slot counts. After pm_coarsen all slots are live (the phase ends
 * with a stable renumbering); otherwise dead slots may be included. */
pm_status pm_mesh_sizes(const pm_mesh* m, int64_t* V, int64_t* T);

/* Device memory held by the handle: now, and the most at any time since it
 * was created (store, adjacency pools and phase scratch; the inputs and
 * outputs the caller owns are not counted). Either output may be NULL. */
pm_status pm_mesh_memory(const pm_mesh* m, int64_t* current_bytes, int64_t* peak_bytes);

/* Copies the live mesh out (V x 2, T x 3, V x 3, V) in slot order, which is
 * the live order after pm_coarsen. Any output may be NULL. mem_kind says
 * whether the outputs are host or device pointers; they must hold the sizes
 * reported by pm_mesh_sizes. valive/talive (host or device, may be NULL)
 * receive 1 for live slots. */
pm_status pm_mesh_export(pm_mesh* m, double* xy, int32_t* tri, double* metric, uint8_t* tags,
                         uint8_t* valive, uint8_t* talive, int32_t mem_kind);

/* Adjacency rows as host CSR: nn_off/ne_off hold V+1 entries. Call first with
 * NULL arrays to get the totals. */
pm_status pm_mesh_rows(pm_mesh* m, int64_t* nn_total, int64_t* ne_total, int64_t* nn_off, int32_t* nn,
                       int64_t* ne_off, int32_t* ne);

/* Jones-Plassmann colouring (Sec. 3.2) of the subgraph induced by the active
 * live vertices: priorities are the uint32 SplitMix64 values of
 * (handle seed, ctx, vertex id), ties by id, and a vertex takes the smallest
 * colour unused by its active neighbours of larger key (the result equals the
 * greedy colouring in descending key order). active: V bytes, host or device
 * per mem_kind, NULL = all live vertices. colour_out: V int32 (-1 inactive),
 * host or device per mem_kind, may be NULL. */
pm_status pm_colour(pm_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out,
                    int32_t* ncolours, int32_t mem_kind);

/* Coarsening (Sec. 2.4.1): rounds of edge collapses over colour classes until
 * no vertex with a short edge is left or o->coarsen_rounds is reached; ends
 * with a stable renumbering of live vertices and elements. */
pm_status pm_coarsen(pm_mesh* m, const pm_options* o, pm_stats* st);

/* Refinement (Sec. 2.4.2): passes that split every edge with L^2 > L_up2 and
 * cut elements with the 1-, 2- and 3-edge templates, until none is long or
 * o->refine_passes is reached. */
pm_status pm_refine(pm_mesh* m, const pm_options* o, pm_stats* st);

/* Swapping (Sec. 2.4.3): rounds of edge flips that raise the smaller quality
 * of the two elements, until none is left or o->swap_rounds is reached. */
pm_status pm_swap(pm_mesh* m, const pm_options* o, pm_stats* st);

/* Smoothing (Sec. 2.4.4): o->smooth_sweeps coloured sweeps over interior
 * vertices. PM_SMOOTH_LAPLACE: the Laplacian in the metric, kept if every area
 * stays positive and the patch's minimum quality does not drop;
 * PM_SMOOTH_GRADIENT: a step along the gradient of the patch's quality sum,
 * kept on the same conditions when the sum rises; PM_SMOOTH_MINMAX: a step
 * along the ascent direction of the patch's worst quality (the worst
 * element's gradient, or the nearest-to-origin point between the two worst
 * within 1%), kept when every area stays positive and the minimum rises. */
pm_status pm_smooth(pm_mesh* m, const pm_options* o, pm_stats* st);

/* Algorithm 1 (Sec. 2.3), the mesh optimisation procedure: repeat coarsen,
 * swap, refine until an outer iteration changes nothing (no collapse, flip or
 * split) or o->max_iterations iterations have run, then smooth once
 * (o->smooth_kind, o->smooth_sweeps). Iteration i runs its phases with sweep
 * index i in the priority context; the final smoothing uses sweep index 0
 * (o->sweep is ignored). The loop state lives in the handle (pm_context,
 * which starts at iteration 0, phase PM_PHASE_COARSEN): with o->max_phases > 0
 * at most that many phases run and the call returns PM_W_PAUSED at a resume
 * point, from which the next call goes on; PM_OK once the final smoothing has
 * run (further calls do nothing). A phase that stops at its round or pass cap
 * does not stop the loop. Stats: the phases' counters summed, v[0] = outer
 * iterations completed in this call, v[7] = 1 if one of them changed nothing. */
pm_status pm_adapt(pm_mesh* m, const pm_options* o, pm_stats* st);

/* Checkpoint and resume of Algorithm 1's loop state. seed: the handle's
 * priority seed; iteration: the outer iteration in progress (its sweep
 * index); phase: the next phase (PM_PHASE_*); changed: 1 if the iteration in
 * progress has changed the mesh. A checkpoint is pm_get_context plus
 * pm_mesh_export (whose arrays are in the handle's slot order); a handle
 * created from those arrays and given the context with pm_set_context
 * continues exactly as the saved handle would (pm_set_context also sets the
 * handle's priority seed). */
typedef struct {
  uint64_t seed;
  int32_t iteration;
  int32_t phase;
  int32_t changed;
  int32_t reserved;  /* 0 */
} pm_context;
pm_status pm_get_context(const pm_mesh* m, pm_context* c);
pm_status pm_set_context(pm_mesh* m, const pm_context* c);

/* Replaces the coordinates (V x 2) and/or the metric (V x 3, stored entries)
 * of every vertex slot; either pointer may be NULL; host or device memory per
 * mem_kind; sizes as reported by pm_mesh_sizes. The new values are checked as
 * pm_mesh_create checks its input (every live element counter-clockwise with
 * positive area, every metric finite and SPD); on failure the old values are
 * kept and PM_E_MESH is returned. Not for batches (PM_E_ARG). */
pm_status pm_mesh_update(pm_mesh* m, const double* xy, const double* metric, int32_t mem_kind);

/* Quality functional (Sec. 2.2): Q = sum over elements of the mean ratio
 * q = 4 sqrt(3) sqrt(det M) A / sum of squared metric edge lengths, M the mean
 * of the element's vertex tensors; qmin = the smallest q. Q and qmin are host
 * pointers (may be NULL). dQdx (V x 2) and dQdM (V x 3, stored entries) are
 * device pointers or NULL; when given, the adjoint is written there. */
pm_status pm_quality(pm_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM);

/* pm_quality for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same results as pm_quality (the same reduction, bit for bit), with no
 * allocation of any kind during the call. The reduction's partial sums go to a
 * fixed array of 2 x 2048 + 2 doubles (32 KB) inside the library, one copy
 * per device, held until the process ends; a reduction of more than 2048
 * partial sums is rejected with PM_E_ARG (pm_quality never takes more, so
 * no handle this library creates reaches it). Call it with the handle's
 * device current (else PM_E_ARG). Calls that overlap on one device, from any
 * handles or streams, race on that array; serialise them. Outputs as
 * pm_quality: Q and qmin host pointers, dQdx and dQdM device pointers, any
 * may be NULL. */
pm_status pm_quality_noalloc(pm_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM);

/* Diagnostic: computes quot[i] = a[i] / b[i] and root[i] = sqrt(a[i]) in FP64
 * on the current device (host arrays of n doubles), so a caller can check
 * that the device rounds division and square root exactly as IEEE-754 binary64
 * does; every threshold decision of the path relies on that. */
pm_status pm_fp64_selfcheck(const double* a, const double* b, int64_t n, double* quot, double* root);

/* Batches of independent meshes (Sec. 3: many small independent sets at
 * once). pm_batch_create concatenates `count` meshes (host arrays only) into
 * one store, each in its own vertex and element range with headroom for
 * refinement. The phase calls (pm_coarsen, pm_refine, pm_swap, pm_smooth,
 * pm_colour, pm_quality) then run every mesh of the batch in the same kernel
 * launches; each mesh draws priorities from its own local vertex ids, so its
 * result equals that of the same calls on a handle holding it alone. Rounds
 * advance in lockstep; stats are summed over the meshes (rounds: the maximum;
 * colours: per colouring of the whole batch). */
pm_status pm_batch_create(const pm_mesh_desc* meshes, int32_t count, const pm_options* o, void* stream,
                          pm_mesh** out);
pm_status pm_batch_count(const pm_mesh* m, int32_t* count);
/* slots of mesh i (its live mesh after pm_coarsen: all slots live) */
pm_status pm_batch_sizes(const pm_mesh* m, int32_t i, int64_t* V, int64_t* T);
/* host copies of mesh i with its own local ids; arrays sized by pm_batch_sizes */
pm_status pm_batch_export(pm_mesh* m, int32_t i, double* xy, int32_t* tri, double* metric, uint8_t* tags,
                          uint8_t* valive, uint8_t* talive);
/* per-mesh quality functional and minimum quality (host arrays of count) */
pm_status pm_batch_quality(pm_mesh* m, double* Q, double* qmin);

/* Per-kernel timing. Kernel ids for pm_profile / pm_profile_read: */
enum {
  PM_K_JP = 0,       /* Jones-Plassmann iteration; units: active vertices visited   */
  PM_K_COLLAPSE = 1, /* collapse class kernel; units: class members                 */
  PM_K_FLIP = 2,     /* flip class kernel; units: class members                     */
  PM_K_SMOOTH = 3,   /* smoothing class kernel; units: class members                */
  PM_K_COMMIT = 4,   /* deferred-update commit (three kernels); units: dirty rows   */
  PM_K_ADJOINT = 5,  /* quality adjoint; units: vertices                            */
  PM_K_QUALITY = 6,  /* quality functional; units: elements                         */
  PM_K_SELECT = 7,   /* worklist selection over all vertices; units: vertices       */
  PM_K_COUNT = 8,
  /* pm_profile_read only: the commit kernels' time and launches, with units =
   * the committed operations (collapses, flips) whose rows they rebuilt */
  PM_K_COMMIT_OPS = 8
};

/* Enables HIP-event timing (on the handle's stream) around every launch of
 * the kernels whose bit (1 << id) is set in mask; 0 disables it. Resets the
 * accumulated totals. Timing adds two event records per timed launch. */
pm_status pm_profile(pm_mesh* m, uint32_t mask);

/* Totals since pm_profile for kernel id: device milliseconds, launches and
 * units of work (see the enum). Host pointers, any may be NULL. */
pm_status pm_profile_read(pm_mesh* m, int32_t id, double* ms, int64_t* launches, int64_t* units);

/* Message for the last non-OK status on this handle (never NULL). With a NULL
 * handle: the message of the calling thread's last failed pm_mesh_create. */
const char* pm_last_error(const pm_mesh* m);

/* Library build string. */
const char* pm_version(void);

#ifdef __cplusplus
}
#endif
#endif
