/* pm3: tetrahedral meshes of the unit cube, the paper's extrusion of the method
 * to three dimensions (arXiv:1505.04694, Sec. 4: coarsening, refinement and
 * smoothing on tetrahedra; swaps are not parallelised there and not offered
 * here). Same round structure as the 2D path (include/pm.h): rounds of
 * Jones-Plassmann colour classes (Sec. 3.2) processed as independent sets,
 * re-validated against the current graph, each class's operations applied by
 * one kernel, the touched neighbourhood carried to the next round (Sec. 2.4.5).
 *
 * Conventions are those of pm.h: statuses, stream ordering, pm_options (the
 * fields read here: L_low2, L_up2, q_min, seed (at creation), sweep,
 * coarsen_rounds, refine_passes, smooth_sweeps), pm_stats slots. One handle is
 * not thread-safe.
 *
 * Geometry (Sec. 2.2 read for tetrahedra): a vertex metric is a 3x3 SPD
 * tensor stored as (m00, m01, m02, m11, m12, m22); an edge's tensor is the
 * mean of its end points', an element's the mean of its four vertices' in
 * stored order. Element quality is the mean ratio
 * q = 12 (3 sqrt(det M) |K|)^(2/3) / (sum of the six squared metric edge
 * lengths), 1 for the regular tetrahedron with unit metric edges; decisions
 * compare q^3 = 432 det(M) D^2 / S^3 (D = 6 |K|) with q_min^3. Elements are
 * positively oriented and stored with the smallest id first (an even
 * permutation of the input order), the other three rotated so that the
 * smallest of them comes second. Boundary tags are 6 bits (x = 0, x = 1,
 * y = 0, y = 1, z = 0, z = 1). */
#ifndef PM3_H
#define PM3_H
#include <stddef.h>
#include <stdint.h>

#include "pm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm3_mesh pm3_mesh;

typedef struct {
  const void* xyz;     /* V x 3 double                                          */
  const void* tet;     /* T x 4 int32, positively oriented                      */
  const void* metric;  /* V x 6 double: m00, m01, m02, m11, m12, m22            */
  const void* tags;    /* V uint8, or NULL: tags from exact coordinates 0 and 1  */
  int64_t V, T;
  int32_t mem_kind;    /* PM_MEM_HOST or PM_MEM_DEVICE for all four arrays      */
} pm3_mesh_desc;

/* Creates a handle from a copy of the arrays (the caller keeps ownership).
 * Checks every element for ids in range and distinct and a positive volume,
 * every vertex metric for positive definiteness: PM_E_MESH otherwise.
 * o: NULL for defaults; the seed is fixed here. stream: a hipStream_t or NULL. */
pm_status pm3_mesh_create(const pm3_mesh_desc* d, const pm_options* o, void* stream, pm3_mesh** out);
pm_status pm3_mesh_destroy(pm3_mesh* m);
/* slot counts (dead slots included until the next compaction) */
pm_status pm3_mesh_sizes(const pm3_mesh* m, int64_t* V, int64_t* T);
/* Copies the mesh out (arrays sized by pm3_mesh_sizes; any may be NULL),
 * host or device pointers per mem_kind. valive/talive receive 1 for live slots. */
pm_status pm3_mesh_export(pm3_mesh* m, double* xyz, int32_t* tet, double* metric, uint8_t* tags, uint8_t* valive,
                          uint8_t* talive, int32_t mem_kind);
/* Adjacency rows as host CSR (sorted ids; nn_off/ne_off hold V+1 entries);
 * call with NULL arrays first for the totals. */
pm_status pm3_mesh_rows(pm3_mesh* m, int64_t* nn_total, int64_t* ne_total, int64_t* nn_off, int32_t* nn,
                        int64_t* ne_off, int32_t* ne);

/* Jones-Plassmann colouring (Sec. 3.2) of the subgraph induced by the active
 * vertices (V host bytes, NULL = every live vertex) with priorities from the
 * handle's seed and ctx; colour_out: V host int32 (-1 inactive) or NULL. */
pm_status pm3_colour(pm3_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out, int32_t* ncolours);

/* Coarsening (Sec. 2.4.1): rounds of edge collapses over colour classes until
 * no vertex has a short edge it may collapse along, or o->coarsen_rounds. A
 * vertex v collapses onto a neighbour u on every boundary face v lies on,
 * with L^2 < L_low2, candidates in ascending (L^2, u), the first whose
 * re-pointed elements all keep a positive volume and q^3 >= q_min^3; v's
 * elements holding u die. Live vertices and elements are renumbered stably
 * at the end. PM_W_NOT_CONVERGED at the round cap (the mesh is valid). */
pm_status pm3_coarsen(pm3_mesh* m, const pm_options* o, pm_stats* st);

/* Refinement (Sec. 2.4.2): passes until no edge has L^2 > L_up2, or
 * o->refine_passes. Every long edge splits at its midpoint (edge-mean
 * metric, the AND of its end tags); new vertex ids follow the (min id, max id)
 * order of the split edges. An element with split edges is bisected along
 * them one at a time in one global order (larger L^2 first, ties by (min id,
 * max id)), children depth first, the child holding the edge's smaller id
 * first; the first leaf keeps the element's id, the others take new ids in
 * element order. Two elements sharing a face cut it identically, so the mesh
 * stays conforming. */
pm_status pm3_refine(pm3_mesh* m, const pm_options* o, pm_stats* st);

/* Smoothing (Sec. 2.4.4): o->smooth_sweeps coloured sweeps over interior
 * vertices; the Laplacian in the metric p = x_v + G^-1 r (G the sum of the
 * edge tensors over NN(v), r the sum of M_vj (x_j - x_v), in ascending
 * neighbour order, G^-1 by its adjugate), kept when every element keeps a
 * positive volume and the patch minimum of q^3 does not drop. */
pm_status pm3_smooth(pm3_mesh* m, const pm_options* o, pm_stats* st);

/* Sum and minimum of the element quality q over live elements (host scalars). */
pm_status pm3_quality(pm3_mesh* m, double* Q, double* qmin);

/* Message for the last non-OK status on this handle. */
const char* pm3_last_error(const pm3_mesh* m);

#ifdef __cplusplus
}
#endif
#endif
