// Host-side view of the device mesh store and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "common.hpp"

namespace pm {

// Device counters (one int array, zeroed where noted by the drivers)
enum Ctr {
  C_NN_TOP = 0,     // bump pointer of the NN pool
  C_NE_TOP = 1,     // bump pointer of the NE pool
  C_ERR = 2,        // error bits (see Err)
  C_LIST_A = 3,     // generic list counters
  C_LIST_B = 4,
  C_DIRTY = 5,      // dirty rows of the current class
  C_REC = 6,        // records of the current class
  C_STAGE = 7,      // staging space handed out by the commit
  C_EVAL = 8,       // stats accumulated on the device
  C_DEFER = 9,
  C_COMMIT = 10,
  C_RELOC = 11,
  C_RECS = 12,
  C_EDGES = 13,
  C_TOTAL = 14,     // scan totals
  C_TOTAL2 = 15,
  C_JP = 16,        // 16..63: JP iteration list counters
  C_HIST = 64,      // 64..319: colour histogram (class sizes)
  C_OFF = 320,      // 320..575: class offsets
  C_CUR = 576,      // 576..831: class cursors
  C_NCOL = 832,     // number of colours
  C_PROF_JP = 833,  // profiling: active vertices visited by JP iterations
  C_PROF_DIRTY = 834,  // profiling: dirty rows committed
  C_COUNT = 896
};
constexpr int kMaxColours = 255;  // colour 0xFF marks "uncoloured"
enum Err {
  E_NN_POOL = 1,
  E_NE_POOL = 2,
  E_STAGE = 4,
  E_REC = 8,
  E_MESH_ORIENT = 16,
  E_MESH_MANIFOLD = 32,
  E_MESH_ID = 64,
  E_MESH_METRIC = 128,
  E_COLOURS = 256,
  E_ROWCAP = 512
};

struct Store {
  int V = 0, T = 0;        // slot counts
  int Vcap = 0, Tcap = 0;  // allocated slots
  double2* xy = nullptr;
  Met* met = nullptr;
  uint8_t* tag = nullptr;
  uint8_t* valive = nullptr;
  Elem* tri = nullptr;
  Hdr* hdr = nullptr;      // (nn_off, nn_cnt, ne_off, ne_cnt)
  int2* cap = nullptr;     // (nn_cap, ne_cap)
  int* nn = nullptr;
  int* ne = nullptr;
  int64_t nn_pool = 0, ne_pool = 0;  // pool capacities (entries)
  // Several independent meshes may share one store, each in its own
  // contiguous vertex range [vbase[i], vbase[i+1]) and element range
  // [tbase[i], tbase[i+1]), of which the first vused[i] / tused[i] slots are
  // in use. vmesh / tmesh give the mesh of a slot (null for a single mesh).
  int B = 1;
  int* vmesh = nullptr;
  int* tmesh = nullptr;
  int* vbase = nullptr;  // B + 1 entries (device)
  int* vused = nullptr;  // B
  int* tbase = nullptr;  // B + 1
  int* tused = nullptr;  // B
  int* mdone = nullptr;  // B flags: mesh finished refining (refinement skips it); may be null
  // per-element mean tensor, valid while topology and metrics are fixed (smoothing); may be null
  Met* emet = nullptr;
};

// local id of a vertex within its mesh (priorities are drawn per mesh)
__device__ __forceinline__ int local_id(const Store& st, int v) {
  return st.vmesh ? v - st.vbase[st.vmesh[v]] : v;
}

// launch shape used by every grid-stride kernel
constexpr int kBlock = 256;
inline int grid_for(int64_t n, int maxg = 8192) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

// ---- store.hip ----
// exclusive scan of n ints; writes the total to *total (device)
void scan_excl(const int* in, int* out, int n, int* total, int* partial, hipStream_t s);
int scan_partials_needed(int n);

void zero_ints(int* p, int n, hipStream_t s);
void fill_u8(uint8_t* p, int n, uint8_t v, hipStream_t s);
void set_int(int* p, int v, hipStream_t s);
void tri_in(const int* tri3, int T, Elem* tri, hipStream_t s);
void xy_in(const double* xy, int V, double2* out, hipStream_t s);
void tags_from_xy(const double2* xy, int V, uint8_t* tag, hipStream_t s);
void k_validate(const Store& st, int* ctr, hipStream_t s);

// rows from the element list
void build_count(const Store& st, int* ne_cnt, hipStream_t s);
void build_caps(const Store& st, const int* ne_cnt, double slack, int* nn_cap, int* ne_cap, hipStream_t s);
void set_headers(const Store& st, const int* nn_off, const int* ne_off, const int* nn_cap, const int* ne_cap,
                 hipStream_t s);
void build_fill(const Store& st, int* unused, hipStream_t s);
void build_finish(const Store& st, int* ctr, hipStream_t s);

// compaction
void flag_live_vertices(const Store& st, int* flag, hipStream_t s);
void flag_live_elements(const Store& st, int* flag, hipStream_t s);
void compact_vertices(const Store& st, const int* vmap, double2* xy2, Met* met2, uint8_t* tag2, uint8_t* va2,
                      hipStream_t s);
void compact_elements(const Store& st, const int* vmap, const int* tmap, Elem* tri2, hipStream_t s);

// refinement
void refine_mark(const Store& st, double L_up2, int* cnt, int* ctr, hipStream_t s);
// new ids inside each mesh's range: base + used + (scan - scan at the range start)
void refine_mint(const Store& st, double L_up2, const int* vscan, int* mid, hipStream_t s);
void refine_count(const Store& st, double L_up2, int* ecnt, hipStream_t s);
void refine_split(const Store& st, double L_up2, const int* mid, const int* escan, hipStream_t s);

// per-mesh sums of a 0/1 (or count) array over the used slots, from its exclusive scan
void range_sums(const int* scan, const int* src, const int* base, const int* used, int B, int* out, hipStream_t s);
// per-mesh renumbering maps: map[x] = nbase[mesh] + scan[x] - scan[base[mesh]] for flagged slots
void mesh_maps(const int* flag, const int* scan, const int* mesh, const int* base, const int* nbase, int n, int* map,
               hipStream_t s);
// mesh index of every slot of the ranges given by base (B + 1 entries)
void fill_mesh_ids(const int* base, int B, int n, int* mesh, hipStream_t s);

void export_tri(const Store& st, int* tri3, uint8_t* talive, hipStream_t s);

// ---- ops.hip ----
struct Round {
  uint64_t sseed;      // stream seed of this round's priorities
  uint64_t* key;       // per vertex: (priority, local id) of the active vertices
};

struct Commit {
  int* dirty;      // V ints, 0 when clean
  int* dlist;      // dirty rows of the class
  int* pend;       // V ints: queued addition weight per row
  int* dbase;      // V ints: staging base per row
  int* rec_row;    // queued additions
  int* rec_val;
  int* rec_off;
  int rec_cap;
  int* stage;
  int64_t stage_cap;
  uint8_t* nxt;    // next-round flags
};

struct OpArgs {
  const uint8_t* act;
  const uint8_t* col;
  int cls;
  Round rd;
  double L_low2, qmin2;
};

void set_flags(const int* list, int n, uint8_t* flag, uint8_t val, hipStream_t s);
// mode: 0 colour (active flags or all live), 1 coarsen, 2 swap, 3 smooth
// selected vertices in ascending order; flag/pos: V ints, partial: scan scratch
void select_vertices(const Store& st, int mode, double L_low2, const uint8_t* active, uint8_t* nxt, int* out,
                     int* n, int* flag, int* pos, int* partial, hipStream_t s);
void jp_init(const Store& st, const int* A, int n, uint8_t* col, uint8_t* act, Round rd, hipStream_t s);
// one JP iteration over *nU entries of U (grid sized for nmax >= *nU)
void jp_step(const Store& st, const int* U, const int* nU, int nmax, int* U2, int* nU2, const uint8_t* act,
             uint8_t* col, Round rd, int* ctr, hipStream_t s);
// stable class lists; tab/tabscan: 256 * ceil(n/256) ints each
void class_lists(const int* A, int n, const uint8_t* col, int* ctr, int* out, int* tab, int* tabscan, int* partial,
                 hipStream_t s);
void colour_out(const Store& st, const uint8_t* act, const uint8_t* col, int* out, hipStream_t s);

// variant 0: one thread per member; 1: a group of 8 lanes per member
void collapse_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, int variant,
                    hipStream_t s);
void flip_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, hipStream_t s);
void smooth_class(const Store& st, const int* list, int n, int kind, int* ctr, int variant, hipStream_t s);
void commit_rows(const Store& st, Commit cm, int* ctr, int vmax, hipStream_t s);

void quality_sum(const Store& st, double* psum, double* pmin, int nparts, double* out2, hipStream_t s);
void quality_adjoint(const Store& st, double* dQdx, double* dQdM, hipStream_t s);
void quality_per_mesh(const Store& st, double* out, hipStream_t s);
void element_metrics(const Store& st, Met* out, hipStream_t s);
void fp64_probe(const double* a, const double* b, int n, double* q, double* r, hipStream_t s);

}  // namespace pm
