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
  C_TOUCH = 5,      // rows rebuilt in the current round (small rounds)
  C_STAGE = 7,      // fallback staging space handed out by the commit
  C_EVAL = 8,       // 8..13: stats, summed from the stripes (same order as the S_ slots)
  C_DEFER = 9,
  C_COMMIT = 10,
  C_RELOC = 11,
  C_ROWS = 12,
  C_EDGES = 13,
  C_TOTAL = 14,     // scan totals
  C_TOTAL2 = 15,
  C_JP = 16,        // JP: vertices still waiting after the last iteration (summed)
  C_CWIDE = 17,     // class lists: the call number of the last list with a colour past the narrow table
  C_FAILEP = 18,    // smallest commit epoch whose rows ran out of pool or staging room (INT_MAX: none)
  // device-driven small rounds (the kernels decide, the host reads back every few rounds)
  C_DROUND = 19,    // the round in progress
  C_DEPOCH = 20,    // the next commit epoch
  C_DEPOCH0 = 21,   // the first epoch of the last round run
  C_DMARK = 22,     // the selection stamp last used
  C_DSTOP = 23,     // 1: no further round (list empty, round cap, or a selection that declined)
  C_ACC_COL = 24,   // vertices coloured, colours and colouring iterations of the rounds run
  C_ACC_NCOL = 25,
  C_ACC_IT = 26,
  C_HIST = 64,      // 64..319: colour histogram (class sizes)
  C_OFF = 320,      // 320..575: class offsets
  C_CUR = 576,      // 576..831: class cursors
  C_NCOL = 832,     // number of colours
  C_PROF_JP = 833,  // profiling: active vertices visited by JP iterations (summed)
  C_PROF_ROWS = 834,  // profiling: rows rebuilt by the commit (summed)
  C_PROF_OPS = 835,   // profiling: committed operations whose rows the commit kernels rebuilt (summed)
  C_STRIPE = 1024,  // kStripes stripes of kStripeW ints, one 128-byte line each
  C_COUNT = 1024 + 64 * 32
};
// Counters that many wavefronts bump are striped: a wavefront adds to the
// stripe of its index modulo kStripes, so concurrent atomics spread over 64
// cache lines instead of queueing on one; the host sums a slot over stripes.
constexpr int kStripes = 64, kStripeW = 32;
enum Slot {
  S_EVAL = 0, S_DEFER = 1, S_COMMIT = 2, S_RELOC = 3, S_ROWS = 4, S_EDGES = 5,  // stats
  S_PJP = 6, S_PROWS = 7,  // profiling units
  S_JPL = 8,               // 8..15: JP vertices left, by iteration modulo 8
  S_POPS = 16              // profiling units: operations committed by the grid-wide class kernels,
                           // whose rows the separate commit kernels rebuild
};
__device__ __forceinline__ int* stripe_ptr(int* ctr, int slot) {
  int w = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kStripes - 1));
  return ctr + C_STRIPE + w * kStripeW + slot;
}
void stripe_zero(int* ctr, int slot, int nslots, hipStream_t s);
// ctr[dst + k] = sum over stripes of slot + k, k < nslots
void stripe_sum(int* ctr, int slot, int nslots, int dst, hipStream_t s);
constexpr int kMaxColours = 255;  // colour 0xFF marks "uncoloured"
enum Err {
  E_NN_POOL = 1,
  E_NE_POOL = 2,
  E_STAGE = 4,
  E_MESH_ORIENT = 16,
  E_MESH_MANIFOLD = 32,
  E_MESH_ID = 64,
  E_MESH_METRIC = 128,
  E_COLOURS = 256,
  E_ROWCAP = 512
};
// A commit that runs out of adjacency-pool or staging room leaves some rows
// unwritten (the element list and the next-round flags stay right). Every
// later class and commit kernel then exits at once, and the host rebuilds
// the rows from the element list with more room and redoes the rest of the
// round.
constexpr int kRoomErr = E_NN_POOL | E_NE_POOL | E_STAGE;
__device__ __forceinline__ bool room_failed(const int* ctr) {
  return (__hip_atomic_load(ctr + C_ERR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kRoomErr) != 0;
}
// the same answer for every thread of the block (call it where every thread
// of the block reaches it)
__device__ __forceinline__ bool room_failed_block(const int* ctr) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = room_failed(ctr) ? 1 : 0;
  __syncthreads();
  bool f = flag != 0;
  __syncthreads();
  return f;
}
__device__ __forceinline__ void room_fail(int* ctr, int err, int epoch) {
  atomicOr(&ctr[C_ERR], err);
  atomicMin(&ctr[C_FAILEP], epoch);
}

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
  // V: coordinates, metric and tag per vertex in one line, valid while
  // vertices stay fixed (coarsening and swapping rounds); may be null
  VRec* vr = nullptr;
  // element functional of every decision and of the quality outputs:
  // 0 the mean ratio, 1 Vasilevskii's with its size factor
  int qk = 0;
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
// Round word of a vertex (one 64-bit load answers every question a neighbour
// asks during a round): priority in bits 63..32, bit 8 set while the vertex is
// active, colour in bits 7..0 (0xFF: not coloured yet). Zero = inactive.
// Keys are (priority, id); within a mesh the global id order is the local id
// order, so ties are broken by the vertex ids themselves.
constexpr uint64_t kRwAct = 1ull << 8;
__host__ __device__ __forceinline__ bool rw_beats(uint64_t rw_w, int w, uint64_t rw_v, int v) {
  uint32_t pw = (uint32_t)(rw_w >> 32), pv = (uint32_t)(rw_v >> 32);
  return pw != pv ? pw > pv : w > v;
}

struct Round {
  uint64_t sseed;      // stream seed of this round's priorities
  uint64_t* rw;        // round words
  // device-driven rounds: the stream seed of round r is seeds[r], r =
  // ctr[C_DROUND] (null: sseed above)
  const uint64_t* seeds = nullptr;
};

// Deferred update by pull: a committing member stamps its operation and
// claims the rows it changes; the commit then rebuilds every claimed row once,
// by its owner, from the row's old NE set plus what its committed neighbours
// hand over. Epochs grow by one per class, so stale stamps never match.
struct Commit {
  int epoch;
  // V: the vertex's last committed operation, (epoch, a, b, c): a collapse
  // onto u is (epoch, -(u+1), ne_off, ne_cnt) with the member's NE row, a
  // flip (epoch, t1, t2, 0) with its two elements
  int4* ops;
  uint64_t* own;   // V: row owner key, maximised: (epoch << 32) | ~member
  // V: collapses onto the vertex, (epoch << 32) | count, and the last one's
  // (member, ne_off, ne_cnt, epoch): a collapse target finds the row it
  // absorbs without reading its neighbours' records
  uint64_t* tk;
  int4* tgt;
  int* stage;      // staging for rows past the register paths
  int64_t stage_cap;
  int* touched;    // small rounds: every row rebuilt, for the list-based selection (else null)
  int touched_cap;
  uint8_t* nxt;    // next-round flags
};
__device__ __forceinline__ uint64_t own_key(int epoch, int v) {
  return ((uint64_t)(uint32_t)epoch << 32) | (uint64_t)(uint32_t)(~v);
}

struct OpArgs {
  const uint64_t* rw;
  int cls;
  Round rd;
  double L_low2, qmin2;
};

void set_flags(const int* list, int n, uint8_t* flag, uint8_t val, hipStream_t s);
void clear_round(const int* list, int n, uint64_t* rw, hipStream_t s);
// the same with the list length read from the device (*n_dev; nothing when <= 0)
void clear_round_dev(const int* list, const int* n_dev, uint64_t* rw, hipStream_t s);
// mode: 0 colour (active flags or all live), 1 coarsen, 2 swap, 3 smooth
// selected vertices in ascending order, their count to ctr[C_LIST_B];
// flag/pos: V ints, partial: scan scratch
void select_vertices(const Store& st, int mode, double L_low2, const uint8_t* active, uint8_t* nxt, int* out,
                     int* ctr, int* flag, int* pos, int* partial, hipStream_t s);
void jp_init(const Store& st, const int* A, int n, Round rd, hipStream_t s);
// round words of the n vertices of the class lists cls (class c starts at
// off[c], the device copy of the class offsets) as their colouring set them
void restore_round(const Store& st, const int* cls, int n, const int* off, int ncol, Round rd, hipStream_t s);
void dev_rounds_start(int* ctr, int r, int epoch, int mark, int stop, hipStream_t s);
// One JP iteration over a chunked list: chunk k of kJpChunk slots holds cnt[k]
// vertices at W[k * kJpChunk ...]; the first iteration reads the n entries of
// A instead. Waiting vertices are compacted in place, in order, per chunk.
constexpr int kJpChunk = 512;
// WB holds, beside each waiting vertex, the neighbour that blocked it
void jp_chunk(const Store& st, const int* A, int n, int* W, int* WB, int* cnt, bool first, Round rd, int* ctr,
              int it, hipStream_t s);
// stable class lists; tab/tabscan: 256 * ceil(n/256) ints each. cm (4,
// kClassNarrow or 256): the colours the table holds; a list with a colour of
// cm or more reports C_NCOL = -2 and is to be cut again with cm = 256. seq: a
// nonzero number no earlier call on this counter block used
constexpr int kClassNarrow = 32;
void class_lists(const int* A, int n, const uint64_t* rw, int* ctr, int* out, int* tab, int* tabscan, int* partial,
                 int cm, int seq, hipStream_t s);
void colour_out(const Store& st, const uint64_t* rw, int* out, hipStream_t s);
// next-round list of a small round from its own lists: the members A (the
// deferred ones carry the next-round flag) and the rows rebuilt, each vertex
// once (stamp array `seen`, marker `mark`); writes the count to C_LIST_B, or
// -1 when the rebuilt rows overflowed their list (then select over all slots)
// nA < 0: device-driven round (length ctr[C_LIST_B], stamp ctr[C_DMARK] + 1;
// at the end the round counter advances and C_DSTOP is raised when the list
// is empty or max_rounds is reached; nothing runs while C_DSTOP is set)
void select_small(const Store& st, int mode, double L_low2, const int* A, int nA, const int* touched, int cap,
                  uint8_t* nxt, int* seen, int mark, int max_rounds, int* out, int* ctr, hipStream_t s);
// lists up to kSmallColour entries: colouring and class lists in one block;
// writes class sizes, offsets and count like class_lists, iterations to C_TOTAL
constexpr int kSmallColour = 8192;
// WB: 2 * kSmallColour ints for the blockers of the waiting lists
// n_dev: when given, the list length is read there instead (n ignored), and a
// length outside [0, kSmallColour] leaves the list uncoloured with C_NCOL = -1
void colour_small(const Store& st, const int* A, int n, const int* n_dev, Round rd, int* W0, int* W1, int* WB,
                  int* out, int* ctr, hipStream_t s);

// lanes per member: 1 (one thread), 8 or 16
void collapse_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, int lanes,
                    hipStream_t s);
void flip_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, hipStream_t s);
// flips on groups of 16 lanes per member
void flip_class_g(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, hipStream_t s);
// lanes per vertex: 1 (one thread) or 8
void smooth_class(const Store& st, const int* list, int n, int kind, int* ctr, int lanes, hipStream_t s);
// rebuild the rows claimed by the committed members of list[0..n) (the class
// just processed, launched in the same shape); flips: members' own rows too
// chunk: class members per work-group (0: by class size)
void commit_rows(const Store& st, const int* list, int n, Commit cm, bool flips, int chunk, int* ctr, hipStream_t s);
// the same in vertex order: every row claimed in this epoch, one thread per vertex slot
void commit_sweep(const Store& st, Commit cm, bool flips, int* ctr, hipStream_t s);
// a class of at most kSmallClass members: operation and commit in one block
// (kind 0 collapse, 1 flip)
constexpr int kSmallClass = 32;
void class_small(const Store& st, const int* list, int n, OpArgs a, Commit cm, int kind, int* ctr, hipStream_t s);
// all ncol classes of a round (every one of at most kSmallClass members) in one
// block: class c with epoch cm.epoch + c, size and offset from ctr[C_HIST + c],
// ctr[C_OFF + c] (a.cls is ignored)
// ncol < 0: device-driven round (ncol = ctr[C_NCOL], epochs from C_DEPOCH,
// nothing while C_DSTOP is set)
void round_small(const Store& st, const int* cls, int ncol, OpArgs a, Commit cm, int kind, int* ctr, hipStream_t s);

void quality_sum(const Store& st, double* psum, double* pmin, int nparts, double* out2, hipStream_t s);
void quality_adjoint(const Store& st, double* dQdx, double* dQdM, hipStream_t s);
void quality_per_mesh(const Store& st, double* out, hipStream_t s);
void element_metrics(const Store& st, Met* out, hipStream_t s);
void vertex_records(const Store& st, VRec* out, hipStream_t s);
void fp64_probe(const double* a, const double* b, int n, double* q, double* r, hipStream_t s);

}  // namespace pm
