// Adaptation kernels: Jones-Plassmann colouring, colour-class lists, the four
// operations (collapse, flip, smoothing; refinement lives in store.hip), the
// deferred-update commit and the quality functional with its adjoint.
//
// Round structure (Sec. 3.2-3.4): the active vertices are coloured once per
// round; the colour classes run one kernel after another. A class kernel
// re-validates each member against same-class neighbours in the current
// graph, evaluates its operation from the state left by the previous class,
// rewrites only elements the member owns, marks the adjacency rows it touches
// dirty and queues the additions those rows need. The commit then lets the
// owner of each dirty row rebuild it, so no two threads ever write one row.
#include <algorithm>
#include <atomic>

#include "kern.hpp"

namespace pm {

constexpr int kG = 8;    // lanes per vertex in the lane-group kernels
constexpr int kGC = 16;  // lanes per vertex in the lane-group collapse

__device__ __forceinline__ uint64_t key_of(const Store& st, const Round& rd, int v) {
  return vkey(rd.sseed, (uint32_t)local_id(st, v));
}
__device__ __forceinline__ void rw_put(uint64_t* rw, int v, uint64_t x) { ((volatile uint64_t*)rw)[v] = x; }

__global__ void k_clear_round(const int* __restrict__ list, int n, uint64_t* __restrict__ rw) {
  for (int i = gtid(); i < n; i += gstride()) rw[list[i]] = 0;
}
void clear_round(const int* list, int n, uint64_t* rw, hipStream_t s) {
  if (n > 0) k_clear_round<<<grid_for(n), kBlock, 0, s>>>(list, n, rw);
}
__global__ void k_clear_round_dev(const int* __restrict__ list, const int* n_dev, uint64_t* __restrict__ rw) {
  int n = *n_dev;
  for (int i = gtid(); i < n; i += gstride()) rw[list[i]] = 0;
}
void clear_round_dev(const int* list, const int* n_dev, uint64_t* rw, hipStream_t s) {
  k_clear_round_dev<<<grid_for(kSmallColour), kBlock, 0, s>>>(list, n_dev, rw);
}

// ---- flags and lists -----------------------------------------------------------------
__global__ void k_set_flags(const int* __restrict__ list, int n, uint8_t* __restrict__ flag, uint8_t val) {
  for (int i = gtid(); i < n; i += gstride()) flag[list[i]] = val;
}
void set_flags(const int* list, int n, uint8_t* flag, uint8_t val, hipStream_t s) {
  if (n > 0) k_set_flags<<<grid_for(n), kBlock, 0, s>>>(list, n, flag, val);
}

__device__ bool has_candidate(const Store& st, int v, double L_low2) {
  Hdr h = st.hdr[v];
  double2 pv = st.xy[v];
  Met mv = st.met[v];
  uint8_t tv = st.tag[v];
  for (int j = 0; j < h.y; ++j) {
    int u = st.nn[h.x + j];
    if (tv & ~st.tag[u]) continue;
    if (len2(pv, mv, st.xy[u], st.met[u]) < L_low2) return true;
  }
  return false;
}

// mode: 0 colour (active flags or all live), 1 coarsen (has a short edge),
// 2 swap (all live), 3 smooth (live interior)
__device__ __forceinline__ bool want(const Store& st, int v, int mode, double L_low2, const uint8_t* active) {
  if (!st.valive[v]) return false;
  switch (mode) {
    case 0: return active ? active[v] != 0 : true;
    case 1: return has_candidate(st, v, L_low2);
    case 2: return true;
    default: return st.tag[v] == 0;
  }
}

// flag[v] = 1 for every vertex v with (nxt == null or nxt[v]) and want(v); clears nxt.
// After a commit that ran out of room (the rows are being rebuilt) it selects
// nothing and leaves the flags for the selection that follows the rebuild.
__global__ void k_select_flags(Store st, int mode, double L_low2, const uint8_t* __restrict__ active,
                               uint8_t* __restrict__ nxt, int* __restrict__ flag, const int* ctr) {
  if (nxt && room_failed(ctr)) {
    for (int v = xtid(); v < st.V; v += gstride()) flag[v] = 0;
    return;
  }
  for (int v = xtid(); v < st.V; v += gstride()) {
    bool on = nxt ? nxt[v] != 0 : true;
    if (nxt && on) nxt[v] = 0;
    flag[v] = (on && want(st, v, mode, L_low2, active)) ? 1 : 0;
  }
}
__global__ void k_select_scatter(int V, const int* __restrict__ flag, const int* __restrict__ pos,
                                 int* __restrict__ out) {
  for (int v = gtid(); v < V; v += gstride())
    if (flag[v]) out[pos[v]] = v;
}
// the selected vertices in ascending id order (an ordered compaction), so
// that lists and the colour classes cut from them follow the mesh's layout
void select_vertices(const Store& st, int mode, double L_low2, const uint8_t* active, uint8_t* nxt, int* out,
                     int* ctr, int* flag, int* pos, int* partial, hipStream_t s) {
  int* n = ctr + C_LIST_B;
  k_select_flags<<<grid_for(st.V), kBlock, 0, s>>>(st, mode, L_low2, active, nxt, flag, ctr);
  scan_excl(flag, pos, st.V, n, partial, s);
  k_select_scatter<<<grid_for(st.V), kBlock, 0, s>>>(st.V, flag, pos, out);
}

// ---- Jones-Plassmann colouring (Sec. 3.2) ------------------------------------------------
__global__ void k_jp_init(Store st, const int* __restrict__ A, int n, Round rd) {
  for (int i = gtid(); i < n; i += gstride()) {
    int v = A[i];
    uint64_t prio = key_of(st, rd, v) >> 32;
    rd.rw[v] = (prio << 32) | kRwAct | 0xFFull;
  }
}
void jp_init(const Store& st, const int* A, int n, Round rd, hipStream_t s) {
  if (n > 0) k_jp_init<<<grid_for(n), kBlock, 0, s>>>(st, A, n, rd);
}

// start of device-driven rounds: round r, next epoch, last stamp; the
// accumulated statistics cleared
__global__ void k_dev_rounds_start(int* ctr, int r, int epoch, int mark, int stop) {
  if (threadIdx.x == 0) {
    ctr[C_DROUND] = r;
    ctr[C_DEPOCH] = epoch;
    ctr[C_DEPOCH0] = epoch;
    ctr[C_DMARK] = mark;
    ctr[C_DSTOP] = stop;
    ctr[C_ACC_COL] = 0;
    ctr[C_ACC_NCOL] = 0;
    ctr[C_ACC_IT] = 0;
  }
}
void dev_rounds_start(int* ctr, int r, int epoch, int mark, int stop, hipStream_t s) {
  k_dev_rounds_start<<<1, 64, 0, s>>>(ctr, r, epoch, mark, stop);
}

// round words of a coloured list again, from its class lists (the list is
// the classes' union, class c holds the vertices of colour c)
__global__ void k_restore_round(Store st, const int* __restrict__ cls, int n, const int* __restrict__ off, int ncol,
                                Round rd) {
  for (int i = gtid(); i < n; i += gstride()) {
    int c = 0;
    while (c + 1 < ncol && off[c + 1] <= i) ++c;
    int v = cls[i];
    uint64_t prio = key_of(st, rd, v) >> 32;
    rd.rw[v] = (prio << 32) | kRwAct | (uint64_t)c;
  }
}
void restore_round(const Store& st, const int* cls, int n, const int* off, int ncol, Round rd, hipStream_t s) {
  if (n > 0) k_restore_round<<<grid_for(n), kBlock, 0, s>>>(st, cls, n, off, ncol, rd);
}

// A vertex is ready once every active neighbour of larger key has a colour;
// it then takes the smallest colour none of them has. Colours read while a
// neighbour is being written are either unset (not ready yet) or final, so
// the result does not depend on timing. Returns false while v must wait.
// blocker: in, a neighbour that kept v waiting before (or -1); out, the
// neighbour that keeps it waiting now. While that neighbour has no colour, v
// cannot be ready, and one load settles the visit.
// The round words are read through the caches. At a launch's start
// every colour set before it is visible; a colour set during the launch may
// read as unset, which only makes v wait (priorities and active bits do not
// change during the colouring), and the vertex of largest key still waiting
// is ready at every launch, so each chunked launch makes progress. The
// one-block colouring runs to completion in one launch: its iterations are
// separated by block barriers, and a work-group's waves share one CU's
// vector L1, which the CU's own stores write through, so every iteration
// sees the colours of the ones before it (its loop is bounded regardless).
__device__ bool jp_try(const Store& st, int v, const Round& rd, int* ctr, int& blocker) {
  constexpr int B = 8;  // neighbours fetched side by side
  const uint64_t* rw = rd.rw;
  if (blocker >= 0 && (rw[blocker] & 0xFF) == 0xFF) return false;
  uint64_t rv = rw[v];
  Hdr h = st.hdr[v];
  uint64_t used = 0;
  bool big = false;
  for (int j0 = 0; j0 < h.y; j0 += B) {
    int w[B];
    uint64_t x[B];
    row8(st.nn, h.x + j0, h.y - j0, w);
#pragma unroll
    for (int q = 0; q < B; ++q) x[q] = w[q] >= 0 ? rw[w[q]] : 0ull;
    int wait = -1;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (!(x[q] & kRwAct) || !rw_beats(x[q], w[q], rv, v)) continue;
      int c = (int)(x[q] & 0xFF);
      if (c == 0xFF) wait = wait < 0 ? w[q] : wait;
      else if (c < 64) used |= 1ull << c;
      else big = true;
    }
    if (wait >= 0) {
      blocker = wait;
      return false;
    }
  }
  int c;
  if (~used != 0ull && !big) {
    c = __ffsll((unsigned long long)~used) - 1;
  } else {
    // slow path: colours beyond 63 among the neighbours
    c = 0;
    for (;;) {
      bool taken = false;
      for (int j = 0; j < h.y && !taken; ++j) {
        int w = st.nn[h.x + j];
        uint64_t x = rw[w];
        if (!(x & kRwAct) || !rw_beats(x, w, rv, v)) continue;
        taken = (int)(x & 0xFF) == c;
      }
      if (!taken) break;
      ++c;
    }
  }
  if (c >= kMaxColours) {
    atomicOr(&ctr[C_ERR], E_COLOURS);
    c = kMaxColours - 1;
  }
  rw_put(rd.rw, v, (rv & ~0xFFull) | (uint64_t)c);
  return true;
}

// One block per chunk; each thread takes kJpItems entries (item r of thread
// t is entry r * kBlock + t). The waiting vertices are packed to the front of
// the chunk in their old order: every read happens before the block barrier,
// every write after it, so the compaction can run in place. One atomic per
// chunk (on a stripe) counts what is left.
constexpr int kJpItems = kJpChunk / kBlock;
constexpr int kJpLocal = 3;  // passes per launch over a chunk that makes progress
__global__ void __launch_bounds__(256) k_jp_chunk(Store st, const int* __restrict__ A, int n, int* W, int* WB,
                                                  int* __restrict__ cnt, int first, Round rd, int* ctr, int slot,
                                                  int next_slot) {
  __shared__ int wtot[kJpItems][kBlock / kWave];
  int kb = xcd_block();
  if (blockIdx.x == 0 && threadIdx.x < kStripes) ctr[C_STRIPE + threadIdx.x * kStripeW + next_slot] = 0;
  int m = first ? min(kJpChunk, n - kb * kJpChunk) : cnt[kb];
  if (m <= 0) {
    if (first && threadIdx.x == 0) cnt[kb] = 0;
    return;
  }
  const int* in = (first ? A : W) + (size_t)kb * kJpChunk;
  const int* inb = WB + (size_t)kb * kJpChunk;
  int vv[kJpItems], bl[kJpItems];
#pragma unroll
  for (int r = 0; r < kJpItems; ++r) {
    int i = r * kBlock + (int)threadIdx.x;
    vv[r] = i < m ? in[i] : -1;
    bl[r] = (i < m && !first) ? inb[i] : -1;
  }
  bool keep[kJpItems];
  int tries = 0;  // this thread's vertex visits, for the profile's unit count
  bool moved = false;
#pragma unroll
  for (int r = 0; r < kJpItems; ++r) {
    keep[r] = vv[r] >= 0 && !jp_try(st, vv[r], rd, ctr, bl[r]);
    moved |= vv[r] >= 0 && !keep[r];
    tries += vv[r] >= 0 ? 1 : 0;
  }
  // more passes over the chunk's waiting vertices while the chunk makes
  // progress: chains of neighbours inside the chunk resolve in one launch
  for (int pass = 1; pass < kJpLocal; ++pass) {
    bool waiting = false;
#pragma unroll
    for (int r = 0; r < kJpItems; ++r) waiting |= keep[r];
    if (!__syncthreads_or(moved && waiting)) break;
    moved = false;
#pragma unroll
    for (int r = 0; r < kJpItems; ++r)
      if (keep[r]) {
        ++tries;
        keep[r] = !jp_try(st, vv[r], rd, ctr, bl[r]);
        moved |= !keep[r];
      }
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) tries += __shfl_xor(tries, d);
  int lane = __lane_id(), wv = (int)threadIdx.x / kWave;
  uint64_t bal[kJpItems];
#pragma unroll
  for (int r = 0; r < kJpItems; ++r) {
    bal[r] = __ballot(keep[r]);
    if (lane == 0) wtot[r][wv] = __popcll(bal[r]);
  }
  __syncthreads();
  int base = 0, pos[kJpItems];
  uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kJpItems; ++r) {
    int before = 0, row = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) {
      int c = wtot[r][q];
      row += c;
      if (q < wv) before += c;
    }
    pos[r] = base + before + __popcll(bal[r] & below);
    base += row;
  }
  int* out = W + (size_t)kb * kJpChunk;
  int* outb = WB + (size_t)kb * kJpChunk;
#pragma unroll
  for (int r = 0; r < kJpItems; ++r)
    if (keep[r]) {
      out[pos[r]] = vv[r];
      outb[pos[r]] = bl[r];
    }
  if (threadIdx.x == 0) {
    cnt[kb] = base;
    int* sp = ctr + C_STRIPE + (kb & (kStripes - 1)) * kStripeW;
    if (base) atomicAdd(sp + slot, base);
  }
  if (lane == 0 && tries) atomicAdd(stripe_ptr(ctr, S_PJP), tries);
}

void jp_chunk(const Store& st, const int* A, int n, int* W, int* WB, int* cnt, bool first, Round rd, int* ctr,
              int it, hipStream_t s) {
  int nch = (n + kJpChunk - 1) / kJpChunk;
  if (nch > 0)
    k_jp_chunk<<<nch, kBlock, 0, s>>>(st, A, n, W, WB, cnt, first ? 1 : 0, rd, ctr, S_JPL + (it & 7),
                                       S_JPL + ((it + 1) & 7));
}

// ---- striped counters --------------------------------------------------------------------------
__global__ void k_stripe_zero(int* ctr, int slot, int nslots) {
  int w = (int)threadIdx.x;
  for (int k = 0; k < nslots; ++k) ctr[C_STRIPE + w * kStripeW + slot + k] = 0;
}
void stripe_zero(int* ctr, int slot, int nslots, hipStream_t s) {
  k_stripe_zero<<<1, kStripes, 0, s>>>(ctr, slot, nslots);
}
__global__ void k_stripe_sum(int* ctr, int slot, int nslots, int dst) {
  int w = (int)threadIdx.x;
  for (int k = 0; k < nslots; ++k) {
    int x = ctr[C_STRIPE + w * kStripeW + slot + k];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
    if (w == 0) ctr[dst + k] = x;
  }
}
void stripe_sum(int* ctr, int slot, int nslots, int dst, hipStream_t s) {
  static_assert(kStripes == kWave, "one lane per stripe");
  k_stripe_sum<<<1, kStripes, 0, s>>>(ctr, slot, nslots, dst);
}

// Class lists by a stable counting sort on the colour: per block (256 list
// entries) the number of each colour, an exclusive scan over (colour, block),
// then every entry goes to its colour's range at the position of its rank
// among equal colours in the block. Class lists keep the order of A.
// Class lists for colours below CM: per block a colour histogram in LDS,
// the (colour, block) table scanned in colour-major order, then each vertex
// placed at its colour's block offset plus its rank in the block. A block
// that meets a colour of CM or more stores seq to ctr[C_CWIDE] (only while it
// does not hold seq yet); the lists then report -2 colours, and the caller
// cuts them again with CM = 256. With CM = 32 the scanned table is an eighth
// of the full one.
template <int CM>
__global__ void k_class_count(const int* __restrict__ A, int n, const uint64_t* __restrict__ rw, int nb,
                              int* __restrict__ tab, int* ctr, int seq) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&h[(int)(rw[A[i]] & 0xFF)], 1);
  __syncthreads();
  if ((int)threadIdx.x < CM) tab[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
  if (CM < 256) {
    bool wide = (int)threadIdx.x >= CM && h[threadIdx.x] > 0;
    if (__ballot(wide) && __lane_id() == 0 && ((volatile int*)ctr)[C_CWIDE] != seq) ctr[C_CWIDE] = seq;
  }
}

// rank of each lane among the lanes of its block holding the same colour, in lane order
__device__ int block_rank(int c, bool valid, int* wcnt /* 4 waves x 256 */) {
  int lane = __lane_id(), w = threadIdx.x / kWave;
  uint64_t lt = (1ull << lane) - 1ull;
  int rank = 0, mine = 0;
  uint64_t left = __ballot(valid);
  while (left) {
    int lead = __ffsll((unsigned long long)left) - 1;
    int cc = __shfl(c, lead);
    uint64_t mask = __ballot(valid && c == cc);
    if (valid && c == cc) {
      rank = __popcll(mask & lt);
      mine = __popcll(mask);
    }
    if (lane == lead) wcnt[w * 256 + cc] = __popcll(mask);
    left &= ~mask;
  }
  __syncthreads();
  if (valid)
    for (int k = 0; k < w; ++k) rank += wcnt[k * 256 + c];
  (void)mine;
  return rank;
}

template <int CM>
__global__ void k_class_place(const int* __restrict__ A, int n, const uint64_t* __restrict__ rw, int nb,
                              const int* __restrict__ tabscan, int* __restrict__ out) {
  __shared__ int wcnt[4 * 256];
  for (int k = threadIdx.x; k < 4 * 256; k += blockDim.x) wcnt[k] = 0;
  __syncthreads();
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = i < n;
  int v = valid ? A[i] : -1;
  int c = valid ? (int)(rw[v] & 0xFF) : 0;
  int r = block_rank(c, valid, wcnt);
  if (valid && c < CM) out[tabscan[(int64_t)c * nb + blockIdx.x] + r] = v;
}

template <int CM>
__global__ void k_class_sizes(const int* __restrict__ tabscan, int nb, int n, int* ctr, int seq) {
  int c = threadIdx.x;
  int lo = tabscan[(int64_t)c * nb];
  int hi = c < CM - 1 ? tabscan[(int64_t)(c + 1) * nb] : n;
  ctr[C_HIST + c] = hi - lo;
  ctr[C_OFF + c] = lo;
  __syncthreads();
  if (c == 0) {
    int ncol = 0;
    for (int k = 0; k < CM; ++k)
      if (ctr[C_HIST + k]) ncol = k + 1;
    if (CM < 256 && ctr[C_CWIDE] == seq) ncol = -2;
    ctr[C_NCOL] = ncol;
  }
}

template <int CM>
static void class_lists_cm(const int* A, int n, const uint64_t* rw, int* ctr, int* out, int* tab, int* tabscan,
                           int* partial, int nb, int seq, hipStream_t s) {
  k_class_count<CM><<<nb, kBlock, 0, s>>>(A, n, rw, nb, tab, ctr, seq);
  scan_excl(tab, tabscan, CM * nb, ctr + C_TOTAL, partial, s);
  k_class_place<CM><<<nb, kBlock, 0, s>>>(A, n, rw, nb, tabscan, out);
  k_class_sizes<CM><<<1, CM, 0, s>>>(tabscan, nb, n, ctr, seq);
}

void class_lists(const int* A, int n, const uint64_t* rw, int* ctr, int* out, int* tab, int* tabscan, int* partial,
                 int cm, int seq, hipStream_t s) {
  static_assert(kBlock == 256, "class kernels use one LDS slot per colour and thread");
  int nb = (n + kBlock - 1) / kBlock;
  if (nb < 1) nb = 1;
  switch (cm) {
    case 4: class_lists_cm<4>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    case 8: class_lists_cm<8>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    case 16: class_lists_cm<16>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    case 32: class_lists_cm<32>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    case 64: class_lists_cm<64>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    case 128: class_lists_cm<128>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
    default: class_lists_cm<256>(A, n, rw, ctr, out, tab, tabscan, partial, nb, seq, s); break;
  }
}

// Small lists: one block runs the whole colouring (JP iterations separated
// by block barriers until no vertex waits) and cuts the class lists, in one
// launch. Classes come out in no particular order; the members of a class
// are an independent set, so their order does not change any result.
constexpr int kSmallThreads = 1024;
__global__ void __launch_bounds__(kSmallThreads) k_colour_small(Store st, const int* __restrict__ A, int n,
                                                              const int* n_dev, Round rd, int* W0, int* W1, int* WB,
                                                              int* __restrict__ out, int* ctr) {
  __shared__ int nwait, hist[256], cur[256];
  int tid = (int)threadIdx.x;
  if (n_dev) {
    // the list length from the device (a colouring launched ahead of the
    // read-back); a list this kernel does not take is reported as -1 colours
    // a device-driven chain that has stopped leaves the counters as they
    // are (they describe the round that ran last)
    if (rd.seeds && ctr[C_DSTOP]) return;
    n = *n_dev;
    if (n < 0 || n > kSmallColour) {
      __syncthreads();
      if (tid == 0) {
        ctr[C_NCOL] = -1;
        if (rd.seeds) ctr[C_DSTOP] = 1;  // a device-driven chain ends here
      }
      return;
    }
  }
  if (rd.seeds) rd.sseed = rd.seeds[ctr[C_DROUND]];
  for (int i = tid; i < n; i += kSmallThreads) {
    int v = A[i];
    uint64_t prio = key_of(st, rd, v) >> 32;
    rd.rw[v] = (prio << 32) | kRwAct | 0xFFull;
  }
  if (tid < 256) hist[tid] = 0;
  __syncthreads();
  const int* in = A;
  int nw = n, it = 0, visited = 0;
  while (nw > 0) {
    if (tid == 0) nwait = 0;
    __syncthreads();
    int* wout = (it & 1) ? W1 : W0;
    const int* bin = WB + ((it & 1) ? 0 : kSmallColour);  // blockers beside the entries read
    int* bout = WB + ((it & 1) ? kSmallColour : 0);
    for (int i = tid; i < nw; i += kSmallThreads) {
      int v = in[i];
      int bl = it > 0 ? bin[i] : -1;
      if (!jp_try(st, v, rd, ctr, bl)) {
        int k = atomicAdd(&nwait, 1);
        wout[k] = v;
        bout[k] = bl;
      }
    }
    __syncthreads();
    visited += nw;
    nw = nwait;
    in = wout;
    ++it;
    __syncthreads();
    if (it > 4 * kMaxColours + n) {  // cannot happen: the largest waiting key is always ready
      if (tid == 0) atomicOr(&ctr[C_ERR], E_COLOURS);
      return;
    }
  }
  for (int i = tid; i < n; i += kSmallThreads) atomicAdd(&hist[(int)(rd.rw[A[i]] & 0xFF)], 1);
  __syncthreads();
  if (tid == 0) {
    int o = 0, ncol = 0;
    for (int c = 0; c < 256; ++c) {
      cur[c] = o;
      ctr[C_OFF + c] = o;
      ctr[C_HIST + c] = hist[c];
      o += hist[c];
      if (hist[c]) ncol = c + 1;
    }
    ctr[C_NCOL] = ncol;
    ctr[C_JP] = 0;
    ctr[C_TOUCH] = 0;
    ctr[C_TOTAL] = it;
    atomicAdd(ctr + C_STRIPE + S_PJP, visited);
    if (rd.seeds) {
      // a device-driven chain takes rounds whose classes all fit one block's
      // pass; a larger class ends it here, coloured, for the host to run
      // (and count)
      bool big = false;
      for (int c = 0; c < ncol; ++c) big |= hist[c] > kSmallClass;
      if (big) {
        ctr[C_DSTOP] = 1;
      } else {
        ctr[C_ACC_COL] += n;
        ctr[C_ACC_NCOL] += ncol;
        ctr[C_ACC_IT] += it;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kSmallThreads) {
    int v = A[i];
    out[atomicAdd(&cur[(int)(rd.rw[v] & 0xFF)], 1)] = v;
  }
}
void colour_small(const Store& st, const int* A, int n, const int* n_dev, Round rd, int* W0, int* W1, int* WB,
                  int* out, int* ctr, hipStream_t s) {
  k_colour_small<<<1, kSmallThreads, 0, s>>>(st, A, n, n_dev, rd, W0, W1, WB, out, ctr);
}

__global__ void __launch_bounds__(kSmallThreads) k_select_small(Store st, int mode, double L_low2,
                                                               const int* __restrict__ A, int nA,
                                                               const int* __restrict__ touched, int cap,
                                                               uint8_t* __restrict__ nxt, int* __restrict__ seen,
                                                               int mark, int max_rounds, int* __restrict__ out,
                                                               int* ctr) {
  __shared__ int cnt;
  bool dev = nA < 0;
  if (dev) {
    if (ctr[C_DSTOP]) return;
    nA = ctr[C_LIST_B];
    mark = ctr[C_DMARK] + 1;
  }
  int nt = ctr[C_TOUCH];
  if (nt > cap || room_failed(ctr)) {
    // the host selects over every slot (and rebuilds the rows first after a
    // commit that ran out of room)
    __syncthreads();
    if (threadIdx.x == 0) {
      ctr[C_LIST_B] = -1;
      if (dev) ctr[C_DSTOP] = 1;
    }
    return;
  }
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int i = (int)threadIdx.x; i < nA + nt; i += kSmallThreads) {
    int x = i < nA ? A[i] : touched[i - nA];
    if (!nxt[x] || atomicMax(&seen[x], mark) >= mark) continue;
    nxt[x] = 0;
    if (want(st, x, mode, L_low2, nullptr)) out[atomicAdd(&cnt, 1)] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ctr[C_LIST_B] = cnt;
    if (dev) {
      int r = ctr[C_DROUND] + 1;
      ctr[C_DROUND] = r;
      ctr[C_DMARK] = mark;
      if (cnt == 0 || r >= max_rounds) ctr[C_DSTOP] = 1;
    }
  }
}
void select_small(const Store& st, int mode, double L_low2, const int* A, int nA, const int* touched, int cap,
                  uint8_t* nxt, int* seen, int mark, int max_rounds, int* out, int* ctr, hipStream_t s) {
  k_select_small<<<1, kSmallThreads, 0, s>>>(st, mode, L_low2, A, nA, touched, cap, nxt, seen, mark, max_rounds,
                                             out, ctr);
}

__global__ void k_colour_out(int V, const uint64_t* __restrict__ rw, int* __restrict__ out) {
  for (int v = gtid(); v < V; v += gstride()) out[v] = (rw[v] & kRwAct) ? (int)(rw[v] & 0xFF) : -1;
}
void colour_out(const Store& st, const uint64_t* rw, int* out, hipStream_t s) {
  k_colour_out<<<grid_for(st.V), kBlock, 0, s>>>(st.V, rw, out);
}

// ---- deferred update: stamps and claims (Sec. 3.3) -------------------------------------------
// A committed member stamps its operation and claims every row it changes;
// the claim with the largest key (the smallest member id) wins the row.
__device__ __forceinline__ void claim_row(const Commit& cm, int x, int v) {
  atomicMax((unsigned long long*)&cm.own[x], (unsigned long long)own_key(cm.epoch, v));
}
__device__ __forceinline__ void stamp(const Commit& cm, int v, int a, int b, int c) {
  cm.ops[v] = make_int4(cm.epoch, a, b, c);
}
// a record (a, b, c) for row u in this epoch: the count's epoch is raised
// first (a count of an older epoch restarts at zero). A member v collapsing
// onto u hands over its NE row: (v, ne_off, ne_cnt). A flip of the edge
// (v, w) with far vertices a and b gives rows a and b its two elements
// (lo, hi, -1); rows v and w only lose elements.
__device__ __forceinline__ void mark_target(const Commit& cm, int u, int a, int b, int c) {
  cm.tgt[u] = make_int4(a, b, c, cm.epoch);
  unsigned long long e = (unsigned long long)(uint32_t)cm.epoch << 32;
  atomicMax((unsigned long long*)&cm.tk[u], e);
  atomicAdd((unsigned long long*)&cm.tk[u], 1ull);
}

// a member is deferred when a same-class active neighbour has a larger key
__device__ __forceinline__ bool same_class_beats(const OpArgs& a, int w, uint64_t rv, int v) {
  uint64_t x = a.rw[w];
  return (x & kRwAct) && (int)(x & 0xFF) == a.cls && rw_beats(x, w, rv, v);
}
__device__ __forceinline__ bool beaten(const Store& st, int v, const OpArgs& a) {
  uint64_t rv = a.rw[v];
  Hdr h = st.hdr[v];
  for (int j = 0; j < h.y; ++j)
    if (same_class_beats(a, st.nn[h.x + j], rv, v)) return true;
  return false;
}

__device__ __forceinline__ Geo geo_of(const Store& st, int3 t) {
  return make_geo(st.xy[t.x], st.xy[t.y], st.xy[t.z], st.met[t.x], st.met[t.y], st.met[t.z]);
}
__device__ __forceinline__ Geo geo_of(const Store& st, const Elem& e) {
  return make_geo(st.xy[e.x], st.xy[e.y], st.xy[e.z], st.met[e.x], st.met[e.y], st.met[e.z]);
}

// per-wave stats: evaluated / deferred / committed; pops: also count the
// committed operations as the unit of the separate commit kernel that follows
// (grid-wide class kernels)
__device__ __forceinline__ void count_status(int status, int* ctr, bool pops = false) {
  // status: -1 idle lane, 0 deferred, 1 evaluated, 2 evaluated + committed
  uint64_t d = __ballot(status == 0);
  uint64_t e = __ballot(status >= 1);
  uint64_t c = __ballot(status == 2);
  if (__lane_id() == 0) {
    int* sp = stripe_ptr(ctr, 0);
    if (d) atomicAdd(sp + S_DEFER, __popcll(d));
    if (e) atomicAdd(sp + S_EVAL, __popcll(e));
    if (c) atomicAdd(sp + S_COMMIT, __popcll(c));
    if (c && pops) atomicAdd(sp + S_POPS, __popcll(c));
  }
}

// ---- coarsening (Sec. 2.4.1) --------------------------------------------------------------
// Candidates u: neighbours on every boundary side v lies on, with L^2 < L_low2,
// tried in ascending (L^2, u); the first whose re-pointed elements all keep
// area > 0 and q^2 >= q_min^2 is taken.
__device__ __forceinline__ int collapse_one(const Store& st, int v, const OpArgs& a, const Commit& cm, int* ctr) {
  Hdr h = st.hdr[v];
  double2 pv = st.xy[v];
  Met mv = st.met[v];
  uint8_t tv = st.tag[v];
  uint64_t rv = a.rw[v];
  // one pass over the 1-ring: re-validation and the first candidate together
  double bL = INFINITY;
  int bU = -1;
  for (int j = 0; j < h.y; ++j) {
    int w = st.nn[h.x + j];
    if (same_class_beats(a, w, rv, v)) {
      cm.nxt[v] = 1;
      return 0;
    }
    if (tv & ~st.tag[w]) continue;
    double L = len2(pv, mv, st.xy[w], st.met[w]);
    if (!(L < a.L_low2)) continue;
    if (bU < 0 || L < bL || (L == bL && w < bU)) {
      bL = L;
      bU = w;
    }
  }
  double lastL = -INFINITY;
  int lastU = -1;
  int u = -1;
  for (bool first = true;; first = false) {
    if (!first) {
      bL = INFINITY;
      bU = -1;
      for (int j = 0; j < h.y; ++j) {
      int w = st.nn[h.x + j];
      if (tv & ~st.tag[w]) continue;
      double L = len2(pv, mv, st.xy[w], st.met[w]);
      if (!(L < a.L_low2)) continue;
      bool after = L > lastL || (L == lastL && w > lastU);
      bool better = bU < 0 || L < bL || (L == bL && w < bU);
      if (after && better) {
        bL = L;
        bU = w;
      }
      }
    }
    if (bU < 0) break;
    bool ok = true;
    for (int i = 0; i < h.w && ok; ++i) {
      Elem e = st.tri[st.ne[h.z + i]];
      if (holds(e, bU)) continue;
      int k = slot_of(e, v);
      int3 r = rot_min(k == 0 ? bU : e.x, k == 1 ? bU : e.y, k == 2 ? bU : e.z);
      Geo g = geo_of(st, r);
      if (!(area2(g) > 0.0) || !(qd2(g, st.qk) >= a.qmin2)) ok = false;
    }
    if (ok) {
      u = bU;
      break;
    }
    lastL = bL;
    lastU = bU;
  }
  if (u < 0) return 1;
  // apply: v's elements are owned by v within this independent set
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    if (holds(e, u)) {
      e.w = 0;
    } else {
      int k = slot_of(e, v);
      int3 r = rot_min(k == 0 ? u : e.x, k == 1 ? u : e.y, k == 2 ? u : e.z);
      e = make_int4(r.x, r.y, r.z, 1);
    }
    st.tri[t] = e;
  }
  st.valive[v] = 0;
  stamp(cm, v, -(u + 1), h.z, h.w);
  mark_target(cm, u, v, h.z, h.w);
  for (int j = 0; j < h.y; ++j) claim_row(cm, st.nn[h.x + j], v);
  return 2;
}

template <int QK>
__global__ void k_collapse(Store st, const int* __restrict__ list, int n, OpArgs a, Commit cm, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  if (room_failed(ctr)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[C_STAGE] = 0;  // the commit's fallback staging
  int i = xtid();
  int status = -1;
  if (i < n) status = collapse_one(st, list[i], a, cm, ctr);
  count_status(status, ctr, true);
}
template <int G, int QK>
__global__ void __launch_bounds__(256, 5) k_collapse_g(Store st, const int* __restrict__ list, int n, OpArgs a,
                                                    Commit cm, int* ctr);
void collapse_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, int lanes,
                    hipStream_t s) {
  if (n <= 0) return;
  if (lanes == 16)
    (st.qk ? k_collapse_g<16, 1> : k_collapse_g<16, 0>)<<<(int)(((int64_t)n * 16 + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        st, list, n, a, cm, ctr);
  else if (lanes == 8)
    (st.qk ? k_collapse_g<8, 1> : k_collapse_g<8, 0>)<<<(int)(((int64_t)n * 8 + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        st, list, n, a, cm, ctr);
  else
    (st.qk ? k_collapse<1> : k_collapse<0>)<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(st, list, n, a, cm, ctr);
}

// ---- swapping (Sec. 2.4.3) ------------------------------------------------------------------
// For every interior edge (v, w): (v,w,a) and (w,v,b) become (v,b,a) and (w,a,b)
// when both areas stay positive and the smaller q^2 rises strictly; the best
// new minimum wins, ties to the smaller w; the element holding v keeps the
// smaller id.
__device__ __forceinline__ int flip_one(const Store& st, int v, const OpArgs& a, const Commit& cm, int* ctr) {
  if (beaten(st, v, a)) {
    cm.nxt[v] = 1;
    return 0;
  }
  Hdr h = st.hdr[v];
  double best = 0.0;
  int bw = -1, bT1 = -1, bT2 = -1, ba = -1, bb = -1;
  for (int i = 0; i < h.w; ++i) {
    int T1 = st.ne[h.z + i];
    Elem e1 = st.tri[T1];
    int k1 = slot_of(e1, v);
    int w = at(e1, k1 == 2 ? 0 : k1 + 1);
    int av = at(e1, k1 == 0 ? 2 : k1 - 1);
    int T2 = -1, bv = -1;
    Elem e2;
    for (int j = 0; j < h.w; ++j) {
      int t = st.ne[h.z + j];
      Elem e = st.tri[t];
      int k = slot_of(e, v);
      if (at(e, k == 0 ? 2 : k - 1) == w) {
        T2 = t;
        e2 = e;
        bv = at(e, k == 2 ? 0 : k + 1);
        break;
      }
    }
    if (T2 < 0) continue;
    Geo gv = geo_of(st, rot_min(v, bv, av));
    Geo gw = geo_of(st, rot_min(w, av, bv));
    if (!(area2(gv) > 0.0) || !(area2(gw) > 0.0)) continue;
    double qv = qd2(gv, st.qk), qw = qd2(gw, st.qk);
    double q1 = qd2(geo_of(st, e1), st.qk), q2 = qd2(geo_of(st, e2), st.qk);
    double nmin = qw < qv ? qw : qv;
    double omin = q2 < q1 ? q2 : q1;
    if (!(nmin > omin)) continue;
    if (bw < 0 || nmin > best || (nmin == best && w < bw)) {
      best = nmin;
      bw = w;
      bT1 = T1;
      bT2 = T2;
      ba = av;
      bb = bv;
    }
  }
  if (bw < 0) return 1;
  int lo = min(bT1, bT2), hi = max(bT1, bT2);
  int3 tv = rot_min(v, bb, ba), tw = rot_min(bw, ba, bb);
  st.tri[lo] = make_int4(tv.x, tv.y, tv.z, 1);
  st.tri[hi] = make_int4(tw.x, tw.y, tw.z, 1);
  stamp(cm, v, lo, hi, 0);
  mark_target(cm, ba, lo, hi, -1);
  mark_target(cm, bb, lo, hi, -1);
  claim_row(cm, v, v);
  claim_row(cm, bw, v);
  claim_row(cm, ba, v);
  claim_row(cm, bb, v);
  return 2;
}

template <int QK>
__global__ void k_flip(Store st, const int* __restrict__ list, int n, OpArgs a, Commit cm, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  if (room_failed(ctr)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[C_STAGE] = 0;  // the commit's fallback staging
  int i = xtid();
  int status = -1;
  if (i < n) status = flip_one(st, list[i], a, cm, ctr);
  count_status(status, ctr, true);
}
void flip_class(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, hipStream_t s) {
  if (n > 0) (st.qk ? k_flip<1> : k_flip<0>)<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(st, list, n, a, cm, ctr);
}

// ---- deferred update: commit ------------------------------------------------------------------
// Each claimed row is rebuilt once, by the owner's thread, from its candidate
// elements: the old NE(x), all of NE(w) for a neighbour w collapsed onto x,
// and the two elements of every committed flip around x. NE(x) becomes the
// sorted candidates that are live and hold x (the canonical order); NN(x) is
// then the set of the other vertices of those elements.

// the candidates of row x that are live and hold x (possibly repeated),
// written to dst[k * stride] for k < lim; returns how many there are. A class
// holds one kind of operation: F, flips (records (epoch, t1, t2, 0)), else
// collapses (records (epoch, -(u+1), ne_off, ne_cnt), the member's NE row).
// Rows of up to kCandB entries are gathered level by level, each level's
// loads issued together: NE(x), NN(x) and x's own record; then the elements
// of NE(x) and the neighbours' records; then what those records name (an
// absorbed NE row, then its elements; or each flip's two elements). Element
// and record loads take index 0 for an empty slot, so that no load waits on
// a branch. Longer rows go through the same steps B entries at a time.
// Filtering here keeps the candidate count at the new row's size (a collapse
// target's old row and the absorbed row share only the two elements that die).
constexpr int kCandB = 8;  // row entries per batch (two 16-byte loads)
__device__ __forceinline__ bool keeps(const Elem& e, int x) { return e.w && holds(e, x); }

template <bool F>
__device__ __forceinline__ int row_candidates(const Store& st, const Commit& cm, int x, Hdr h, int* dst, int stride,
                                              int lim) {
  constexpr int B = kCandB;
  int n = 0;
  auto put = [&](int t) {
    if (n < lim) dst[n * stride] = t;
    ++n;
  };
  // the elements t[0 .. B) (t < 0: none) that are live and hold x
  auto put_live = [&](const int (&t)[B]) {
    Elem e[B];
#pragma unroll
    for (int q = 0; q < B; ++q) e[q] = st.tri[max(t[q], 0)];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t[q] >= 0 && keeps(e[q], x)) put(t[q]);
  };
  // NE(w) of a neighbour w collapsed onto x
  auto absorb = [&](int z, int cnt) {
    for (int k0 = 0; k0 < cnt; k0 += B) {
      int t[B];
      row8(st.ne, z + k0, cnt - k0, t);
      put_live(t);
    }
  };
  if (!F) {
    // collapses onto x: their count (this epoch's, else none) and the last
    // one's NE range
    uint64_t tk = cm.tk[x];
    int4 tg = cm.tgt[x];
    int nt = (uint32_t)(tk >> 32) == (uint32_t)cm.epoch ? (int)(uint32_t)tk : 0;
    if (h.w <= B && (nt == 0 || (nt == 1 && tg.z <= B))) {
      // the entries of NE(x) and of the absorbed row side by side, then the
      // elements of each
      int t[B], u[B];
      row8(st.ne, h.z, h.w, t);
      row8(st.ne, tg.y, nt == 1 ? tg.z : 0, u);
      put_live(t);
      if (nt == 1) put_live(u);
      return n;
    }
    absorb(h.z, h.w);
    if (nt == 1) {
      absorb(tg.y, tg.z);
    } else if (nt > 1) {
      // several members collapsed onto x: their ranges, from their records
      for (int j = 0; j < h.y; ++j) {
        int4 r = cm.ops[st.nn[h.x + j]];
        if (r.x == cm.epoch && r.y == -x - 1) absorb(r.z, r.w);
      }
    }
    return n;
  }
  // flips: NE(x), and the two elements of a flip whose far vertex x is,
  // from x's record; x the far vertex of several flips: the two elements of
  // every committed flip around x (x's own and its neighbours'), four
  // neighbour records at a time
  uint64_t tkf = cm.tk[x];
  int4 tgf = cm.tgt[x];
  int ntf = (uint32_t)(tkf >> 32) == (uint32_t)cm.epoch ? (int)(uint32_t)tkf : 0;
  if (ntf <= 1) {
    int t[B], u[B];
    row8(st.ne, h.z, h.w, t);
#pragma unroll
    for (int q = 0; q < B; ++q) u[q] = -1;
    if (ntf == 1) {
      u[0] = tgf.x;
      u[1] = tgf.y;
    }
    put_live(t);
    if (ntf == 1) put_live(u);
    for (int k0 = B; k0 < h.w; k0 += B) {
      row8(st.ne, h.z + k0, h.w - k0, t);
      put_live(t);
    }
    return n;
  }
  int4 rx = cm.ops[x];
  auto scan_flips = [&](const int (&w)[B]) {
#pragma unroll
    for (int q0 = 0; q0 < B; q0 += B / 2) {
      int4 r[B / 2];
#pragma unroll
      for (int q = 0; q < B / 2; ++q) r[q] = cm.ops[max(w[q0 + q], 0)];
      int f0[B / 2], f1[B / 2];
#pragma unroll
      for (int q = 0; q < B / 2; ++q) {
        bool c = w[q0 + q] >= 0 && r[q].x == cm.epoch && r[q].y >= 0;
        f0[q] = c ? r[q].y : -1;
        f1[q] = c ? r[q].z : -1;
      }
      Elem e0[B / 2], e1[B / 2];
#pragma unroll
      for (int q = 0; q < B / 2; ++q) e0[q] = st.tri[max(f0[q], 0)];
#pragma unroll
      for (int q = 0; q < B / 2; ++q) e1[q] = st.tri[max(f1[q], 0)];
#pragma unroll
      for (int q = 0; q < B / 2; ++q) {
        if (f0[q] >= 0 && keeps(e0[q], x)) put(f0[q]);
        if (f1[q] >= 0 && keeps(e1[q], x)) put(f1[q]);
      }
    }
  };
  if (h.w <= B && h.y <= B) {
    int t[B], w[B];
    row8(st.ne, h.z, h.w, t);
    row8(st.nn, h.x, h.y, w);
    put_live(t);
    scan_flips(w);
  } else {
    absorb(h.z, h.w);
    for (int j0 = 0; j0 < h.y; j0 += B) {
      int w[B];
      row8(st.nn, h.x + j0, h.y - j0, w);
      scan_flips(w);
    }
  }
  if (rx.x == cm.epoch && rx.y >= 0) {
    Elem a = st.tri[rx.y], b = st.tri[rx.z];
    if (keeps(a, x)) put(rx.y);
    if (keeps(b, x)) put(rx.z);
  }
  return n;
}

__device__ void sort_unique(int* a, int& n) {
  for (int i = 1; i < n; ++i) {
    int x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (m == 0 || a[i] != a[m - 1]) a[m++] = a[i];
  n = m;
}

__device__ __forceinline__ int grown_cap(int n) { return max(8, (2 * n + 3) & ~3); }

// write a sorted row, in place when it fits, else in fresh pool space; on
// pool exhaustion the row keeps its slot and is cut to its capacity, so no
// later read leaves the pool, and the error bit has the host rebuild every
// row before the round goes on
__device__ int put_row(int* pool, int64_t pool_cap, int* top, int& off, int& cap, const int* src, int n, int err,
                       int epoch, int* ctr) {
  if (n > cap) {
    int nc = grown_cap(n);
    int o = atomicAdd(top, nc);
    if ((int64_t)o + nc > pool_cap) {
      room_fail(ctr, err, epoch);
      n = cap;
    } else {
      off = o;
      cap = nc;
      atomicAdd(stripe_ptr(ctr, S_RELOC), 1);
    }
  }
  for (int k = 0; k < n; ++k) pool[off + k] = src[k];
  return n;
}

// general path: candidates in a private staging range, insertion sorts there
template <bool F>
__device__ __forceinline__ void rebuild_staged(const Store& st, const Commit& cm, int x, int* ctr) {
  Hdr h = st.hdr[x];
  int2 cp = st.cap[x];
  int tot = row_candidates<F>(st, cm, x, h, nullptr, 0, 0);
  int64_t need = 4 * (int64_t)tot + 4;
  int base = atomicAdd(&ctr[C_STAGE], (int)need);
  if ((int64_t)base + need > cm.stage_cap) {
    room_fail(ctr, E_STAGE, cm.epoch);
    return;
  }
  int* s = cm.stage + base;
  row_candidates<F>(st, cm, x, h, s, 1, tot);
  int m = tot;
  sort_unique(s, m);
  int* q = s + tot;
  int nq = 0;
  for (int k = 0; k < m; ++k) {
    Elem e = st.tri[s[k]];
    if (e.x != x) q[nq++] = e.x;
    if (e.y != x) q[nq++] = e.y;
    if (e.z != x) q[nq++] = e.z;
  }
  sort_unique(q, nq);
  int ne_off = h.z, ne_cap = cp.y, nn_off = h.x, nn_cap = cp.x;
  m = put_row(st.ne, st.ne_pool, &ctr[C_NE_TOP], ne_off, ne_cap, s, m, E_NE_POOL, cm.epoch, ctr);
  nq = put_row(st.nn, st.nn_pool, &ctr[C_NN_TOP], nn_off, nn_cap, q, nq, E_NN_POOL, cm.epoch, ctr);
  st.hdr[x] = make_int4(nn_off, nq, ne_off, m);
  st.cap[x] = make_int2(nn_cap, ne_cap);
}

// the three vertex ids of element t (its live flag not loaded)
__device__ __forceinline__ Elem tri_ids(const Store& st, int t) {
  const int* p = (const int*)(st.tri + t);
  return make_int4(p[0], p[1], p[2], 1);
}

constexpr int kRegSmall = 16;  // rows up to this many candidates: the small register path
constexpr int kRegRow = 32;    // up to this many: the large register path

// wave-wide exclusive offsets into two counters, both atomics in flight together
__device__ __forceinline__ int2 wave_add2(int* c0, int a0, int* c1, int a1) {
  int lane = __lane_id();
  int i0 = a0, i1 = a1;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int o0 = __shfl_up(i0, d), o1 = __shfl_up(i1, d);
    if (lane >= d) {
      i0 += o0;
      i1 += o1;
    }
  }
  int b0 = 0, b1 = 0;
  if (lane == kWave - 1) {
    if (i0 > 0) b0 = atomicAdd(c0, i0);
    if (i1 > 0) b1 = atomicAdd(c1, i1);
  }
  b0 = __shfl(b0, kWave - 1);
  b1 = __shfl(b1, kWave - 1);
  return make_int2(b0 + i0 - a0, b1 + i1 - a1);
}

// Register path for rows of at most N candidates, staged in this thread's
// LDS column (x < 0: idle lane). Every lane of the wavefront makes this call
// together, so fresh pool space is handed out with one atomic per wavefront
// and pool. NE(x) = the sorted, distinct candidates that are live and hold
// x, written back to the column; NN(x) = the sorted "next" vertices of those
// elements plus the one "previous" vertex that is no "next" (x on the
// boundary). Returns true for a row whose elements do not form a disk or a
// half-disk around x; such a row is left to the general path.
template <int N, int S>
__device__ __forceinline__ bool rebuild_reg(const Store& st, const Commit& cm, int x, Hdr h, int2 cp, int tot, int* col,
                                            int* ctr) {
  bool act = x >= 0;
  int m = 0;
  {
    int c[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int t = INT_MAX;
      if (act && k < tot) t = col[k * S];
      c[k] = t;
    }
    bitonic<N>(c);
    int prev = INT_MAX;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int t = c[k];
      if (t != INT_MAX && t != prev) col[(m++) * S] = t;
      prev = t;
    }
  }
  // next vertex of x in each element (and, for the small path, the previous
  // one from the same load; the large path loads the elements again rather
  // than hold both arrays)
  constexpr bool kBoth = N <= kRegSmall;
  int nx[N], pv[kBoth ? N : 1];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int t = k < m ? col[k * S] : -1;
    Elem e = tri_ids(st, max(t, 0));
    int sl = slot_of(e, x);
    nx[k] = t >= 0 ? at(e, sl == 2 ? 0 : sl + 1) : INT_MAX;
    if constexpr (kBoth) pv[k] = t >= 0 ? at(e, sl == 0 ? 2 : sl - 1) : -1;
    // the large path keeps at most eight element loads in flight
    if constexpr (!kBoth)
      if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
  }
  bitonic<N>(nx);
  // previous vertices that are no next (one for a boundary vertex; more:
  // the elements form no disk or half-disk, and the general path decides)
  int extra = INT_MAX, nextra = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < m) {
      int b;
      if constexpr (kBoth) {
        b = pv[k];
      } else {
        Elem e = tri_ids(st, col[k * S]);
        int sl = slot_of(e, x);
        b = at(e, sl == 0 ? 2 : sl - 1);
      }
      bool found = false;
#pragma unroll
      for (int q = 0; q < N; ++q) found |= nx[q] == b;
      if (!found) {
        extra = b;
        ++nextra;
      }
    }
  }
  bool odd = act && nextra > 1;
  bool reg = act && !odd;
  int nq = nextra;
#pragma unroll
  for (int k = 0; k < N; ++k) nq += nx[k] != INT_MAX;
  // slots: in place when the row fits, else fresh pool space
  int ne_off = h.z, ne_cap = cp.y, nn_off = h.x, nn_cap = cp.x;
  int ne_need = reg && m > ne_cap ? grown_cap(m) : 0;
  int nn_need = reg && nq > nn_cap ? grown_cap(nq) : 0;
  int2 at2 = wave_add2(&ctr[C_NE_TOP], ne_need, &ctr[C_NN_TOP], nn_need);
  int lim_ne = m, lim_nn = nq;
  if (ne_need) {
    if ((int64_t)at2.x + ne_need > st.ne_pool) {
      room_fail(ctr, E_NE_POOL, cm.epoch);
      lim_ne = min(m, ne_cap);
    } else {
      ne_off = at2.x;
      ne_cap = ne_need;
    }
  }
  if (nn_need) {
    if ((int64_t)at2.y + nn_need > st.nn_pool) {
      room_fail(ctr, E_NN_POOL, cm.epoch);
      lim_nn = min(nq, nn_cap);
    } else {
      nn_off = at2.y;
      nn_cap = nn_need;
    }
  }
  uint64_t rel = __ballot(ne_need > 0), rel2 = __ballot(nn_need > 0);
  if (__lane_id() == 0 && (rel | rel2)) atomicAdd(stripe_ptr(ctr, S_RELOC), __popcll(rel) + __popcll(rel2));
  if (reg) {
    // NE(x) four entries per store (the slot holds a multiple of four; the
    // entries past the row are padding)
    for (int k = 0; k < lim_ne; k += 4)
      *(int4*)(st.ne + ne_off + k) = make_int4(col[k * S], col[(k + 1) * S], col[(k + 2) * S], col[(k + 3) * S]);
    int w = 0;
    bool put = nextra == 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int v = nx[k];
      if (v == INT_MAX) continue;
      if (!put && extra < v) {
        if (w < lim_nn) st.nn[nn_off + w] = extra;
        ++w;
        put = true;
      }
      if (w < lim_nn) st.nn[nn_off + w] = v;
      ++w;
    }
    if (!put) {
      if (w < lim_nn) st.nn[nn_off + w] = extra;
      ++w;
    }
    st.hdr[x] = make_int4(nn_off, lim_nn, ne_off, lim_ne);
    st.cap[x] = make_int2(nn_cap, ne_cap);
  }
  return odd;
}

// Rebuild row x (x < 0: idle lane); every lane of the wavefront makes this
// call together. Rows of up to N candidates (staged in this thread's LDS
// column: N slots, stride S) take the register path. Rows with more are
// queued in the block's LDS queue bq when one is given (for the larger
// register path after the small rows), else they and rows that are no disk
// take the general path. A row's first visit (bq given) flags it for the
// next round and, in small rounds, appends it to the list of rebuilt rows;
// that append's atomic is in flight while the row is gathered.
template <bool F, int N, int S>
__device__ __forceinline__ void rebuild_row(const Store& st, const Commit& cm, int x, int* col, int* ctr, int* bq,
                                            int* bqn) {
  bool act = x >= 0;
  bool first = bq != nullptr;
  int tbase = 0, tincl = 0;
  if (first && cm.touched) {
    int lane = __lane_id();
    tincl = act ? 1 : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      int o = __shfl_up(tincl, d);
      if (lane >= d) tincl += o;
    }
    if (lane == kWave - 1 && tincl > 0) tbase = atomicAdd(&ctr[C_TOUCH], tincl);
  }
  int tot = 0;
  Hdr h = make_int4(0, 0, 0, 0);
  int2 cp = make_int2(0, 0);
  if (act) {
    h = st.hdr[x];
    cp = st.cap[x];
    tot = row_candidates<F>(st, cm, x, h, col, S, N);
  }
  bool reg = act && tot <= N;
  bool later = false;
  if (first && act && !reg) {
    int slot = atomicAdd(bqn, 1);
    if (slot < kBlock) {
      bq[slot] = x;
      later = true;
    }
  }
  bool general = act && !reg && !later;
  if (__ballot(reg)) general |= rebuild_reg<N, S>(st, cm, reg ? x : -1, h, cp, tot, col, ctr);
  if (general) rebuild_staged<F>(st, cm, x, ctr);
  if (first) {
    if (act) cm.nxt[x] = 1;
    if (cm.touched) {
      int slot = __shfl(tbase, kWave - 1) + tincl - 1;
      if (act && slot < cm.touched_cap) cm.touched[slot] = x;
    }
  }
  bool done = act && !later;  // a queued row is counted when it is rebuilt
  uint64_t rows = __ballot(done);
  if (__lane_id() == 0 && rows) {
    int* sp = stripe_ptr(ctr, 0);
    atomicAdd(sp + S_ROWS, __popcll(rows));
    atomicAdd(sp + S_PROWS, __popcll(rows));
  }
}

// block-wide exclusive scan of one int per thread; returns the block total
__device__ __forceinline__ int block_scan(int x, int& excl, int* wsum) {
  int lane = __lane_id(), wv = (int)threadIdx.x / kWave;
  int incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kBlock / kWave; ++q) {
    int c = wsum[q];
    total += c;
    if (q < wv) before += c;
  }
  excl = before + incl - x;
  return total;
}

// LDS of one commit block
constexpr int kPairB = 8;  // neighbours per member taken per pair round (two 16-byte loads)
struct CommitLds {
  int col[kRegSmall * kBlock];  // candidate staging: kRegSmall per thread, or kRegRow for half the threads
  int q[kPairB * kBlock];       // rows queued in a pair round
  int bq[kBlock];               // rows of more than kRegSmall candidates
  int bqn;
  int wsum[kBlock / kWave];
};
static_assert(kRegSmall * kBlock == kRegRow * (kBlock / 2), "the large path stages in the same LDS");

// Rebuild the rows claimed by the committed members list[base .. base + cnt)
// (cnt <= kBlock), with all kBlock threads of the block. Each member has tpm
// threads (a power of two: as many as fit, so a block of few members spreads
// each member's neighbours over its threads); a thread takes kPairB of its
// member's neighbours per pair round (row entries, then owner keys, loaded
// side by side). The rows a member owns are queued in LDS in block order and
// rebuilt 256 at a time. For flips one more round queues the members' own
// rows, after the rounds that read the members' rows.
template <bool F>
__device__ __forceinline__ void commit_chunk(const Store& st, const int* __restrict__ list, int base, int cnt,
                                             const Commit& cm, int* ctr, CommitLds& L) {
  int tid = (int)threadIdx.x;
  int lg = 0;
  while ((cnt << (lg + 1)) <= kBlock) ++lg;
  int mi = tid >> lg, sl = tid & ((1 << lg) - 1);
  int v = -1, deg = 0, off = 0;
  bool com = false;
  if (mi < cnt) {
    v = list[base + mi];
    int ep = cm.ops[v].x;
    Hdr h = st.hdr[v];
    com = ep == cm.epoch;
    if (com) {
      deg = h.y;
      off = h.x;
    }
  }
  uint64_t key = own_key(cm.epoch, v);
  int* mycol = L.col + tid;
  if (tid == 0) L.bqn = 0;
  bool own_round = F;
  for (int j0 = sl * kPairB;; j0 += kPairB << lg) {
    bool pairs = __syncthreads_or(j0 < deg);
    if (!pairs && !own_round) break;
    int y[kPairB];
    uint64_t k[kPairB];
    if (pairs) {
      row8(st.nn, off + j0, deg - j0, y);
#pragma unroll
      for (int q = 0; q < kPairB; ++q) k[q] = y[q] >= 0 ? cm.own[y[q]] : 0ull;
    } else {
      own_round = false;
      bool mine_row = com && sl == 0;
#pragma unroll
      for (int q = 0; q < kPairB; ++q) y[q] = -1;
      if (mine_row) y[0] = v;
      k[0] = mine_row ? cm.own[v] : 0ull;
#pragma unroll
      for (int q = 1; q < kPairB; ++q) k[q] = 0ull;
    }
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kPairB; ++q) mine += (y[q] >= 0 && k[q] == key) ? 1 : 0;
    int at;
    int tot = block_scan(mine, at, L.wsum);
#pragma unroll
    for (int q = 0; q < kPairB; ++q)
      if (y[q] >= 0 && k[q] == key) L.q[at++] = y[q];
    __syncthreads();
    for (int r0 = 0; r0 < tot; r0 += kBlock)
      rebuild_row<F, kRegSmall, kBlock>(st, cm, r0 + tid < tot ? L.q[r0 + tid] : -1, mycol, ctr, L.bq, &L.bqn);
  }
  // rows of more than kRegSmall candidates, half the block at a time
  __syncthreads();
  int nbig = min(L.bqn, kBlock);
  constexpr int H = kBlock / 2;
  for (int b0 = 0; b0 < nbig; b0 += H) {
    int x = (tid < H && b0 + tid < nbig) ? L.bq[b0 + tid] : -1;
    rebuild_row<F, kRegRow, H>(st, cm, x, L.col + (tid & (H - 1)), ctr, nullptr, nullptr);
  }
  __syncthreads();  // the LDS is reused by the next chunk
}

// One block per mpb class members (commit_rows chooses mpb), in XCD-aware
// block order; one kernel per kind of operation.
template <bool F>
__global__ void __launch_bounds__(256, 5) k_commit(Store st, const int* __restrict__ list, int n, int mpb, Commit cm,
                                                int* ctr) {
  __shared__ CommitLds L;
  if (room_failed_block(ctr)) return;  // other blocks may set it meanwhile: one answer per block
  int base = xcd_block() * mpb;
  commit_chunk<F>(st, list, base, min(mpb, n - base), cm, ctr, L);
}

// The same rebuild in vertex order, for classes whose claimed rows cover a
// good part of the mesh: a work-group scans `chunk` consecutive vertex slots
// (at most kSweepMax), queues the rows claimed in this epoch in LDS in slot
// order (a block-wide ordered compaction, so every lane of a rebuild pass has
// a row), and rebuilds them kBlock at a time. Consecutive rows then read
// nearby headers, capacities, owner keys and target records, and walk rows
// and elements in the order they are laid out, where the member-driven form
// above touches them in its members' neighbour order. Every row is still
// rebuilt once, from the same candidates, so the rows are the same.
constexpr int kSweepStep = kPairB * kBlock;  // slots scanned per block-wide pass
constexpr int kSweepMax = 2 * kSweepStep;    // most slots per work-group (16-bit offsets in LDS)
struct SweepLds {
  int col[kRegSmall * kBlock];
  uint16_t q[kSweepMax];
  int bq[kBlock];
  int bqn;
  int wsum[kBlock / kWave];
};
static_assert(kSweepMax <= 65536, "slot offsets are 16-bit");

template <bool F>
__global__ void __launch_bounds__(256, 5) k_commit_sweep(Store st, Commit cm, int chunk, int* ctr) {
  __shared__ SweepLds L;
  if (room_failed_block(ctr)) return;
  int tid = (int)threadIdx.x;
  int base = xcd_block() * chunk;
  int end = min(st.V, base + chunk);
  // each pass: thread tid reads the owner keys of kPairB consecutive slots,
  // all in flight together, and one block-wide scan places the claimed rows
  // in slot order
  int qn = 0;
  for (int s0 = base; s0 < end; s0 += kSweepStep) {
    int first = s0 + tid * kPairB;
    bool dirty[kPairB];
    int mine = 0;
    {
      uint64_t k[kPairB];
#pragma unroll
      for (int q = 0; q < kPairB; ++q) k[q] = first + q < end ? cm.own[first + q] : 0ull;
#pragma unroll
      for (int q = 0; q < kPairB; ++q) {
        dirty[q] = first + q < end && (uint32_t)(k[q] >> 32) == (uint32_t)cm.epoch;
        mine += dirty[q] ? 1 : 0;
      }
    }
    int at;
    int tot = block_scan(mine, at, L.wsum);
    at += qn;
#pragma unroll
    for (int q = 0; q < kPairB; ++q)
      if (dirty[q]) L.q[at++] = (uint16_t)(first + q - base);
    qn += tot;
    __syncthreads();  // wsum is reused by the next scan
  }
  if (tid == 0) L.bqn = 0;
  __syncthreads();
  for (int r0 = 0; r0 < qn; r0 += kBlock)
    rebuild_row<F, kRegSmall, kBlock>(st, cm, r0 + tid < qn ? base + (int)L.q[r0 + tid] : -1, L.col + tid, ctr,
                                      L.bq, &L.bqn);
  __syncthreads();
  int nbig = min(L.bqn, kBlock);
  constexpr int H = kBlock / 2;
  for (int b0 = 0; b0 < nbig; b0 += H) {
    int y = (tid < H && b0 + tid < nbig) ? L.bq[b0 + tid] : -1;
    rebuild_row<F, kRegRow, H>(st, cm, y, L.col + (tid & (H - 1)), ctr, nullptr, nullptr);
  }
}

// Work-groups of `fn` (kBlock threads) resident on the current device at
// once: work-groups per CU from the occupancy calculator times the CUs,
// kept per device. The commits size their grids by it, so that a grid runs
// as one generation of resident work-groups: a grid slightly larger than
// that runs a second, short generation that leaves most of the chip idle.
constexpr int kMaxDevices = 64;
int resident_blocks(const void* fn, int which) {
  static std::atomic<int> cache[4][kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = -1;
  if (dev >= 0) {
    int r = cache[which][dev].load(std::memory_order_relaxed);
    if (r > 0) return r;
  }
  int per = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBlock, 0) != hipSuccess || per <= 0) per = 4;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  int r = per * cus;
  if (dev >= 0) cache[which][dev].store(r, std::memory_order_relaxed);
  return r;
}

void commit_sweep(const Store& st, Commit cm, bool flips, int* ctr, hipStream_t s) {
  if (st.V <= 0) return;
  int res = flips ? resident_blocks((const void*)&k_commit_sweep<true>, 0)
                  : resident_blocks((const void*)&k_commit_sweep<false>, 1);
  // slots per work-group: a multiple of kBlock, at most kSweepMax
  int64_t per = ((int64_t)st.V + res - 1) / res;
  int chunk = (int)std::min<int64_t>(kSweepMax, std::max<int64_t>(kBlock, (per + kBlock - 1) / kBlock * kBlock));
  int nb = (st.V + chunk - 1) / chunk;
  if (flips)
    k_commit_sweep<true><<<nb, kBlock, 0, s>>>(st, cm, chunk, ctr);
  else
    k_commit_sweep<false><<<nb, kBlock, 0, s>>>(st, cm, chunk, ctr);
}

void commit_rows(const Store& st, const int* list, int n, Commit cm, bool flips, int chunk, int* ctr, hipStream_t s) {
  if (n <= 0) return;
  int mpb = chunk;
  if (mpb <= 0) {
    // members per work-group: at least 4 (a small class then spreads over
    // more work-groups, each with several threads per member), more when
    // that keeps the grid within one generation of resident work-groups
    int res = flips ? resident_blocks((const void*)&k_commit<true>, 2)
                    : resident_blocks((const void*)&k_commit<false>, 3);
    mpb = std::min(kBlock, std::max(4, (n + res - 1) / res));
  }
  int nb = (n + mpb - 1) / mpb;
  if (flips)
    k_commit<true><<<nb, kBlock, 0, s>>>(st, list, n, mpb, cm, ctr);
  else
    k_commit<false><<<nb, kBlock, 0, s>>>(st, list, n, mpb, cm, ctr);
}


// ---- smoothing (Sec. 2.4.4) ---------------------------------------------------------------------
__global__ void k_elem_metric(Store st, Met* __restrict__ out) {
  for (int t = gtid(); t < st.T; t += gstride()) {
    Elem e = st.tri[t];
    if (!e.w) continue;
    Met m0 = st.met[e.x], m1 = st.met[e.y], m2 = st.met[e.z];
    Met r;
    r.a = ((m0.a + m1.a) + m2.a) / 3.0;
    r.b = ((m0.b + m1.b) + m2.b) / 3.0;
    r.c = ((m0.c + m1.c) + m2.c) / 3.0;
    out[t] = r;
  }
}
void element_metrics(const Store& st, Met* out, hipStream_t s) {
  k_elem_metric<<<grid_for(st.T), kBlock, 0, s>>>(st, out);
}

__global__ void k_vertex_records(Store st, VRec* __restrict__ out) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    double2 p = st.xy[v];
    Met m = st.met[v];
    VRec r;
    r.x = p.x;
    r.y = p.y;
    r.a = m.a;
    r.b = m.b;
    r.c = m.c;
    r.tag = st.tag[v];
    r.pad0 = 0;
    r.pad1 = 0.0;
    r.pad2 = 0.0;
    out[v] = r;
  }
}
void vertex_records(const Store& st, VRec* out, hipStream_t s) {
  if (st.V > 0) k_vertex_records<<<grid_for(st.V), kBlock, 0, s>>>(st, out);
}

// element t's geometry with vertex v at p; the mean tensor comes from the
// per-element array when present (the same value, computed once)
__device__ __forceinline__ Geo patch_elem_geo(const Store& st, int t, const Elem& e, int v, double2 p) {
  double2 p0 = e.x == v ? p : st.xy[e.x];
  double2 p1 = e.y == v ? p : st.xy[e.y];
  double2 p2 = e.z == v ? p : st.xy[e.z];
  if (st.emet) {
    Geo g;
    g.x[0] = p0.x; g.y[0] = p0.y;
    g.x[1] = p1.x; g.y[1] = p1.y;
    g.x[2] = p2.x; g.y[2] = p2.y;
    Met m = st.emet[t];
    g.a = m.a;
    g.b = m.b;
    g.c = m.c;
    return g;
  }
  return make_geo(p0, p1, p2, st.met[e.x], st.met[e.y], st.met[e.z]);
}

// smallest q^2 over v's elements with v placed at p; valid = all areas positive
__device__ double patch_min_q2(const Store& st, int v, Hdr h, double2 p, bool& valid) {
  valid = true;
  double mn = 0.0;
  bool first = true;
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    Geo g = patch_elem_geo(st, t, e, v, p);
    if (!(area2(g) > 0.0)) valid = false;
    double q2 = qd2(g, st.qk);
    if (first || q2 < mn) mn = q2;
    first = false;
  }
  return mn;
}

__device__ double patch_q(const Store& st, int v, Hdr h, double2 p) {
  double s = 0.0;
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    s = s + qval(patch_elem_geo(st, t, e, v, p), st.qk);
  }
  return s;
}

// "first or smaller" running minimum, as in a serial loop over the row
__device__ __forceinline__ void run_min(double q, bool first, double& mn) {
  if (first || q < mn) mn = q;
}

__device__ bool smooth_laplace(Store st, int v) {
  Hdr h = st.hdr[v];
  double2 pv = st.xy[v];
  Met mv = st.met[v];
  double Ga = 0.0, Gb = 0.0, Gc = 0.0, rx = 0.0, ry = 0.0;
  for (int j = 0; j < h.y; ++j) {
    int w = st.nn[h.x + j];
    Met mw = st.met[w];
    double2 pw = st.xy[w];
    double ea = (mv.a + mw.a) * 0.5;
    double eb = (mv.b + mw.b) * 0.5;
    double ec = (mv.c + mw.c) * 0.5;
    double dx = pw.x - pv.x, dy = pw.y - pv.y;
    Ga = Ga + ea;
    Gb = Gb + eb;
    Gc = Gc + ec;
    rx = rx + (ea * dx + eb * dy);
    ry = ry + (eb * dx + ec * dy);
  }
  double det = Ga * Gc - Gb * Gb;
  double2 p = make_double2(pv.x + (Gc * rx - Gb * ry) / det, pv.y + (Ga * ry - Gb * rx) / det);
  // one pass over the patch: minimum q^2 at the old and at the new position
  double oldmin = 0.0, newmin = 0.0;
  bool vn = true;
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    Geo go = patch_elem_geo(st, t, e, v, pv);
    Geo gn = go;
    int k = slot_of(e, v);
    gn.x[0] = k == 0 ? p.x : go.x[0];
    gn.y[0] = k == 0 ? p.y : go.y[0];
    gn.x[1] = k == 1 ? p.x : go.x[1];
    gn.y[1] = k == 1 ? p.y : go.y[1];
    gn.x[2] = k == 2 ? p.x : go.x[2];
    gn.y[2] = k == 2 ? p.y : go.y[2];
    run_min(qd2(go, st.qk), i == 0, oldmin);
    if (!(area2(gn) > 0.0)) vn = false;
    run_min(qd2(gn, st.qk), i == 0, newmin);
  }
  if (vn && newmin >= oldmin) {
    st.xy[v] = p;
    return true;
  }
  return false;
}

// geometry with slot k moved to p
__device__ __forceinline__ Geo moved(const Geo& g, int k, double2 p) {
  Geo r = g;
  r.x[0] = k == 0 ? p.x : g.x[0];
  r.y[0] = k == 0 ? p.y : g.y[0];
  r.x[1] = k == 1 ? p.x : g.x[1];
  r.y[1] = k == 1 ? p.y : g.y[1];
  r.x[2] = k == 2 ? p.x : g.x[2];
  r.y[2] = k == 2 ? p.y : g.y[2];
  return r;
}

__device__ bool smooth_gradient(Store st, int v) {
  Hdr h = st.hdr[v];
  double2 pv = st.xy[v];
  // pass 1: gradient of Q_v, Q_v and the minimum q^2 at the current position
  double gx = 0.0, gy = 0.0, Qold = 0.0, oldmin = 0.0;
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    Geo g = patch_elem_geo(st, t, e, v, pv);
    double ex, ey;
    qgrad_x(g, slot_of(e, v), st.qk, ex, ey);
    gx = gx + ex;
    gy = gy + ey;
    Qold = Qold + qval(g, st.qk);
    run_min(qd2(g, st.qk), i == 0, oldmin);
  }
  if (gx == 0.0 && gy == 0.0) return false;
  double ax = fabs(gx), ay = fabs(gy);
  double nrm = ax < ay ? ay : ax;
  double dx = gx / nrm, dy = gy / nrm;
  double hh = 0.0;
  for (int j = 0; j < h.y; ++j) {
    double2 pw = st.xy[st.nn[h.x + j]];
    double hx = fabs(pw.x - pv.x), hy = fabs(pw.y - pv.y);
    double hj = hx < hy ? hy : hx;
    if (j == 0 || hj < hh) hh = hj;
  }
  // pass 2: the four trial steps h/2 .. h/16 together; the first acceptable wins
  double2 p[4];
  double step = hh;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    step = step * 0.5;
    p[k] = make_double2(pv.x + step * dx, pv.y + step * dy);
  }
  double mn[4] = {0.0, 0.0, 0.0, 0.0}, Q[4] = {0.0, 0.0, 0.0, 0.0};
  bool ok[4] = {true, true, true, true};
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    Elem e = st.tri[t];
    Geo g = patch_elem_geo(st, t, e, v, pv);
    int sl = slot_of(e, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Geo gk = moved(g, sl, p[k]);
      if (!(area2(gk) > 0.0)) ok[k] = false;
      run_min(qd2(gk, st.qk), i == 0, mn[k]);
      Q[k] = Q[k] + qval(gk, st.qk);
    }
  }
  int pick = -1;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (pick < 0 && ok[k] && mn[k] >= oldmin && Q[k] > Qold) pick = k;
  if (pick < 0) return false;
  // recompute the chosen point rather than index the trial array
  double sp = hh;
  for (int k = 0; k <= pick; ++k) sp = sp * 0.5;
  st.xy[v] = make_double2(pv.x + sp * dx, pv.y + sp * dy);
  return true;
}

// Min-max: ascent on the patch's smallest quality. The worst element (the
// smallest q, ties to the first in NE(v)) gives the direction, its gradient
// in x_v; when the second worst is within 1% (q2 <= 1.01 q1), the point
// nearest the origin on the segment between the two gradients. Normalised in
// the max-norm; steps h/2 .. h/16 as in the gradient step; the first step
// that keeps every area positive and raises the patch minimum of q^2
// strictly is taken.
__device__ bool smooth_minmax(Store st, int v) {
  Hdr h = st.hdr[v];
  double2 pv = st.xy[v];
  int i1 = -1, i2 = -1;
  double q1 = 0.0, q2 = 0.0;
  for (int i = 0; i < h.w; ++i) {
    int t = st.ne[h.z + i];
    double q = qval(patch_elem_geo(st, t, st.tri[t], v, pv), st.qk);
    if (i1 < 0 || q < q1) {
      i2 = i1;
      q2 = q1;
      i1 = i;
      q1 = q;
    } else if (i2 < 0 || q < q2) {
      i2 = i;
      q2 = q;
    }
  }
  if (i1 < 0) return false;
  int t1 = st.ne[h.z + i1];
  Elem e1 = st.tri[t1];
  double ax, ay;
  qgrad_x(patch_elem_geo(st, t1, e1, v, pv), slot_of(e1, v), st.qk, ax, ay);
  double gx = ax, gy = ay;
  if (i2 >= 0 && q2 <= q1 * 1.01) {
    int t2 = st.ne[h.z + i2];
    Elem e2 = st.tri[t2];
    double bx, by;
    qgrad_x(patch_elem_geo(st, t2, e2, v, pv), slot_of(e2, v), st.qk, bx, by);
    double ex = bx - ax, ey = by - ay;
    double den = ex * ex + ey * ey;
    if (den > 0.0) {
      double lam = -(ax * ex + ay * ey) / den;
      lam = lam < 0.0 ? 0.0 : (lam > 1.0 ? 1.0 : lam);
      gx = ax + lam * ex;
      gy = ay + lam * ey;
    }
  }
  if (gx == 0.0 && gy == 0.0) return false;
  double nx = fabs(gx), ny = fabs(gy);
  double nrm = nx < ny ? ny : nx;
  double dx = gx / nrm, dy = gy / nrm;
  double hh = 0.0;
  for (int j = 0; j < h.y; ++j) {
    double2 pw = st.xy[st.nn[h.x + j]];
    double hx = fabs(pw.x - pv.x), hy = fabs(pw.y - pv.y);
    double hj = hx < hy ? hy : hx;
    if (j == 0 || hj < hh) hh = hj;
  }
  bool vo;
  double oldmin = patch_min_q2(st, v, h, pv, vo);
  double step = hh;
  for (int k = 0; k < 4; ++k) {
    step = step * 0.5;
    double2 p = make_double2(pv.x + step * dx, pv.y + step * dy);
    bool vn;
    double newmin = patch_min_q2(st, v, h, p, vn);
    if (!vn || !(newmin > oldmin)) continue;
    st.xy[v] = p;
    return true;
  }
  return false;
}

template <int QK>
__global__ void k_smooth(Store st, const int* __restrict__ list, int n, int kind, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  int i = xtid();
  int status = -1;
  if (i < n) {
    int v = list[i];
    bool moved = kind == 0 ? smooth_laplace(st, v) : (kind == 1 ? smooth_gradient(st, v) : smooth_minmax(st, v));
    status = moved ? 2 : 1;
  }
  count_status(status, ctr);
}
template <int K, int QK>
__global__ void __launch_bounds__(256, 4) k_smooth_g(Store st, const int* __restrict__ list, int n, int* ctr);
void smooth_class(const Store& st, const int* list, int n, int kind, int* ctr, int lanes, hipStream_t s) {
  if (n <= 0) return;
  int nb = (int)(((int64_t)n * kG + kBlock - 1) / kBlock);
  if (lanes == kG && kind == 2)
    (st.qk ? k_smooth_g<2, 1> : k_smooth_g<2, 0>)<<<nb, kBlock, 0, s>>>(st, list, n, ctr);
  else if (lanes == kG && kind == 0)
    (st.qk ? k_smooth_g<0, 1> : k_smooth_g<0, 0>)<<<nb, kBlock, 0, s>>>(st, list, n, ctr);
  else if (lanes == kG)
    (st.qk ? k_smooth_g<1, 1> : k_smooth_g<1, 0>)<<<nb, kBlock, 0, s>>>(st, list, n, ctr);
  else
    (st.qk ? k_smooth<1> : k_smooth<0>)<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(st, list, n, kind, ctr);
}

// ---- lane groups: 8 lanes per vertex ----------------------------------------------------------
// A vertex's 1-ring is spread over a group of kG lanes: lane j owns the j-th
// neighbour and the j-th element of the vertex's sorted rows, loads them in
// parallel and keeps its element's geometry in registers. Sums run over the
// lanes in row order (one shuffle per term), so every FP64 sum has the same
// rounding sequence as a serial loop over the row. Vertices with more than
// kG neighbours or elements take the one-thread path on the group's lane 0.
struct Grp {
  int j;     // index in the group
  int base;  // first lane of the group in the wavefront
};
__device__ __forceinline__ Grp grp() {
  int l = __lane_id();
  return Grp{l & (kG - 1), l & ~(kG - 1)};
}
__device__ __forceinline__ double gget(double v, int k, const Grp& g) { return __shfl(v, g.base + k); }
__device__ __forceinline__ int gget(int v, int k, const Grp& g) { return __shfl(v, g.base + k); }
// serial sum acc = ((init + v_0) + v_1) + ... over lanes 0..n-1
__device__ __forceinline__ double gsum(double v, int n, const Grp& g) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kG; ++k) {
    double t = gget(v, k, g);
    if (k < n) acc = acc + t;
  }
  return acc;
}
// serial "first or smaller" minimum over lanes 0..n-1
__device__ __forceinline__ double gmin(double v, int n, const Grp& g) {
  double mn = 0.0;
#pragma unroll
  for (int k = 0; k < kG; ++k) {
    double t = gget(v, k, g);
    if (k < n && (k == 0 || t < mn)) mn = t;
  }
  return mn;
}
__device__ __forceinline__ bool gany(bool p, const Grp& g) {
  uint64_t b = __ballot(p);
  return ((b >> g.base) & 0xFFull) != 0;
}
__device__ __forceinline__ uint64_t gor64(uint64_t v, const Grp& g) {
#pragma unroll
  for (int d = 1; d < kG; d <<= 1) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo |= (uint32_t)__shfl_xor((int)lo, d);
    hi |= (uint32_t)__shfl_xor((int)hi, d);
    v = ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// one element of a vertex's patch, in stored order; slot k holds the vertex
struct PatchElem {
  double x0, y0, x1, y1, x2, y2;
  double a, b, c;  // mean tensor (stored order)
  int k;
};

// element t = e of v's patch; the mean tensor from the per-element array
// when present (the same value, computed once per phase), else from the
// three vertices
__device__ __forceinline__ PatchElem load_patch_elem(const Store& st, int t, const Elem& e, int v) {
  PatchElem pe;
  double2 p0 = st.xy[e.x], p1 = st.xy[e.y], p2 = st.xy[e.z];
  pe.x0 = p0.x; pe.y0 = p0.y;
  pe.x1 = p1.x; pe.y1 = p1.y;
  pe.x2 = p2.x; pe.y2 = p2.y;
  if (st.emet) {
    Met m = st.emet[t];
    pe.a = m.a;
    pe.b = m.b;
    pe.c = m.c;
  } else {
    Met m0 = st.met[e.x], m1 = st.met[e.y], m2 = st.met[e.z];
    pe.a = ((m0.a + m1.a) + m2.a) / 3.0;
    pe.b = ((m0.b + m1.b) + m2.b) / 3.0;
    pe.c = ((m0.c + m1.c) + m2.c) / 3.0;
  }
  pe.k = slot_of(e, v);
  return pe;
}

// the element's geometry with the patch vertex placed at p
__device__ __forceinline__ Geo patch_geo(const PatchElem& pe, double2 p) {
  Geo g;
  g.x[0] = pe.k == 0 ? p.x : pe.x0;
  g.y[0] = pe.k == 0 ? p.y : pe.y0;
  g.x[1] = pe.k == 1 ? p.x : pe.x1;
  g.y[1] = pe.k == 1 ? p.y : pe.y1;
  g.x[2] = pe.k == 2 ? p.x : pe.x2;
  g.y[2] = pe.k == 2 ? p.y : pe.y2;
  g.a = pe.a;
  g.b = pe.b;
  g.c = pe.c;
  return g;
}

// patch minimum of q^2 and validity with the vertex at p (lanes j < nw own elements)
__device__ __forceinline__ double gpatch_min(const PatchElem& pe, bool own, double2 p, int nw, const Grp& g,
                                             int qk, bool& valid) {
  double q2 = 0.0;
  bool bad = false;
  if (own) {
    Geo gg = patch_geo(pe, p);
    bad = !(area2(gg) > 0.0);
    q2 = qd2(gg, qk);
  }
  valid = !gany(bad, g);
  return gmin(q2, nw, g);
}

__device__ __forceinline__ double gpatch_q(const PatchElem& pe, bool own, double2 p, int nw, const Grp& g, int qk) {
  double q = own ? qval(patch_geo(pe, p), qk) : 0.0;
  return gsum(q, nw, g);
}

__device__ __forceinline__ bool smooth_group(Store& st, int v, Hdr h, int kind, const Grp& g) {
  double2 pv = st.xy[v];
  Met mv = st.met[v];
  bool ownn = g.j < h.y, owne = g.j < h.w;
  // row entries, then neighbour data and elements, then the elements'
  // vertex data, each level issued together (index 0 for an empty lane)
  int w = ownn ? st.nn[h.x + g.j] : -1;
  int t = owne ? st.ne[h.z + g.j] : -1;
  double2 pw = st.xy[max(w, 0)];
  Met mw = st.met[max(w, 0)];
  Elem e = st.tri[max(t, 0)];
  if (!ownn) {
    pw = make_double2(0.0, 0.0);
    mw = Met{0.0, 0.0, 0.0};
  }
  PatchElem pe = load_patch_elem(st, max(t, 0), e, v);
  if (!owne) pe = PatchElem{};
  double2 p;
  if (kind == 0) {
    double ea = (mv.a + mw.a) * 0.5;
    double eb = (mv.b + mw.b) * 0.5;
    double ec = (mv.c + mw.c) * 0.5;
    double dx = pw.x - pv.x, dy = pw.y - pv.y;
    // the five sums side by side, one lane's terms at a time (each sum keeps
    // the serial rounding sequence; holding all forty shuffled terms at once
    // would spill)
    double fx = ea * dx + eb * dy, fy = eb * dx + ec * dy;
    double Ga = 0.0, Gb = 0.0, Gc = 0.0, rx = 0.0, ry = 0.0;
#pragma unroll
    for (int k = 0; k < kG; ++k) {
      double ta = gget(ea, k, g), tb = gget(eb, k, g), tc = gget(ec, k, g), tx = gget(fx, k, g),
             ty = gget(fy, k, g);
      if (k < h.y) {
        Ga = Ga + ta;
        Gb = Gb + tb;
        Gc = Gc + tc;
        rx = rx + tx;
        ry = ry + ty;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    double det = Ga * Gc - Gb * Gb;
    p = make_double2(pv.x + (Gc * rx - Gb * ry) / det, pv.y + (Ga * ry - Gb * rx) / det);
    bool vo, vn;
    double oldmin = gpatch_min(pe, owne, pv, h.w, g, st.qk, vo);
    double newmin = gpatch_min(pe, owne, p, h.w, g, st.qk, vn);
    if (!(vn && newmin >= oldmin)) return false;
  } else if (kind == 1) {
    double ex = 0.0, ey = 0.0;
    if (owne) qgrad_x(patch_geo(pe, pv), pe.k, st.qk, ex, ey);
    double gx = 0.0, gy = 0.0;
#pragma unroll
    for (int k = 0; k < kG; ++k) {
      double tx = gget(ex, k, g), ty = gget(ey, k, g);
      if (k < h.w) {
        gx = gx + tx;
        gy = gy + ty;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (gx == 0.0 && gy == 0.0) return false;
    double ax = fabs(gx), ay = fabs(gy);
    double nrm = ax < ay ? ay : ax;
    double dx = gx / nrm, dy = gy / nrm;
    double hx = fabs(pw.x - pv.x), hy = fabs(pw.y - pv.y);
    double hh = gmin(hx < hy ? hy : hx, h.y, g);
    bool vo;
    double oldmin = gpatch_min(pe, owne, pv, h.w, g, st.qk, vo);
    double Qold = gpatch_q(pe, owne, pv, h.w, g, st.qk);
    double step = hh;
    bool ok = false;
    for (int k = 1; k <= 4 && !ok; ++k) {
      step = step * 0.5;
      p = make_double2(pv.x + step * dx, pv.y + step * dy);
      bool vn;
      double newmin = gpatch_min(pe, owne, p, h.w, g, st.qk, vn);
      if (!vn || !(newmin >= oldmin)) continue;
      if (!(gpatch_q(pe, owne, p, h.w, g, st.qk) > Qold)) continue;
      ok = true;
    }
    if (!ok) return false;
  } else {
    // min-max: the worst element (smallest q, ties to the first in NE(v)) and
    // the second worst, taken in row order as a serial loop takes them
    double q = owne ? qval(patch_geo(pe, pv), st.qk) : 0.0;
    int i1 = -1, i2 = -1;
    double q1 = 0.0, q2 = 0.0;
#pragma unroll
    for (int k = 0; k < kG; ++k) {
      double t = gget(q, k, g);
      if (k < h.w) {
        if (i1 < 0 || t < q1) {
          i2 = i1;
          q2 = q1;
          i1 = k;
          q1 = t;
        } else if (i2 < 0 || t < q2) {
          i2 = k;
          q2 = t;
        }
      }
    }
    if (i1 < 0) return false;
    double ex = 0.0, ey = 0.0;
    if (owne) qgrad_x(patch_geo(pe, pv), pe.k, st.qk, ex, ey);
    double ax = gget(ex, i1, g), ay = gget(ey, i1, g);
    double bx = gget(ex, max(i2, 0), g), by = gget(ey, max(i2, 0), g);
    double gx = ax, gy = ay;
    if (i2 >= 0 && q2 <= q1 * 1.01) {
      double fx = bx - ax, fy = by - ay;
      double den = fx * fx + fy * fy;
      if (den > 0.0) {
        double lam = -(ax * fx + ay * fy) / den;
        lam = lam < 0.0 ? 0.0 : (lam > 1.0 ? 1.0 : lam);
        gx = ax + lam * fx;
        gy = ay + lam * fy;
      }
    }
    if (gx == 0.0 && gy == 0.0) return false;
    double nx = fabs(gx), ny = fabs(gy);
    double nrm = nx < ny ? ny : nx;
    double dx = gx / nrm, dy = gy / nrm;
    double hx = fabs(pw.x - pv.x), hy = fabs(pw.y - pv.y);
    double hh = gmin(hx < hy ? hy : hx, h.y, g);
    bool vo;
    double oldmin = gpatch_min(pe, owne, pv, h.w, g, st.qk, vo);
    double step = hh;
    bool ok = false;
    for (int k = 0; k < 4 && !ok; ++k) {
      step = step * 0.5;
      p = make_double2(pv.x + step * dx, pv.y + step * dy);
      bool vn;
      double newmin = gpatch_min(pe, owne, p, h.w, g, st.qk, vn);
      if (!vn || !(newmin > oldmin)) continue;
      ok = true;
    }
    if (!ok) return false;
  }
  if (g.j == 0) st.xy[v] = p;
  return true;
}

// one kernel per smoothing kind (K = 0 plain, 1 gradient), each with its own
// register allocation
template <int K, int QK>
__global__ void __launch_bounds__(256, 4) k_smooth_g(Store st, const int* __restrict__ list, int n, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  Grp g = grp();
  int gid = (int)(((int64_t)xcd_block() * blockDim.x + threadIdx.x) / kG);
  int status = -1;
  if (gid < n) {
    int v = list[gid];
    Hdr h = st.hdr[v];
    if (h.y > kG || h.w > kG) {
      if (g.j == 0)
        status = (K == 0 ? smooth_laplace(st, v) : (K == 1 ? smooth_gradient(st, v) : smooth_minmax(st, v))) ? 2 : 1;
    } else {
      bool moved = smooth_group(st, v, h, K, g);
      if (g.j == 0) status = moved ? 2 : 1;
    }
  }
  count_status(status, ctr);
}
template __global__ void k_smooth_g<0, 0>(Store, const int*, int, int*);
template __global__ void k_smooth_g<0, 1>(Store, const int*, int, int*);
template __global__ void k_smooth_g<1, 0>(Store, const int*, int, int*);
template __global__ void k_smooth_g<2, 0>(Store, const int*, int, int*);
template __global__ void k_smooth_g<2, 1>(Store, const int*, int, int*);
template __global__ void k_smooth_g<1, 1>(Store, const int*, int, int*);

// ---- collapse with lane groups -----------------------------------------------------------------
// G lanes per member (G = kGC): small classes are made of the vertices that
// earlier rounds left, often of high degree, so the groups are wider here.
template <int G>
__device__ __forceinline__ Grp grp_of() {
  int l = __lane_id();
  return Grp{l & (G - 1), l & ~(G - 1)};
}
template <int G>
__device__ __forceinline__ bool gany_of(bool p, const Grp& g) {
  uint64_t b = __ballot(p);
  return ((b >> g.base) & ((1ull << G) - 1ull)) != 0;
}
template <int G>
__device__ __forceinline__ int collapse_group(const Store& st, int v, Hdr h, const OpArgs& a, const Commit& cm, int* ctr, const Grp& g) {
  bool ownn = g.j < h.y, owne = g.j < h.w;
  // loads by dependency level, each level issued together (index 0 stands
  // in for a lane with no neighbour or element): the member's own data and
  // its rows' entries; then each neighbour's round word and data and each
  // element; the deferral test comes after them
  uint64_t rv = a.rw[v];
  VRec rcv = st.vr[v];
  double2 pv = make_double2(rcv.x, rcv.y);
  Met mv{rcv.a, rcv.b, rcv.c};
  int tv = rcv.tag;
  int w = ownn ? st.nn[h.x + g.j] : -1;
  int t = owne ? st.ne[h.z + g.j] : -1;
  int ws = max(w, 0);
  uint64_t xw = a.rw[ws];
  VRec rcw = st.vr[ws];
  double2 pw = make_double2(rcw.x, rcw.y);
  Met mw{rcw.a, rcw.b, rcw.c};
  int tw = rcw.tag;
  Elem e = st.tri[max(t, 0)];
  bool beat = ownn && (xw & kRwAct) && (int)(xw & 0xFF) == a.cls && rw_beats(xw, w, rv, v);
  if (gany_of<G>(beat, g)) {
    if (g.j == 0) cm.nxt[v] = 1;
    return 0;
  }
  double L = INFINITY;
  bool cand = false;
  if (ownn) {
    if (!(tv & ~tw)) {
      L = len2(pv, mv, pw, mw);
      cand = L < a.L_low2;
    }
  } else {
    pw = make_double2(0.0, 0.0);
    mw = Met{0.0, 0.0, 0.0};
  }
  // element lane: ids and data of the element's other two vertices
  double2 q0 = make_double2(0.0, 0.0), q1 = q0;
  Met n0{0.0, 0.0, 0.0}, n1 = n0;
  int o0 = -1, o1 = -1, k = 0;
  if (!owne) e = make_int4(0, 0, 0, 0);
  if (owne) {
    k = slot_of(e, v);
    o0 = at(e, k == 2 ? 0 : k + 1);  // next after v
    o1 = at(e, k == 0 ? 2 : k - 1);  // before v
    VRec r0 = st.vr[o0], r1 = st.vr[o1];
    q0 = make_double2(r0.x, r0.y);
    q1 = make_double2(r1.x, r1.y);
    n0 = Met{r0.a, r0.b, r0.c};
    n1 = Met{r1.a, r1.b, r1.c};
  }
  double lastL = -INFINITY;
  int lastU = -1, u = -1;
  for (;;) {
    // group minimum of (L, w) over candidates after (lastL, lastU)
    bool after = cand && (L > lastL || (L == lastL && w > lastU));
    double bL = after ? L : INFINITY;
    int bU = after ? w : INT_MAX;
    int bj = after ? g.j : -1;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      double oL = __shfl_xor(bL, d);
      int oU = __shfl_xor(bU, d);
      int oj = __shfl_xor(bj, d);
      if (oL < bL || (oL == bL && oU < bU)) {
        bL = oL;
        bU = oU;
        bj = oj;
      }
    }
    if (bj < 0) break;
    // the candidate's data from the lane that owns it
    double2 pu = make_double2(gget(pw.x, bj, g), gget(pw.y, bj, g));
    Met mu{gget(mw.a, bj, g), gget(mw.b, bj, g), gget(mw.c, bj, g)};
    bool bad = false;
    if (owne && o0 != bU && o1 != bU) {
      // element (u, o0, o1) in cyclic order, rotated smallest id first
      int r;  // rotation: which of (u, o0, o1) comes first
      if (bU < o0 && bU < o1) r = 0;
      else if (o0 < bU && o0 < o1) r = 1;
      else r = 2;
      double2 c0 = r == 0 ? pu : (r == 1 ? q0 : q1);
      double2 c1 = r == 0 ? q0 : (r == 1 ? q1 : pu);
      double2 c2 = r == 0 ? q1 : (r == 1 ? pu : q0);
      Met d0 = r == 0 ? mu : (r == 1 ? n0 : n1);
      Met d1 = r == 0 ? n0 : (r == 1 ? n1 : mu);
      Met d2 = r == 0 ? n1 : (r == 1 ? mu : n0);
      Geo gg = make_geo(c0, c1, c2, d0, d1, d2);
      bad = !(area2(gg) > 0.0) || !(qd2(gg, st.qk) >= a.qmin2);
    }
    if (!gany_of<G>(bad, g)) {
      u = bU;
      break;
    }
    lastL = bL;
    lastU = bU;
  }
  if (u < 0) return 1;
  if (owne) {
    Elem ne;
    if (o0 == u || o1 == u) {
      ne = e;
      ne.w = 0;
    } else {
      int3 r3 = rot_min(u, o0, o1);
      ne = make_int4(r3.x, r3.y, r3.z, 1);
    }
    st.tri[t] = ne;
  }
  if (ownn) claim_row(cm, w, v);
  if (g.j == 0) {
    st.valive[v] = 0;
    stamp(cm, v, -(u + 1), h.z, h.w);
    mark_target(cm, u, v, h.z, h.w);
  }
  return 2;
}

template <int G, int QK>
__global__ void __launch_bounds__(256, 5) k_collapse_g(Store st, const int* __restrict__ list, int n, OpArgs a,
                                                    Commit cm, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  if (room_failed(ctr)) return;
  Grp g = grp_of<G>();
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[C_STAGE] = 0;  // the commit's fallback staging
  int gid = (int)(((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G);
  int status = -1;
  if (gid < n) {
    int v = list[gid];
    Hdr h = st.hdr[v];
    if (h.y > G || h.w > G) {
      if (g.j == 0) status = collapse_one(st, v, a, cm, ctr);
    } else {
      int r = collapse_group<G>(st, v, h, a, cm, ctr, g);
      if (g.j == 0) status = r;
    }
  }
  count_status(status, ctr, true);
}
template __global__ void k_collapse_g<8, 0>(Store, const int*, int, OpArgs, Commit, int*);
template __global__ void k_collapse_g<8, 1>(Store, const int*, int, OpArgs, Commit, int*);
template __global__ void k_collapse_g<16, 0>(Store, const int*, int, OpArgs, Commit, int*);
template __global__ void k_collapse_g<16, 1>(Store, const int*, int, OpArgs, Commit, int*);

// ---- flips with lane groups -----------------------------------------------------------------------
// Lane j owns the member's j-th element T1 = (v, w, a) (cyclic from v): the
// edge (v, w) and its data. The element across that edge, T2, is the one
// whose vertex before v is w; the lane holding it hands over its id, its
// other vertex b and its quality. Each lane then evaluates the flip of its
// edge; the group keeps the largest new minimum quality, ties to the smaller
// w, as the one-thread scan does.
template <int G>
__device__ __forceinline__ int flip_group(const Store& st, int v, Hdr h, const OpArgs& a, const Commit& cm,
                                          const Grp& g) {
  bool ownn = g.j < h.y, owne = g.j < h.w;
  // loads by dependency level, each level issued together: the member's
  // data and its rows' entries, then the neighbours' round words and the
  // elements; the deferral test comes after them
  uint64_t rv = a.rw[v];
  VRec rcv = st.vr[v];
  double2 pv = make_double2(rcv.x, rcv.y);
  Met mv{rcv.a, rcv.b, rcv.c};
  int y = ownn ? st.nn[h.x + g.j] : -1;
  int T1 = owne ? st.ne[h.z + g.j] : -1;
  uint64_t ry = a.rw[max(y, 0)];
  Elem e1 = st.tri[max(T1, 0)];
  bool beat = ownn && (ry & kRwAct) && (int)(ry & 0xFF) == a.cls && rw_beats(ry, y, rv, v);
  if (gany_of<G>(beat, g)) {
    if (g.j == 0) cm.nxt[v] = 1;
    return 0;
  }
  int k1 = 0, w = -1, av = -1;
  double2 pw = make_double2(0.0, 0.0), pa = pw;
  Met mw{0.0, 0.0, 0.0}, ma = mw;
  if (owne) {
    k1 = slot_of(e1, v);
    w = at(e1, k1 == 2 ? 0 : k1 + 1);
    av = at(e1, k1 == 0 ? 2 : k1 - 1);
    VRec rcw = st.vr[w], rca = st.vr[av];
    pw = make_double2(rcw.x, rcw.y);
    mw = Met{rcw.a, rcw.b, rcw.c};
    pa = make_double2(rca.x, rca.y);
    ma = Met{rca.a, rca.b, rca.c};
  }
  // quality of T1 in its stored order (slot k1 holds v, then w, then a)
  double q1 = 0.0;
  if (owne) {
    double2 s0 = k1 == 0 ? pv : (k1 == 1 ? pa : pw);
    double2 s1 = k1 == 1 ? pv : (k1 == 2 ? pa : pw);
    double2 s2 = k1 == 2 ? pv : (k1 == 0 ? pa : pw);
    Met n0 = k1 == 0 ? mv : (k1 == 1 ? ma : mw);
    Met n1 = k1 == 1 ? mv : (k1 == 2 ? ma : mw);
    Met n2 = k1 == 2 ? mv : (k1 == 0 ? ma : mw);
    q1 = qd2(make_geo(s0, s1, s2, n0, n1, n2), st.qk);
  }
  // the lane whose element has w before v holds T2
  int j2 = -1;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    int pq = gget(av, q, g);
    if (j2 < 0 && owne && q < h.w && pq == w) j2 = q;
  }
  int src = g.base + (j2 >= 0 ? j2 : 0);
  int T2 = __shfl(T1, src);
  int bv = __shfl(w, src);
  double2 pb = make_double2(__shfl(pw.x, src), __shfl(pw.y, src));
  Met mb{__shfl(mw.a, src), __shfl(mw.b, src), __shfl(mw.c, src)};
  double q2 = __shfl(q1, src);
  bool cand = owne && j2 >= 0;
  double nmin = 0.0;
  if (cand) {
    // (v, b, a) and (w, a, b), each rotated smallest id first
    int r1 = (v < bv && v < av) ? 0 : ((bv < v && bv < av) ? 1 : 2);
    double2 c0 = r1 == 0 ? pv : (r1 == 1 ? pb : pa);
    double2 c1 = r1 == 0 ? pb : (r1 == 1 ? pa : pv);
    double2 c2 = r1 == 0 ? pa : (r1 == 1 ? pv : pb);
    Met d0 = r1 == 0 ? mv : (r1 == 1 ? mb : ma);
    Met d1 = r1 == 0 ? mb : (r1 == 1 ? ma : mv);
    Met d2 = r1 == 0 ? ma : (r1 == 1 ? mv : mb);
    Geo gv = make_geo(c0, c1, c2, d0, d1, d2);
    int r2 = (w < av && w < bv) ? 0 : ((av < w && av < bv) ? 1 : 2);
    double2 e0 = r2 == 0 ? pw : (r2 == 1 ? pa : pb);
    double2 e1p = r2 == 0 ? pa : (r2 == 1 ? pb : pw);
    double2 e2 = r2 == 0 ? pb : (r2 == 1 ? pw : pa);
    Met f0 = r2 == 0 ? mw : (r2 == 1 ? ma : mb);
    Met f1 = r2 == 0 ? ma : (r2 == 1 ? mb : mw);
    Met f2 = r2 == 0 ? mb : (r2 == 1 ? mw : ma);
    Geo gw = make_geo(e0, e1p, e2, f0, f1, f2);
    if (!(area2(gv) > 0.0) || !(area2(gw) > 0.0)) {
      cand = false;
    } else {
      double qv = qd2(gv, st.qk), qw = qd2(gw, st.qk);
      nmin = qw < qv ? qw : qv;
      double omin = q2 < q1 ? q2 : q1;
      cand = nmin > omin;
    }
  }
  // the best candidate: largest new minimum, ties to the smaller w
  double bq = cand ? nmin : -INFINITY;
  int bw = cand ? w : INT_MAX;
  int bj = cand ? g.j : -1;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    double oq = __shfl_xor(bq, d);
    int ow = __shfl_xor(bw, d);
    int oj = __shfl_xor(bj, d);
    if (oj >= 0 && (bj < 0 || oq > bq || (oq == bq && ow < bw))) {
      bq = oq;
      bw = ow;
      bj = oj;
    }
  }
  if (bj < 0) return 1;
  if (g.j == bj) {
    int lo = min(T1, T2), hi = max(T1, T2);
    int3 tv = rot_min(v, bv, av), tw = rot_min(w, av, bv);
    st.tri[lo] = make_int4(tv.x, tv.y, tv.z, 1);
    st.tri[hi] = make_int4(tw.x, tw.y, tw.z, 1);
    stamp(cm, v, lo, hi, 0);
    mark_target(cm, av, lo, hi, -1);
    mark_target(cm, bv, lo, hi, -1);
    claim_row(cm, v, v);
    claim_row(cm, w, v);
    claim_row(cm, av, v);
    claim_row(cm, bv, v);
  }
  return 2;
}

template <int G, int QK>
__global__ void __launch_bounds__(256) k_flip_g(Store st, const int* __restrict__ list, int n, OpArgs a, Commit cm,
                                                int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  if (room_failed(ctr)) return;
  Grp g = grp_of<G>();
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[C_STAGE] = 0;  // the commit's fallback staging
  int gid = (int)(((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G);
  int status = -1;
  if (gid < n) {
    int v = list[gid];
    Hdr h = st.hdr[v];
    if (h.y > G || h.w > G) {
      if (g.j == 0) status = flip_one(st, v, a, cm, ctr);
    } else {
      int r = flip_group<G>(st, v, h, a, cm, g);
      if (g.j == 0) status = r;
    }
  }
  count_status(status, ctr, true);
}
void flip_class_g(const Store& st, const int* list, int n, OpArgs a, Commit cm, int* ctr, hipStream_t s) {
  if (n > 0) (st.qk ? k_flip_g<16, 1> : k_flip_g<16, 0>)<<<(int)(((int64_t)n * 16 + kBlock - 1) / kBlock), kBlock, 0, s>>>(
      st, list, n, a, cm, ctr);
}

// A small class in one block: the operation (collapse or flips on groups of
// kGC lanes per member), a block barrier, then the commit of the same
// members. Every thread reaches every barrier.
template <bool F>
__device__ __forceinline__ void class_body(const Store& st, const int* __restrict__ list, int n, const OpArgs& a,
                                           const Commit& cm, int* ctr, CommitLds& L) {
  int tid = (int)threadIdx.x;
  if (tid == 0) ctr[C_STAGE] = 0;  // the commit's fallback staging
  Grp g = grp_of<kGC>();
  for (int p0 = 0; p0 < n; p0 += kBlock / kGC) {
    int gid = p0 + tid / kGC;
    int status = -1;
    if (gid < n) {
      int v = list[gid];
      Hdr h = st.hdr[v];
      if (h.y > kGC || h.w > kGC) {
        if (g.j == 0) status = F ? flip_one(st, v, a, cm, ctr) : collapse_one(st, v, a, cm, ctr);
      } else {
        int r = F ? flip_group<kGC>(st, v, h, a, cm, g) : collapse_group<kGC>(st, v, h, a, cm, ctr, g);
        if (g.j == 0) status = r;
      }
    }
    count_status(status, ctr);
  }
  __syncthreads();
  for (int base = 0; base < n; base += kBlock) commit_chunk<F>(st, list, base, min(kBlock, n - base), cm, ctr, L);
}

// one small class, one launch instead of two
template <bool F, int QK>
__global__ void __launch_bounds__(256) k_class_small(Store st, const int* __restrict__ list, int n, OpArgs a,
                                                     Commit cm, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  __shared__ CommitLds L;
  if (room_failed_block(ctr)) return;
  class_body<F>(st, list, n, a, cm, ctr, L);
}
void class_small(const Store& st, const int* list, int n, OpArgs a, Commit cm, int kind, int* ctr, hipStream_t s) {
  if (n <= 0) return;
  if (kind)
    (st.qk ? k_class_small<true, 1> : k_class_small<true, 0>)<<<1, kBlock, 0, s>>>(st, list, n, a, cm, ctr);
  else
    (st.qk ? k_class_small<false, 1> : k_class_small<false, 0>)<<<1, kBlock, 0, s>>>(st, list, n, a, cm, ctr);
}

// Every class of a round in one block, one after the other (a round whose
// classes are all small): class c takes epoch cm.epoch + c and its size and
// offset from the colouring's counters. One launch per round instead of one
// per class, and the block's caches stay warm from class to class.
template <bool F, int QK>
__global__ void __launch_bounds__(256) k_round_small(Store st, const int* __restrict__ cls, int ncol, OpArgs a,
                                                     Commit cm, int* ctr) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  __shared__ CommitLds L;
  int epoch0 = cm.epoch;
  bool dev = ncol < 0;
  if (dev) {
    if (ctr[C_DSTOP]) return;
    ncol = ctr[C_NCOL];
    epoch0 = ctr[C_DEPOCH];
    __syncthreads();  // every thread has read the counters before they change
    if (threadIdx.x == 0) {
      ctr[C_DEPOCH0] = epoch0;
      ctr[C_DEPOCH] = epoch0 + max(ncol, 0);
    }
  }
  for (int c = 0; c < ncol; ++c) {
    // a commit of this block may have run out of room: stop, the host
    // rebuilds the rows and runs the remaining classes
    if (room_failed_block(ctr)) return;
    int n = ctr[C_HIST + c], off = ctr[C_OFF + c];
    if (n == 0) continue;
    Commit cc = cm;
    cc.epoch = epoch0 + c;
    OpArgs ac = a;
    ac.cls = c;
    class_body<F>(st, cls + off, n, ac, cc, ctr, L);
  }
}
void round_small(const Store& st, const int* cls, int ncol, OpArgs a, Commit cm, int kind, int* ctr, hipStream_t s) {
  if (ncol == 0) return;
  if (kind)
    (st.qk ? k_round_small<true, 1> : k_round_small<true, 0>)<<<1, kBlock, 0, s>>>(st, cls, ncol, a, cm, ctr);
  else
    (st.qk ? k_round_small<false, 1> : k_round_small<false, 0>)<<<1, kBlock, 0, s>>>(st, cls, ncol, a, cm, ctr);
}

// ---- adjoint with lane groups ---------------------------------------------------------------------
template <int QK>
__global__ void __launch_bounds__(256) k_adjoint_g(Store st, double* __restrict__ dQdx, double* __restrict__ dQdM) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  Grp g = grp();
  int v = (int)(((int64_t)xcd_block() * blockDim.x + threadIdx.x) / kG);
  if (v >= st.V) return;
  Hdr h = st.hdr[v];
  double gx = 0.0, gy = 0.0, ga = 0.0, gb = 0.0, gc = 0.0;
  for (int c0 = 0; c0 < h.w; c0 += kG) {
    int nw = min(kG, h.w - c0);
    double ex = 0.0, ey = 0.0, da = 0.0, db = 0.0, dc = 0.0;
    if (g.j < nw) {
      Elem e = st.tri[st.ne[h.z + c0 + g.j]];
      Geo gg = geo_of(st, e);
      qgrad_x(gg, slot_of(e, v), st.qk, ex, ey);
      qgrad_m(gg, st.qk, da, db, dc);
      da = da / 3.0;
      db = db / 3.0;
      dc = dc / 3.0;
    }
#pragma unroll
    for (int k = 0; k < kG; ++k) {
      double tx = gget(ex, k, g), ty = gget(ey, k, g), ta = gget(da, k, g), tb = gget(db, k, g),
             tc = gget(dc, k, g);
      if (k < nw) {
        gx = gx + tx;
        gy = gy + ty;
        ga = ga + ta;
        gb = gb + tb;
        gc = gc + tc;
      }
    }
  }
  if (g.j == 0) {
    if (dQdx) {
      dQdx[2 * v] = gx;
      dQdx[2 * v + 1] = gy;
    }
    if (dQdM) {
      dQdM[3 * v] = ga;
      dQdM[3 * v + 1] = gb;
      dQdM[3 * v + 2] = gc;
    }
  }
}

// ---- quality functional and adjoint (Sec. 2.2) --------------------------------------------------
constexpr int QB = 256;

template <int QK>
__global__ void k_quality(Store st, double* __restrict__ psum, double* __restrict__ pmin) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  __shared__ double ls[QB], lm[QB];
  double s = 0.0, mn = INFINITY;
  for (int t = gtid(); t < st.T; t += gstride()) {
    Elem e = st.tri[t];
    if (!e.w) continue;
    double q = qval(geo_of(st, e), st.qk);
    s = s + q;
    mn = q < mn ? q : mn;
  }
  ls[threadIdx.x] = s;
  lm[threadIdx.x] = mn;
  __syncthreads();
  for (int d = QB / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + d];
      double o = lm[threadIdx.x + d];
      lm[threadIdx.x] = o < lm[threadIdx.x] ? o : lm[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = ls[0];
    pmin[blockIdx.x] = lm[0];
  }
}
__global__ void k_quality_final(const double* __restrict__ psum, const double* __restrict__ pmin, int np,
                                double* __restrict__ out) {
  __shared__ double ls[QB], lm[QB];
  double s = 0.0, mn = INFINITY;
  for (int i = threadIdx.x; i < np; i += QB) {
    s = s + psum[i];
    mn = pmin[i] < mn ? pmin[i] : mn;
  }
  ls[threadIdx.x] = s;
  lm[threadIdx.x] = mn;
  __syncthreads();
  for (int d = QB / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + d];
      double o = lm[threadIdx.x + d];
      lm[threadIdx.x] = o < lm[threadIdx.x] ? o : lm[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ls[0];
    out[1] = lm[0];
  }
}
// one block per mesh of a batch: Q and qmin of each mesh's element range
template <int QK>
__global__ void k_quality_mesh(Store st, double* __restrict__ out) {
  st.qk = QK;  // the functional as a constant: one instantiation per kind
  __shared__ double ls[QB], lm[QB];
  int i = blockIdx.x;
  int lo = st.tbase[i], hi = st.tbase[i] + st.tused[i];
  double s = 0.0, mn = INFINITY;
  for (int t = lo + (int)threadIdx.x; t < hi; t += QB) {
    Elem e = st.tri[t];
    if (!e.w) continue;
    double q = qval(geo_of(st, e), st.qk);
    s = s + q;
    mn = q < mn ? q : mn;
  }
  ls[threadIdx.x] = s;
  lm[threadIdx.x] = mn;
  __syncthreads();
  for (int d = QB / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + d];
      double o = lm[threadIdx.x + d];
      lm[threadIdx.x] = o < lm[threadIdx.x] ? o : lm[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * i] = ls[0];
    out[2 * i + 1] = lm[0];
  }
}
void quality_per_mesh(const Store& st, double* out, hipStream_t s) {
  (st.qk ? k_quality_mesh<1> : k_quality_mesh<0>)<<<st.B, QB, 0, s>>>(st, out);
}

void quality_sum(const Store& st, double* psum, double* pmin, int nparts, double* out2, hipStream_t s) {
  (st.qk ? k_quality<1> : k_quality<0>)<<<nparts, QB, 0, s>>>(st, psum, pmin);
  k_quality_final<<<1, QB, 0, s>>>(psum, pmin, nparts, out2);
}

void quality_adjoint(const Store& st, double* dQdx, double* dQdM, hipStream_t s) {
  (st.qk ? k_adjoint_g<1> : k_adjoint_g<0>)<<<(int)(((int64_t)st.V * kG + kBlock - 1) / kBlock), kBlock, 0, s>>>(
      st, dQdx, dQdM);
}

__global__ void k_fp64_probe(const double* __restrict__ a, const double* __restrict__ b, int n,
                             double* __restrict__ q, double* __restrict__ r) {
  for (int i = gtid(); i < n; i += gstride()) {
    q[i] = a[i] / b[i];
    r[i] = sqrt(a[i]);
  }
}
void fp64_probe(const double* a, const double* b, int n, double* q, double* r, hipStream_t s) {
  k_fp64_probe<<<grid_for(n), kBlock, 0, s>>>(a, b, n, q, r);
}

}  // namespace pm
