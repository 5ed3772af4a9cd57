// C ABI and host-side phase drivers: round loops, colour-class sequencing,
// commit points, compaction and store growth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <initializer_list>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pm.h"
#include "kern.hpp"
#include "blocks.hpp"

using namespace pm;

namespace {

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

// per-kernel HIP-event timing
struct Prof {
  uint32_t mask = 0;
  struct Rec {
    int k;
    hipEvent_t a, b;
    int64_t units;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> open;
  double ms[PM_K_COUNT] = {};
  int64_t launches[PM_K_COUNT] = {};
  int64_t units[PM_K_COUNT] = {};
};

struct pm_mesh {
  hipStream_t s = nullptr;
  hipStream_t cap_s = nullptr;  // private stream that graph captures are recorded on
  // device-driven rounds: instantiated graphs, by the bytes of their launch arguments
  std::vector<std::pair<std::string, hipGraphExec_t>> dr_graphs;
  int dev = 0;                // device current at creation
  double* scratch = nullptr;  // that device's copy of the no-allocation scratch array
  Prof prof;
  Store st;
  uint64_t seed = 0;
  double slack = 2.0;
  std::string err;
  int* ctr = nullptr;   // device counters
  int* hctr = nullptr;  // pinned mirror
  double* hq = nullptr; // pinned doubles
  int* haux = nullptr;   // pinned ints for small read-backs (upper half: staged uploads)
  hipEvent_t up_ev = nullptr;  // the last staged upload's copy
  // scratch
  DBuf<int> listA, listB, jpU0, jpU1, cls, vt0, vt1, vt2, vt3, vt4, tt0, tt1, tt2, partial, mid;
  DBuf<uint8_t> nxt, u8tmp;
  DBuf<Met> emet;   // smoothing: per-element mean tensors
  DBuf<VRec> vr;    // coarsening and swapping: vertex records
  DBuf<int> sflag, spos, ctab, ctabs, spart;  // ordered selection and stable class lists
  DBuf<int> stage;       // commit: fallback staging
  DBuf<int> touch, seen; // small rounds: rows rebuilt, selection stamps
  DBuf<int> jpB;         // JP: the neighbour each waiting vertex waits for
  int sel_mark = 0;      // selection stamp, one per small round
  DBuf<int4> ops;        // commit: operation records
  DBuf<uint64_t> own;    // commit: row owner keys
  DBuf<uint64_t> tk;     // commit: collapse-target counts
  DBuf<int4> tgt;        // commit: collapse-target records
  int epoch = 0;         // commit epoch, one per class
  DBuf<double> qpart;
  DBuf<double> upd;  // pm_mesh_update: the previous coordinates and metric
  DBuf<uint64_t> rw;  // round words (priority, active, colour) per vertex
  DBuf<uint64_t> seeds;  // device-driven rounds: the stream seed of every round of the phase
  // mesh ranges (host mirror of Store::vbase/vused/tbase/tused)
  std::vector<int> vbase, vused, tbase, tused;
  int* ranges = nullptr;  // device: vbase[B+1], vused[B], tbase[B+1], tused[B]
  int* mdone = nullptr;   // device: per-mesh "refinement finished" flags
  DBuf<int> rtmp;         // per-mesh scratch (sums, new bases)
  pm_tuning tune{};      // kernel shapes of the current call (zeros: defaults)
  double headroom = 3.0;  // pool and staging room, a multiple of the live entries
  double stage_scale = 1.0;  // grows when the staging area ran out
  int recoveries = 0;     // row rebuilds after running out of room, in the current phase
  // Algorithm 1's loop state (pm_adapt): outer iteration, next phase, whether
  // the iteration has changed the mesh
  int ad_iter = 0, ad_phase = 1, ad_changed = 0;
  int64_t peak_bytes = 0, cur_bytes = 0;
  // caller's device memory provider (pm_options.allocator at creation), and
  // the byte count of each block it handed out
  pm_allocator va{};
  std::unordered_map<void*, size_t> va_live;
  int jp_last = 8;    // JP iterations the last colouring took
  int class_seq = 0;  // class-list calls so far (the wide-colour flag's value)
  // elements change only in coarsening, refinement and swapping: each call
  // starts a new topology version; the per-element tensors are kept for one
  uint64_t topo = 1, emet_topo = 0;
};

namespace {

// message of the last failed pm_mesh_create on this thread (no handle survives it)
thread_local std::string g_create_err;

pm_status fail(pm_mesh* m, pm_status st, const std::string& msg) {
  if (m) m->err = msg;
  return st;
}

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      return fail(m, PM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define TRY(x)                      \
  do {                              \
    pm_status r_ = (x);             \
    if (r_ != PM_OK) return r_;     \
  } while (0)

// Device blocks are recycled through a process-wide cache keyed by device,
// stream and size. A block freed on a stream is handed out again only on the
// same stream, whose order makes the reuse safe without a wait, so handles
// and phase scratch that come and go skip the driver's allocation and free
// (each a synchronising call of tens of microseconds or more). Blocks up to
// twice the request are reused; past kCacheMax cached bytes a freed block is
// returned to the driver, and a failed allocation first empties the cache.
struct CacheKey {
  int dev;
  uintptr_t stream;
  size_t bytes;
  bool operator<(const CacheKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (stream != o.stream) return stream < o.stream;
    return bytes < o.bytes;
  }
};
constexpr size_t kCacheMax = 32ull << 30;
std::mutex g_cache_mu;
std::multimap<CacheKey, void*> g_cache_free;
std::map<void*, CacheKey> g_cache_live;
size_t g_cache_bytes = 0;

void cache_drop_all() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : g_cache_free) (void)hipFree(kv.second);
  g_cache_free.clear();
  g_cache_bytes = 0;
}

// *got: the size of the block handed out (a reused block may be larger)
hipError_t cache_get(hipStream_t s, void** p, size_t bytes, size_t* got) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  CacheKey want{dev, (uintptr_t)s, bytes};
  *got = bytes;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache_free.lower_bound(want);
    if (it != g_cache_free.end() && it->first.dev == dev && it->first.stream == want.stream &&
        it->first.bytes <= 2 * bytes) {
      *p = it->second;
      *got = it->first.bytes;
      g_cache_bytes -= it->first.bytes;
      g_cache_live[*p] = it->first;
      g_cache_free.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cache_drop_all();
    e = hipMalloc(p, bytes);
    if (e != hipSuccess) return e;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache_live[*p] = want;
  return hipSuccess;
}

// returns the block's size (0 if it is not a cache block)
size_t cache_put(void* p) {
  std::unique_lock<std::mutex> lk(g_cache_mu);
  auto it = g_cache_live.find(p);
  if (it == g_cache_live.end()) return 0;
  CacheKey k = it->second;
  g_cache_live.erase(it);
  if (g_cache_bytes + k.bytes > kCacheMax) {
    lk.unlock();
    (void)hipFree(p);
    return k.bytes;
  }
  g_cache_free.insert({k, p});
  g_cache_bytes += k.bytes;
  return k.bytes;
}

template <class T>
pm_status dalloc(pm_mesh* m, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (m->va.alloc) {
    void* q = m->va.alloc(n * sizeof(T), (void*)m->s, m->va.user);
    if (!q) return fail(m, PM_E_NOMEM, "the caller's allocator refused " + std::to_string(n * sizeof(T)) + " bytes");
    m->va_live[q] = n * sizeof(T);
    *p = (T*)q;
  } else {
    size_t got = 0;
    hipError_t e = cache_get(m->s, (void**)p, n * sizeof(T), &got);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(m, PM_E_NOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    m->cur_bytes += (int64_t)got;
    m->peak_bytes = std::max(m->peak_bytes, m->cur_bytes);
    return PM_OK;
  }
  m->cur_bytes += (int64_t)(n * sizeof(T));
  m->peak_bytes = std::max(m->peak_bytes, m->cur_bytes);
  return PM_OK;
}
// Pinned host blocks (the counter mirror and the quality read-back) are kept
// in a process-wide free list: pinning memory is a slow driver call.
constexpr int kAuxInts = 16384;  // pinned room for small read-backs beside the counters
constexpr size_t kPinnedBytes = C_COUNT * sizeof(int) + 64 * sizeof(double) + kAuxInts * sizeof(int);
std::mutex g_pinned_mu;
std::vector<void*> g_pinned_free;
bool pinned_get(pm_mesh* m) {
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      p = g_pinned_free.back();
      g_pinned_free.pop_back();
    }
  }
  if (!p && hipHostMalloc(&p, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  m->hctr = (int*)p;
  m->hq = (double*)((char*)p + C_COUNT * sizeof(int));
  m->haux = (int*)((char*)p + C_COUNT * sizeof(int) + 64 * sizeof(double));
  return true;
}
void pinned_put(pm_mesh* m) {
  if (!m->hctr) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free.push_back(m->hctr);
  m->hctr = nullptr;
  m->hq = nullptr;
  m->haux = nullptr;
}

template <class T>
void dfree(pm_mesh* m, T*& p, size_t n) {
  if (p && m->va.release) {
    auto it = m->va_live.find((void*)p);
    if (it != m->va_live.end()) {
      m->va.release((void*)p, it->second, (void*)m->s, m->va.user);
      m->cur_bytes -= (int64_t)it->second;
      m->va_live.erase(it);
    }
  } else if (p) {
    m->cur_bytes -= (int64_t)cache_put(p);  // the block's real size
  }
  p = nullptr;
}

// grow-only scratch; contents are not preserved; zero = clear new memory.
// Freed blocks go back to the cache of this stream, where only later work of
// the same stream can take them, so a first allocation needs no wait; a
// replaced block is still waited for.
template <class T>
pm_status ensure(pm_mesh* m, DBuf<T>& b, size_t n, bool zero = false) {
  if (b.n >= n && b.p) return PM_OK;
  if (b.p) HIPCHK(hipStreamSynchronize(m->s));
  dfree(m, b.p, b.n);
  b.n = 0;
  size_t want = std::max<size_t>(n + n / 4, 64);
  TRY(dalloc(m, &b.p, want));
  b.n = want;
  if (zero) HIPCHK(hipMemsetAsync(b.p, 0, want * sizeof(T), m->s));
  return PM_OK;
}

pm_status sync(pm_mesh* m) {
  HIPCHK(hipStreamSynchronize(m->s));
  return PM_OK;
}

hipEvent_t prof_event(pm_mesh* m) {
  if (m->prof.pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = m->prof.pool.back();
  m->prof.pool.pop_back();
  return e;
}

// time one launch (or launch sequence) of kernel k when its bit is enabled
template <class F>
void timed(pm_mesh* m, int k, int64_t units, F&& launch) {
  if (!(m->prof.mask & (1u << k))) {
    launch();
    return;
  }
  hipEvent_t a = prof_event(m), b = prof_event(m);
  if (a) (void)hipEventRecord(a, m->s);
  launch();
  if (b) (void)hipEventRecord(b, m->s);
  if (a && b) m->prof.open.push_back({k, a, b, units});
}

// fold finished event pairs into the totals (call after a stream sync)
void prof_flush(pm_mesh* m) {
  for (auto& r : m->prof.open) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      m->prof.ms[r.k] += t;
      m->prof.launches[r.k] += 1;
      m->prof.units[r.k] += r.units;
    }
    m->prof.pool.push_back(r.a);
    m->prof.pool.push_back(r.b);
  }
  m->prof.open.clear();
}

// the counters a round reads back: pool tops, error bits, list length and the
// epoch of a commit that ran out of room
constexpr int kRoundCtrs = C_FAILEP + 1;

// copy device counters [lo, lo+n) to the pinned mirror and wait
pm_status read_ctr(pm_mesh* m, int lo, int n) {
  HIPCHK(hipMemcpyAsync(m->hctr + lo, m->ctr + lo, n * sizeof(int), hipMemcpyDeviceToHost, m->s));
  HIPCHK(hipStreamSynchronize(m->s));
  return PM_OK;
}

// fresh: the host copy of the counters was read after the last kernel
pm_status check_err(pm_mesh* m, bool fresh = false) {
  if (!fresh) TRY(read_ctr(m, C_ERR, 1));
  int e = m->hctr[C_ERR];
  if (!e) return PM_OK;
  std::string msg = "device error bits " + std::to_string(e) + ":";
  if (e & E_MESH_ID) msg += " element id out of range or repeated;";
  if (e & E_MESH_ORIENT) msg += " element not counter-clockwise (area <= 0);";
  if (e & E_MESH_MANIFOLD) msg += " non-manifold edge/vertex or inconsistent orientation;";
  if (e & E_MESH_METRIC) msg += " metric not SPD or non-finite coordinates;";
  if (e & (E_NN_POOL | E_NE_POOL)) msg += " adjacency pool exhausted;";
  if (e & E_STAGE) msg += " commit staging exhausted;";
  if (e & E_COLOURS) msg += " more than 254 colours;";
  set_int(m->ctr + C_ERR, 0, m->s);
  pm_status st = (e & (E_MESH_ID | E_MESH_ORIENT | E_MESH_MANIFOLD | E_MESH_METRIC)) ? PM_E_MESH : PM_E_NOMEM;
  if (e & E_COLOURS) st = PM_E_MESH;
  return fail(m, st, msg);
}

// Records the launches f(stream) issues into an executable graph: captured on
// the handle's private stream (a graph cannot be captured from the null
// stream, which a caller's stream may be) and later launched on the handle's
// stream, in its order. Only kernel launches are recorded (no memsets).
template <class F>
pm_status capture(pm_mesh* m, F&& f, hipGraphExec_t* out) {
  *out = nullptr;
  if (!m->cap_s) HIPCHK(hipStreamCreateWithFlags(&m->cap_s, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(m->cap_s, hipStreamCaptureModeThreadLocal));
  f(m->cap_s);
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamEndCapture(m->cap_s, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(m, PM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return PM_OK;
}

// ---- store allocation -----------------------------------------------------------------------
pm_status grow_vertices(pm_mesh* m, int need) {
  Store& s = m->st;
  if (need <= s.Vcap) return PM_OK;
  int nc = std::max(need, s.Vcap + s.Vcap / 2);
  double2* xy;
  Met* met;
  uint8_t *tag, *va;
  Hdr* hdr;
  int2* cap;
  TRY(dalloc(m, &xy, nc));
  TRY(dalloc(m, &met, nc));
  TRY(dalloc(m, &tag, nc));
  TRY(dalloc(m, &va, nc));
  TRY(dalloc(m, &hdr, nc));
  TRY(dalloc(m, &cap, nc));
  HIPCHK(hipMemsetAsync(va, 0, nc, m->s));
  HIPCHK(hipMemsetAsync(hdr, 0, sizeof(Hdr) * (size_t)nc, m->s));
  HIPCHK(hipMemsetAsync(cap, 0, sizeof(int2) * (size_t)nc, m->s));
  if (s.V > 0) {
    HIPCHK(hipMemcpyAsync(xy, s.xy, sizeof(double2) * s.V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(met, s.met, sizeof(Met) * s.V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(tag, s.tag, s.V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(va, s.valive, s.V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(hdr, s.hdr, sizeof(Hdr) * s.V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(cap, s.cap, sizeof(int2) * s.V, hipMemcpyDeviceToDevice, m->s));
  }
  HIPCHK(hipStreamSynchronize(m->s));
  dfree(m, s.xy, s.Vcap);
  dfree(m, s.met, s.Vcap);
  dfree(m, s.tag, s.Vcap);
  dfree(m, s.valive, s.Vcap);
  dfree(m, s.hdr, s.Vcap);
  dfree(m, s.cap, s.Vcap);
  s.xy = xy;
  s.met = met;
  s.tag = tag;
  s.valive = va;
  s.hdr = hdr;
  s.cap = cap;
  s.Vcap = nc;
  return PM_OK;
}

pm_status grow_elements(pm_mesh* m, int need) {
  Store& s = m->st;
  if (need <= s.Tcap) return PM_OK;
  int nc = std::max(need, s.Tcap + s.Tcap / 2);
  Elem* tri;
  TRY(dalloc(m, &tri, nc));
  HIPCHK(hipMemsetAsync(tri, 0, sizeof(Elem) * (size_t)nc, m->s));
  if (s.T > 0) HIPCHK(hipMemcpyAsync(tri, s.tri, sizeof(Elem) * s.T, hipMemcpyDeviceToDevice, m->s));
  HIPCHK(hipStreamSynchronize(m->s));
  dfree(m, s.tri, s.Tcap);
  s.tri = tri;
  s.Tcap = nc;
  return PM_OK;
}

// copy the host range arrays to the device and point the store at them
pm_status upload_ranges(pm_mesh* m) {
  Store& st = m->st;
  int B = st.B;
  std::vector<int> all;
  all.insert(all.end(), m->vbase.begin(), m->vbase.end());
  all.insert(all.end(), m->vused.begin(), m->vused.end());
  all.insert(all.end(), m->tbase.begin(), m->tbase.end());
  all.insert(all.end(), m->tused.begin(), m->tused.end());
  if (!m->ranges) TRY(dalloc(m, &m->ranges, all.size()));
  if (all.size() <= (size_t)kAuxInts / 2) {
    // staged in the upper half of the pinned ints and copied in stream
    // order; the previous upload's copy has finished before the stage is
    // rewritten
    int* stage = m->haux + kAuxInts / 2;
    if (!m->up_ev) HIPCHK(hipEventCreateWithFlags(&m->up_ev, hipEventDisableTiming));
    else HIPCHK(hipEventSynchronize(m->up_ev));
    std::copy(all.begin(), all.end(), stage);
    HIPCHK(hipMemcpyAsync(m->ranges, stage, sizeof(int) * all.size(), hipMemcpyHostToDevice, m->s));
    HIPCHK(hipEventRecord(m->up_ev, m->s));
  } else {
    HIPCHK(hipStreamSynchronize(m->s));
    HIPCHK(hipMemcpy(m->ranges, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice));
  }
  st.vbase = m->ranges;
  st.vused = st.vbase + B + 1;
  st.tbase = st.vused + B;
  st.tused = st.tbase + B + 1;
  return PM_OK;
}

// ranges of a single mesh: everything in use
pm_status single_ranges(pm_mesh* m) {
  m->vbase = {0, m->st.V};
  m->vused = {m->st.V};
  m->tbase = {0, m->st.T};
  m->tused = {m->st.T};
  return upload_ranges(m);
}

// (Re)build every adjacency row from the element list into fresh pools.
// check: read the error bits back at the end (else they stay set for the
// caller's next read-back)
pm_status build_rows(pm_mesh* m, bool check = true) {
  Store& st = m->st;
  int V = st.V;
  TRY(ensure(m, m->vt0, V));
  TRY(ensure(m, m->vt1, V));
  TRY(ensure(m, m->vt2, V));
  TRY(ensure(m, m->vt3, V));
  TRY(ensure(m, m->vt4, V));
  TRY(ensure(m, m->partial, scan_partials_needed(std::max(V, st.T)) + 2));
  zero_ints(m->vt0.p, V, m->s);
  build_count(st, m->vt0.p, m->s);
  build_caps(st, m->vt0.p, m->slack, m->vt1.p, m->vt2.p, m->s);
  // the slot totals are the pools' new bump pointers
  scan_excl(m->vt1.p, m->vt3.p, V, m->ctr + C_NN_TOP, m->partial.p, m->s);
  scan_excl(m->vt2.p, m->vt4.p, V, m->ctr + C_NE_TOP, m->partial.p, m->s);
  // room for rows that outgrow their slot before the next rebuild: the
  // headroom (3 by default) times the used entries. Slot capacities are at
  // most c(1+slack) + slack + 7 for a vertex in c elements, and the c sum to
  // 3T, which bounds both totals; when the pools hold the headroom times that
  // bound they are large enough without a read-back.
  double bound = 3.0 * st.T * (1.0 + m->slack) + (double)V * (m->slack + 7.0);
  double extra = m->headroom >= 3.0 ? 4096.0 : 64.0;
  double room = m->headroom * bound + extra;
  if (room <= (double)INT32_MAX && (double)st.nn_pool >= room && (double)st.ne_pool >= room) {
    set_headers(st, m->vt3.p, m->vt4.p, m->vt1.p, m->vt2.p, m->s);
    build_fill(st, nullptr, m->s);
    build_finish(st, m->ctr, m->s);
    return check ? check_err(m) : PM_OK;
  }
  TRY(read_ctr(m, C_NN_TOP, 2));
  int64_t nn_used = m->hctr[C_NN_TOP], ne_used = m->hctr[C_NE_TOP];
  int64_t nn_need = (int64_t)(m->headroom * (double)nn_used + extra);
  int64_t ne_need = (int64_t)(m->headroom * (double)ne_used + extra);
  if (nn_need > INT32_MAX || ne_need > INT32_MAX) return fail(m, PM_E_NOMEM, "adjacency pool beyond 2^31 entries");
  if (st.nn_pool < nn_need || st.ne_pool < ne_need) {
    TRY(sync(m));
    dfree(m, st.nn, st.nn_pool);
    dfree(m, st.ne, st.ne_pool);
    st.nn_pool = st.ne_pool = 0;
    TRY(dalloc(m, &st.nn, nn_need));
    TRY(dalloc(m, &st.ne, ne_need));
    st.nn_pool = nn_need;
    st.ne_pool = ne_need;
  }
  set_headers(st, m->vt3.p, m->vt4.p, m->vt1.p, m->vt2.p, m->s);
  build_fill(st, nullptr, m->s);
  build_finish(st, m->ctr, m->s);
  return check ? check_err(m) : PM_OK;
}

// free pool space check between rounds: rebuild (repack) when a round could
// plausibly exhaust it
// from the host copy of the pool tops
bool needs_repack(const pm_mesh* m) {
  int64_t nn_top = m->hctr[C_NN_TOP], ne_top = m->hctr[C_NE_TOP];
  return nn_top * 3 > m->st.nn_pool * 2 || ne_top * 3 > m->st.ne_pool * 2;
}
pm_status maybe_repack(pm_mesh* m, bool fresh = false) {
  if (!fresh) TRY(read_ctr(m, C_NN_TOP, 2));
  if (needs_repack(m)) return build_rows(m);
  return PM_OK;
}

pm_status ensure_phase_scratch(pm_mesh* m) {
  int V = std::max(m->st.V, 1), T = std::max(m->st.T, 1);
  TRY(ensure(m, m->listA, V));
  TRY(ensure(m, m->listB, V));
  TRY(ensure(m, m->jpU0, ((size_t)V + kJpChunk - 1) / kJpChunk * kJpChunk));
  TRY(ensure(m, m->jpB, std::max(((size_t)V + kJpChunk - 1) / kJpChunk * kJpChunk, 2 * (size_t)kSmallColour)));
  // chunk counts of the chunked JP, or the second waiting list of the small colouring
  TRY(ensure(m, m->jpU1, std::max((size_t)V / kJpChunk + 1, (size_t)std::min(V, kSmallColour))));
  TRY(ensure(m, m->cls, V));
  TRY(ensure(m, m->rw, V, true));
  TRY(ensure(m, m->nxt, V, true));
  TRY(ensure(m, m->ops, V, true));
  TRY(ensure(m, m->touch, std::max(V, 65536)));
  TRY(ensure(m, m->seen, V, true));
  TRY(ensure(m, m->own, V, true));
  TRY(ensure(m, m->tk, V, true));
  TRY(ensure(m, m->tgt, V));
  TRY(ensure(m, m->sflag, V));
  TRY(ensure(m, m->spos, V));
  TRY(ensure(m, m->spart, scan_partials_needed(V) + 2));
  // staging for the rows past the register path (more than 32 candidates):
  // 4 ids per candidate; a round that runs out is redone from a row rebuild
  // with twice the staging
  size_t stage = (size_t)(m->stage_scale * m->headroom / 3.0 * (4.0 * T + 4.0 * V)) +
                 (m->headroom >= 3.0 ? 65536 : 64);
  TRY(ensure(m, m->stage, stage));
  return PM_OK;
}

Commit commit_of(pm_mesh* m) {
  Commit c;
  c.epoch = m->epoch;
  c.ops = m->ops.p;
  c.touched = nullptr;
  c.touched_cap = (int)std::min<size_t>(m->touch.n, INT32_MAX);
  c.own = m->own.p;
  c.tk = m->tk.p;
  c.tgt = m->tgt.p;
  c.stage = m->stage.p;
  c.stage_cap = (int64_t)m->stage.n;
  c.nxt = m->nxt.p;
  return c;
}

struct Classes {
  int ncol = 0;
  std::vector<int> size, off;
  int jp_iters = 0;
};

// Jones-Plassmann on list A (n entries): round words in rd.rw (the caller
// clears them), class lists in m->cls. Iterations run on a chunked copy of A
// and are launched in batches between read-backs of the count still waiting;
// a launch past the end of the work finds only empty chunks.
constexpr int kJpBatch = 4;

// the classes of a one-block colouring, from the host copy of the counters
void small_classes(pm_mesh* m, Classes& out) {
  out.jp_iters = m->hctr[C_TOTAL];
  out.ncol = std::max(m->hctr[C_NCOL], 0);
  out.size.assign(m->hctr + C_HIST, m->hctr + C_HIST + out.ncol);
  out.off.assign(m->hctr + C_OFF, m->hctr + C_OFF + out.ncol);
}

pm_status colour_list(pm_mesh* m, const int* A, int n, Round rd, Classes& out) {
  out = Classes();
  if (n == 0) return PM_OK;
  if (n <= kSmallColour && !m->tune.small_work) {
    timed(m, PM_K_JP, 0,
          [&] { colour_small(m->st, A, n, nullptr, rd, m->jpU0.p, m->jpU1.p, m->jpB.p, m->cls.p, m->ctr, m->s); });
    TRY(read_ctr(m, 0, C_NCOL + 1));
    TRY(check_err(m, true));
    small_classes(m, out);
    return PM_OK;
  }
  int nb = (n + kBlock - 1) / kBlock;
  TRY(ensure(m, m->ctab, 256 * (size_t)nb + 256));
  TRY(ensure(m, m->ctabs, 256 * (size_t)nb + 256));
  TRY(ensure(m, m->spart, scan_partials_needed(256 * nb) + 2));
  jp_init(m->st, A, n, rd, m->s);
  stripe_zero(m->ctr, S_JPL, 8, m->s);
  int it = 0;
  for (;;) {
    // first batch: as many iterations as the last colouring needed, so that
    // most colourings need one read-back; the class lists are cut before
    // that read-back, which then also returns them (cut again if the
    // colouring was not finished)
    int batch = it == 0 ? std::min(std::max(m->jp_last, kJpBatch), 64) : kJpBatch;
    for (int b = 0; b < batch; ++b, ++it)
      timed(m, PM_K_JP, 0,
            [&] { jp_chunk(m->st, A, n, m->jpU0.p, m->jpB.p, m->jpU1.p, it == 0, rd, m->ctr, it, m->s); });
    stripe_sum(m->ctr, S_JPL + ((it - 1) & 7), 1, C_JP, m->s);
    m->class_seq = m->class_seq >= 0x3FFFFFFF ? 1 : m->class_seq + 1;
    class_lists(A, n, rd.rw, m->ctr, m->cls.p, m->ctab.p, m->ctabs.p, m->spart.p,
                m->tune.class_colours ? m->tune.class_colours : kClassNarrow, m->class_seq, m->s);
    TRY(read_ctr(m, 0, C_NCOL + 1));
    int left = m->hctr[C_JP];
    if (left == 0) break;
    if (it > 4096) return fail(m, PM_E_DEVICE, "colouring did not finish");
  }
  if (m->hctr[C_NCOL] == -2 && m->tune.class_colours != 256) {
    // a colour past the narrow table: the full table
    class_lists(A, n, rd.rw, m->ctr, m->cls.p, m->ctab.p, m->ctabs.p, m->spart.p, 256, 0, m->s);
    TRY(read_ctr(m, 0, C_NCOL + 1));
  }
  out.jp_iters = it;
  m->jp_last = it;
  TRY(check_err(m, true));
  out.ncol = std::max(m->hctr[C_NCOL], 0);
  out.size.assign(m->hctr + C_HIST, m->hctr + C_HIST + out.ncol);
  out.off.assign(m->hctr + C_OFF, m->hctr + C_OFF + out.ncol);
  return PM_OK;
}

void stats_zero(pm_mesh* m) { stripe_zero(m->ctr, S_EVAL, 6, m->s); }

pm_status stats_read(pm_mesh* m, pm_stats* st) {
  stripe_sum(m->ctr, S_EVAL, 6, C_EVAL, m->s);
  TRY(read_ctr(m, C_EVAL, 6));
  prof_flush(m);
  if (st) {
    st->v[2] += m->hctr[C_EVAL];
    st->v[3] += m->hctr[C_DEFER];
    st->v[4] += m->hctr[C_COMMIT];
    st->v[11] += m->hctr[C_RELOC];
    st->v[10] += m->hctr[C_ROWS];
    st->v[6] += m->hctr[C_EDGES];
  }
  return PM_OK;
}

// headroom a batched mesh keeps after its used slots (refinement grows into it)
int headroom(int used) { return std::max(used / 2, 64); }

// Stable renumbering of live vertices and elements. A single mesh is packed
// densely; the meshes of a batch are packed into consecutive ranges with
// headroom (extra_v / extra_t: further slots a mesh is known to need).
pm_status compact(pm_mesh* m, const std::vector<int>* extra_v = nullptr, const std::vector<int>* extra_t = nullptr) {
  Store& st = m->st;
  int V = st.V, T = st.T, B = st.B;
  TRY(ensure(m, m->vt0, V));
  TRY(ensure(m, m->vt1, V));
  TRY(ensure(m, m->vt2, V));
  TRY(ensure(m, m->tt0, T));
  TRY(ensure(m, m->tt1, T));
  TRY(ensure(m, m->tt2, T));
  TRY(ensure(m, m->rtmp, 4 * (size_t)B + 4));
  TRY(ensure(m, m->partial, scan_partials_needed(std::max(V, T)) + 2));
  flag_live_vertices(st, m->vt0.p, m->s);
  scan_excl(m->vt0.p, m->vt1.p, V, m->ctr + C_TOTAL, m->partial.p, m->s);
  flag_live_elements(st, m->tt0.p, m->s);
  scan_excl(m->tt0.p, m->tt1.p, T, m->ctr + C_TOTAL2, m->partial.p, m->s);
  range_sums(m->vt1.p, m->vt0.p, st.vbase, st.vused, B, m->rtmp.p, m->s);
  range_sums(m->tt1.p, m->tt0.p, st.tbase, st.tused, B, m->rtmp.p + B, m->s);
  std::vector<int> live(2 * B);
  HIPCHK(hipMemcpyAsync(live.data(), m->rtmp.p, sizeof(int) * 2 * B, hipMemcpyDeviceToHost, m->s));
  TRY(sync(m));
  std::vector<int> nvb(B + 1, 0), ntb(B + 1, 0);
  for (int i = 0; i < B; ++i) {
    int lv = live[i], lt = live[B + i];
    int ev = extra_v ? (*extra_v)[i] : 0, et = extra_t ? (*extra_t)[i] : 0;
    int cv = B == 1 ? lv : lv + ev + headroom(lv + ev);
    int ct = B == 1 ? lt : lt + et + headroom(lt + et);
    if ((int64_t)nvb[i] + cv > (1ll << 30) || (int64_t)ntb[i] + ct > (1ll << 30))
      return fail(m, PM_E_NOMEM, "store beyond 2^30 slots");
    nvb[i + 1] = nvb[i] + cv;
    ntb[i + 1] = ntb[i] + ct;
  }
  int nV = nvb[B], nT = ntb[B];
  HIPCHK(hipMemcpyAsync(m->rtmp.p, nvb.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, m->s));
  HIPCHK(hipMemcpyAsync(m->rtmp.p + B + 1, ntb.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, m->s));
  mesh_maps(m->vt0.p, m->vt1.p, st.vmesh, st.vbase, m->rtmp.p, V, m->vt2.p, m->s);
  mesh_maps(m->tt0.p, m->tt1.p, st.tmesh, st.tbase, m->rtmp.p + B + 1, T, m->tt2.p, m->s);
  int vcap = std::max(B == 1 ? st.Vcap : nV, 1), tcap = std::max(B == 1 ? st.Tcap : nT, 1);
  double2* xy2;
  Met* met2;
  uint8_t *tag2, *va2;
  Elem* tri2;
  TRY(dalloc(m, &xy2, vcap));
  TRY(dalloc(m, &met2, vcap));
  TRY(dalloc(m, &tag2, vcap));
  TRY(dalloc(m, &va2, vcap));
  TRY(dalloc(m, &tri2, tcap));
  HIPCHK(hipMemsetAsync(va2, 0, vcap, m->s));
  HIPCHK(hipMemsetAsync(tri2, 0, sizeof(Elem) * (size_t)tcap, m->s));
  compact_vertices(st, m->vt2.p, xy2, met2, tag2, va2, m->s);
  compact_elements(st, m->vt2.p, m->tt2.p, tri2, m->s);
  int *vmesh2 = nullptr, *tmesh2 = nullptr;
  if (B > 1) {
    TRY(dalloc(m, &vmesh2, vcap));
    TRY(dalloc(m, &tmesh2, tcap));
    fill_mesh_ids(m->rtmp.p, B, nV, vmesh2, m->s);
    fill_mesh_ids(m->rtmp.p + B + 1, B, nT, tmesh2, m->s);
  }
  HIPCHK(hipStreamSynchronize(m->s));
  if (B > 1) {
    // headers and capacities follow the new slot count
    Hdr* hdr2;
    int2* cap2;
    TRY(dalloc(m, &hdr2, vcap));
    TRY(dalloc(m, &cap2, vcap));
    HIPCHK(hipMemsetAsync(hdr2, 0, sizeof(Hdr) * (size_t)vcap, m->s));
    HIPCHK(hipMemsetAsync(cap2, 0, sizeof(int2) * (size_t)vcap, m->s));
    dfree(m, st.hdr, st.Vcap);
    dfree(m, st.cap, st.Vcap);
    st.hdr = hdr2;
    st.cap = cap2;
    dfree(m, st.vmesh, st.Vcap);
    dfree(m, st.tmesh, st.Tcap);
    st.vmesh = vmesh2;
    st.tmesh = tmesh2;
  }
  dfree(m, st.xy, st.Vcap);
  dfree(m, st.met, st.Vcap);
  dfree(m, st.tag, st.Vcap);
  dfree(m, st.valive, st.Vcap);
  dfree(m, st.tri, st.Tcap);
  st.xy = xy2;
  st.met = met2;
  st.tag = tag2;
  st.valive = va2;
  st.tri = tri2;
  st.Vcap = vcap;
  st.Tcap = tcap;
  st.V = nV;
  st.T = nT;
  m->vbase = nvb;
  m->tbase = ntb;
  for (int i = 0; i < B; ++i) {
    m->vused[i] = live[i];
    m->tused[i] = live[B + i];
  }
  TRY(upload_ranges(m));
  return build_rows(m);
}

bool bad_tuning(const pm_tuning& t) {
  auto in = [](int v, std::initializer_list<int> ok) {
    for (int x : ok)
      if (v == x) return true;
    return false;
  };
  return !in(t.op_lanes, {0, 1, 8, 16}) || !in(t.smooth_lanes, {0, 1, 8}) ||
         !in(t.commit_chunk, {0, 16, 32, 64, 128}) || !in(t.small_work, {0, 1}) ||
         !in(t.class_colours, {0, 4, 8, 16, 32, 64, 128, 256}) || !in(t.commit_order, {0, 1, 2}) ||
         !in(t.host_rounds, {0, 1, 2}) || t.reserved != 0;
}

bool bad_opts(const pm_options* o) {
  return !(o->L_low2 > 0.0) || !(o->L_up2 > 0.0) || !(o->q_min >= 0.0) || o->coarsen_rounds < 0 ||
         o->swap_rounds < 0 || o->refine_passes < 0 || o->smooth_sweeps < 0 || o->sweep < 0 || o->sweep > 4095 ||
         (o->smooth_kind != PM_SMOOTH_LAPLACE && o->smooth_kind != PM_SMOOTH_GRADIENT &&
          o->smooth_kind != PM_SMOOTH_MINMAX) || !(o->slack >= 1.0) ||
         !(o->pool_headroom == 0.0 || (o->pool_headroom >= 1.0 && o->pool_headroom <= 64.0)) ||
         o->max_iterations < 0 || o->max_iterations > 4095 || o->max_phases < 0 || bad_tuning(o->tune) ||
         (o->quality != PM_QUALITY_MEAN_RATIO && o->quality != PM_QUALITY_VASILEVSKII) || o->reserved != 0 ||
         (o->allocator && (!o->allocator->alloc || !o->allocator->release));
}

// Collapse runs on groups of lanes per member by default: each lane loads
// one neighbour and one element of the member's 1-ring side by side and
// keeps it in registers, so a member costs a few dependent loads and no
// re-reads (one thread per member walks the ring serially and, with tens of
// thousands of members in flight per XCD, re-fetches it from HBM). 16 lanes
// by default; 8, or one thread per member, by tuning.
int op_lanes(const pm_mesh* m) { return m->tune.op_lanes ? m->tune.op_lanes : 16; }
int smooth_lanes(const pm_mesh* m) { return m->tune.smooth_lanes ? m->tune.smooth_lanes : 8; }

pm_status run_rounds_in(pm_mesh* m, const pm_options* o, pm_stats* st, int kind);

// rounds of colour -> classes -> op + commit (coarsen: kind 0, swap: kind 1);
// vertices stay fixed through the rounds, so their records are built once
pm_status run_rounds(pm_mesh* m, const pm_options* o, pm_stats* st, int kind) {
  TRY(ensure(m, m->vr, (size_t)std::max(m->st.V, 1)));
  vertex_records(m->st, m->vr.p, m->s);
  m->st.vr = m->vr.p;
  pm_status r = run_rounds_in(m, o, st, kind);
  m->st.vr = nullptr;
  return r;
}

// One class of a round: the operation over its members, then the commit of
// the rows they changed (one launch for a small class)
void run_class(pm_mesh* m, int kind, const Classes& cl, int c, const OpArgs& a, const Commit& cm) {
  const int* list = m->cls.p + cl.off[c];
  int n = cl.size[c];
  if (n <= kSmallClass && !m->tune.small_work) {
    timed(m, kind == 0 ? PM_K_COLLAPSE : PM_K_FLIP, n, [&] { class_small(m->st, list, n, a, cm, kind, m->ctr, m->s); });
    return;
  }
  if (kind == 0)
    timed(m, PM_K_COLLAPSE, n, [&] { collapse_class(m->st, list, n, a, cm, m->ctr, op_lanes(m), m->s); });
  else
    timed(m, PM_K_FLIP, n, [&] {
      if (op_lanes(m) == 1) flip_class(m->st, list, n, a, cm, m->ctr, m->s);
      else flip_class_g(m->st, list, n, a, cm, m->ctr, m->s);
    });
  bool sweep = m->tune.commit_order == 2 || (m->tune.commit_order == 0 && (int64_t)n * 64 >= m->st.V);
  if (sweep) {
    timed(m, PM_K_COMMIT, 0, [&] { commit_sweep(m->st, cm, kind != 0, m->ctr, m->s); });
  } else {
    timed(m, PM_K_COMMIT, 0,
          [&] { commit_rows(m->st, list, n, cm, kind != 0, m->tune.commit_chunk, m->ctr, m->s); });
  }
}

// A commit ran out of pool or staging room in this round (the host copy of
// the counters says so): rebuild every row from the element list with twice
// the room, then run the classes after the one that ran out. Their kernels
// exited at once; the failing class's operations are all in the element list.
// class_epoch[c]: the epoch class c ran with (-1: not run).
pm_status recover_round(pm_mesh* m, int kind, const Classes& cl, std::vector<int>& class_epoch, Round rd,
                        const pm_options* o, int listA_n) {
  double qmin2 = o->q_min * o->q_min;
  for (;;) {
    int err = m->hctr[C_ERR], fe = m->hctr[C_FAILEP];
    if (!(err & kRoomErr)) return PM_OK;
    int cf = -1;
    for (int c = 0; c < cl.ncol; ++c)
      if (class_epoch[c] == fe) cf = c;
    if (cf < 0) return fail(m, PM_E_DEVICE, "room error of an unknown class");
    ++m->recoveries;
    if (err & (E_NN_POOL | E_NE_POOL)) m->headroom *= 2.0;
    if (err & E_STAGE) m->stage_scale *= 2.0;
    set_int(m->ctr + C_ERR, err & ~kRoomErr, m->s);
    set_int(m->ctr + C_FAILEP, INT_MAX, m->s);
    // every row again from the element list, packed, with the larger room
    TRY(build_rows(m, false));
    TRY(ensure_phase_scratch(m));
    // the round words were cleared with the round: set them again from the
    // class lists, run the remaining classes, clear them again
    std::vector<int> offs(cl.off.begin(), cl.off.end());
    TRY(ensure(m, m->rtmp, (size_t)std::max(cl.ncol, 1)));
    HIPCHK(hipMemcpyAsync(m->rtmp.p, offs.data(), sizeof(int) * cl.ncol, hipMemcpyHostToDevice, m->s));
    restore_round(m->st, m->cls.p, listA_n, m->rtmp.p, cl.ncol, rd, m->s);
    Commit cm = commit_of(m);
    cm.touched = nullptr;
    std::vector<int> ep = class_epoch;
    for (int c = cf + 1; c < cl.ncol; ++c) {
      if (cl.size[c] == 0) continue;
      cm.epoch = ++m->epoch;
      ep[c] = cm.epoch;
      OpArgs a{m->rw.p, c, rd, o->L_low2, qmin2};
      run_class(m, kind, cl, c, a, cm);
    }
    HIPCHK(hipStreamSynchronize(m->s));  // the offsets' host copy is a local vector
    clear_round(m->cls.p, listA_n, m->rw.p, m->s);
    TRY(read_ctr(m, 0, kRoundCtrs));
    class_epoch = ep;
  }
}

// Rounds r, r + 1, ... of a phase whose lists fit one work-group, driven by
// the device: each kernel takes its sizes from the counters, so the host
// issues rounds without reading anything back. Two rounds (list A -> B -> A)
// are captured once as a graph, replayed twice per read-back. Round r's
// classes must be coloured (counters and class lists set). Returns with the
// round counter, list and length of where the chain stopped: the list empty,
// the round cap, a list too long for one work-group (r_out's list, not
// coloured), or a selection that declined (declined: round r_out ran, its
// next list is not selected; the host selects over every slot, after
// rebuilding the rows if a commit ran out of room).
pm_status device_rounds(pm_mesh* m, const pm_options* o, pm_stats* st, int kind, int phase, int max_rounds, int r,
                        int* r_out, int* n_out, bool* declined) {
  int mode = kind == 0 ? 1 : 2;
  double qmin2 = o->q_min * o->q_min;
  std::vector<uint64_t> seeds(max_rounds + 1);
  for (int k = 0; k <= max_rounds; ++k) seeds[k] = stream_seed(m->seed, make_ctx(o->sweep, phase, k));
  TRY(ensure(m, m->seeds, seeds.size()));
  HIPCHK(hipMemcpyAsync(m->seeds.p, seeds.data(), sizeof(uint64_t) * seeds.size(), hipMemcpyHostToDevice, m->s));
  dev_rounds_start(m->ctr, r, m->epoch + 1, m->sel_mark, r >= max_rounds ? 1 : 0, m->s);
  int* L[2] = {m->listA.p, m->listB.p};
  Round rd{0, m->rw.p, m->seeds.p};
  OpArgs a{m->rw.p, 0, rd, o->L_low2, qmin2};
  Commit cm = commit_of(m);
  cm.touched = m->touch.p;
  auto rounds = [&](hipStream_t q) {
    for (int k = 0; k < 2; ++k) {
      const int* A = L[k];
      int* B = L[k ^ 1];
      round_small(m->st, m->cls.p, -1, a, cm, kind, m->ctr, q);
      clear_round_dev(A, m->ctr + C_LIST_B, m->rw.p, q);
      select_small(m->st, mode, o->L_low2, A, -1, m->touch.p, cm.touched_cap, m->nxt.p, m->seen.p, 0, max_rounds, B,
                   m->ctr, q);
      colour_small(m->st, B, 0, m->ctr + C_LIST_B, rd, m->jpU0.p, m->jpU1.p, m->jpB.p, m->cls.p, m->ctr, q);
    }
  };
  // the graph of two rounds is kept while its launch arguments stay the same
  // (the same store layout, buffers and parameters; the seed table is read
  // when it runs)
  hipGraphExec_t ge = nullptr;
  if (m->tune.host_rounds == 2) {
    std::string key;
    auto add = [&](const void* p, size_t n) { key.append((const char*)p, n); };
    add(&m->st, sizeof(Store));
    add(L, sizeof(L));
    add(&a, sizeof(a));
    add(&cm, sizeof(cm));
    int ints[4] = {kind, mode, max_rounds, 0};
    add(ints, sizeof(ints));
    void* ptrs[8] = {m->cls.p, m->ctr, m->nxt.p, m->seen.p, m->jpU0.p, m->jpU1.p, m->jpB.p, m->touch.p};
    add(ptrs, sizeof(ptrs));
    for (auto& g : m->dr_graphs)
      if (g.first == key) ge = g.second;
    if (!ge) {
      TRY(capture(m, rounds, &ge));
      if (m->dr_graphs.size() >= 4) {
        (void)hipGraphExecDestroy(m->dr_graphs.front().second);
        m->dr_graphs.erase(m->dr_graphs.begin());
      }
      m->dr_graphs.push_back({key, ge});
    }
  }
  pm_status res = PM_OK;
  for (;;) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
      timed(m, kind == 0 ? PM_K_COLLAPSE : PM_K_FLIP, 0, [&] {
        if (ge) e = hipGraphLaunch(ge, m->s);
        else rounds(m->s);
      });
    if (e != hipSuccess) {
      res = fail(m, PM_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
      break;
    }
    res = read_ctr(m, 0, C_NCOL + 1);
    if (res != PM_OK || m->hctr[C_DSTOP]) break;
  }
  TRY(res);
  int rr = m->hctr[C_DROUND];
  st->v[1] += m->hctr[C_ACC_COL];
  st->v[5] += m->hctr[C_ACC_NCOL];
  st->v[12] += m->hctr[C_ACC_IT];
  m->epoch = m->hctr[C_DEPOCH] - 1;
  m->sel_mark = m->hctr[C_DMARK];
  // the list of round rr is L[(rr - r) & 1]
  int cur = (rr - r) & 1;
  m->listA.p = L[cur];
  m->listB.p = L[cur ^ 1];
  *r_out = rr;
  *n_out = m->hctr[C_LIST_B];
  *declined = m->hctr[C_LIST_B] < 0;
  return PM_OK;
}

pm_status run_rounds_in(pm_mesh* m, const pm_options* o, pm_stats* st, int kind) {
  TRY(ensure_phase_scratch(m));
  m->tune = o->tune;
  m->recoveries = 0;
  int mode = kind == 0 ? 1 : 2;
  int max_rounds = kind == 0 ? o->coarsen_rounds : o->swap_rounds;
  int phase = kind == 0 ? PH_COARSEN : PH_SWAP;
  double qmin2 = o->q_min * o->q_min;
  stats_zero(m);
  set_int(m->ctr + C_LIST_B, 0, m->s);
  set_int(m->ctr + C_FAILEP, INT_MAX, m->s);
  timed(m, PM_K_SELECT, m->st.V,
        [&] { select_vertices(m->st, mode, o->L_low2, nullptr, nullptr, m->listA.p, m->ctr, m->sflag.p,
                          m->spos.p, m->spart.p, m->s); });
  TRY(read_ctr(m, 0, kRoundCtrs));  // pool tops, error bits and the list length at once
  TRY(check_err(m, true));
  int nA = m->hctr[C_LIST_B];
  int r = 0;
  // a small round colours the next round's list as soon as it is selected,
  // before the read-back that returns its length: one read-back for both
  bool ahead = false;
  Classes next;
  while (nA > 0 && r < max_rounds) {
    // after a repack (all rows rebuilt) the list is coloured again rather
    // than keep classes found before it
    bool repacked = needs_repack(m);
    TRY(maybe_repack(m, true));
    Round rd{stream_seed(m->seed, make_ctx(o->sweep, phase, r)), m->rw.p};
    Classes cl;
    if (ahead && !repacked) {
      cl = next;
    } else {
      TRY(colour_list(m, m->listA.p, nA, rd, cl));
    }
    ahead = false;
    Commit cm = commit_of(m);
    // a small round (coloured by one block) records the rows it rebuilds, so
    // the next round's list comes from its own lists, not from every slot
    bool small = nA <= kSmallColour && !m->tune.small_work;
    cm.touched = small ? m->touch.p : nullptr;
    st->v[1] += nA;
    st->v[5] += cl.ncol;
    st->v[12] += cl.jp_iters;
    bool fits = cl.ncol > 0;
    for (int c = 0; c < cl.ncol && fits; ++c) fits = cl.size[c] <= kSmallClass;
    if (small && m->tune.host_rounds != 1 && fits) {
      int rr = r, nl = 0;
      bool declined = false;
      TRY(device_rounds(m, o, st, kind, phase, max_rounds, r, &rr, &nl, &declined));
      if (!declined) {
        // the next round's list is coloured when it fits one work-group (the
        // counters hold its classes; a class too large for the chain stopped
        // it), else the host colours it
        nA = nl;
        r = rr;
        ahead = m->hctr[C_NCOL] >= 0 && nl > 0;
        if (ahead) small_classes(m, next);
        continue;
      }
      // round rr ran, its selection declined: the classes from the counters
      if (m->hctr[C_NCOL] < 0 || m->hctr[C_NCOL] > kMaxColours)
        return fail(m, PM_E_DEVICE, "device-driven round left no class counters");
      Classes dc;
      small_classes(m, dc);
      std::vector<int> dep(dc.ncol);
      for (int c = 0; c < dc.ncol; ++c) dep[c] = m->hctr[C_DEPOCH0] + c;
      int n_rr = 0;
      for (int c = 0; c < dc.ncol; ++c) n_rr += dc.size[c];
      if (m->hctr[C_ERR] & kRoomErr) {
        Round rdd{stream_seed(m->seed, make_ctx(o->sweep, phase, rr)), m->rw.p};
        TRY(recover_round(m, kind, dc, dep, rdd, o, n_rr));
      }
      set_int(m->ctr + C_LIST_B, 0, m->s);
      timed(m, PM_K_SELECT, m->st.V, [&] {
        select_vertices(m->st, mode, o->L_low2, nullptr, m->nxt.p, m->listB.p, m->ctr, m->sflag.p, m->spos.p,
                        m->spart.p, m->s);
      });
      TRY(read_ctr(m, 0, kRoundCtrs));
      TRY(check_err(m, true));
      nA = m->hctr[C_LIST_B];
      std::swap(m->listA, m->listB);
      r = rr + 1;
      ahead = false;
      continue;
    }
    std::vector<int> class_epoch(cl.ncol, -1);
    // a small round whose classes are all small: every class in one block,
    // one launch
    bool all_small = small && cl.ncol > 1;
    for (int c = 0; c < cl.ncol && all_small; ++c) all_small = cl.size[c] <= kSmallClass;
    if (all_small) {
      cm.epoch = m->epoch + 1;
      for (int c = 0; c < cl.ncol; ++c) class_epoch[c] = cm.epoch + c;
      m->epoch += cl.ncol;
      OpArgs a{m->rw.p, 0, rd, o->L_low2, qmin2};
      timed(m, kind == 0 ? PM_K_COLLAPSE : PM_K_FLIP, nA,
            [&] { round_small(m->st, m->cls.p, cl.ncol, a, cm, kind, m->ctr, m->s); });
    }
    for (int c = 0; c < cl.ncol && !all_small; ++c) {
      if (cl.size[c] == 0) continue;
      cm.epoch = ++m->epoch;
      class_epoch[c] = cm.epoch;
      OpArgs a{m->rw.p, c, rd, o->L_low2, qmin2};
      run_class(m, kind, cl, c, a, cm);
    }
    clear_round(m->listA.p, nA, m->rw.p, m->s);
    bool listed = false;
    if (small) {
      timed(m, PM_K_SELECT, nA, [&] {
        select_small(m->st, mode, o->L_low2, m->listA.p, nA, m->touch.p, cm.touched_cap, m->nxt.p, m->seen.p,
                     ++m->sel_mark, max_rounds, m->listB.p, m->ctr, m->s);
      });
      bool launch = r + 1 < max_rounds;
      if (launch) {
        Round rn{stream_seed(m->seed, make_ctx(o->sweep, phase, r + 1)), m->rw.p};
        timed(m, PM_K_JP, 0, [&] {
          colour_small(m->st, m->listB.p, 0, m->ctr + C_LIST_B, rn, m->jpU0.p, m->jpU1.p, m->jpB.p, m->cls.p,
                       m->ctr, m->s);
        });
      }
      TRY(read_ctr(m, 0, launch ? C_NCOL + 1 : kRoundCtrs));
      listed = m->hctr[C_LIST_B] >= 0;
      if (launch && listed && m->hctr[C_NCOL] >= 0) {
        ahead = true;
        small_classes(m, next);
      }
    }
    auto select_all = [&]() -> pm_status {
      set_int(m->ctr + C_LIST_B, 0, m->s);
      timed(m, PM_K_SELECT, m->st.V, [&] {
        select_vertices(m->st, mode, o->L_low2, nullptr, m->nxt.p, m->listB.p, m->ctr, m->sflag.p, m->spos.p,
                        m->spart.p, m->s);
      });
      return read_ctr(m, 0, kRoundCtrs);
    };
    if (!listed) TRY(select_all());
    if (m->hctr[C_ERR] & kRoomErr) {
      // the selections and the next colouring declined (they saw the error):
      // rebuild, finish the round, then select over every slot
      TRY(recover_round(m, kind, cl, class_epoch, rd, o, nA));
      ahead = false;
      TRY(select_all());
    }
    TRY(check_err(m, true));
    nA = m->hctr[C_LIST_B];
    std::swap(m->listA, m->listB);
    ++r;
  }
  TRY(stats_read(m, st));
  st->v[0] = r;
  st->v[7] = nA == 0 ? 1 : 0;
  st->v[13] = m->recoveries;
  return PM_OK;
}

// partial sums of the quality reduction: one per 256 element slots, at most
// kQualityParts (the same shape for pm_quality and pm_quality_noalloc)
constexpr int kQualityParts = 2048;
int quality_parts(const pm_mesh* m) { return std::min(std::max((m->st.T + 255) / 256, 1), kQualityParts); }

// Device memory that pm_quality_noalloc works in instead of allocating: the
// quality reduction's partial sums and minima and its two results. Each
// device that runs the library holds its own copy until the process ends.
// Host code never uses this name as an address: the device address of each
// device's copy comes from hipGetSymbolAddress, taken once per device with
// that device current (at the first handle created on it).
constexpr int kScratchDoubles = 2 * kQualityParts + 2;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_at[kMaxDevices] = {};

// the current device's copy of the scratch array, for handle m
pm_status scratch_setup(pm_mesh* m) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(m, PM_E_DEVICE, "device index past the scratch table");
  m->dev = dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(m, PM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_at[dev] = (double*)p;
  }
  m->scratch = g_scratch_at[dev];
  return PM_OK;
}

void fill_defaults(pm_options* o) {
  o->L_low2 = 0.5;
  o->L_up2 = 2.0;
  o->q_min = 0.1;
  o->seed = 0;
  o->sweep = 0;
  o->coarsen_rounds = 200;
  o->swap_rounds = 100;
  o->refine_passes = 32;
  o->smooth_kind = PM_SMOOTH_LAPLACE;
  o->smooth_sweeps = 1;
  o->slack = 2.0;
  o->pool_headroom = 3.0;
  o->max_iterations = 8;
  o->max_phases = 0;
  o->tune = pm_tuning{};
  o->quality = PM_QUALITY_MEAN_RATIO;
  o->reserved = 0;
  o->allocator = nullptr;
}

}  // namespace

namespace pm {
hipError_t block_alloc(hipStream_t s, void** p, size_t bytes) {
  size_t got = 0;
  return cache_get(s, p, bytes, &got);
}
void block_free(void* p) {
  if (p && cache_put(p) == 0) (void)hipFree(p);
}
}  // namespace pm

extern "C" {

const char* pm_version(void) { return "pmesh 0.1 gfx950"; }

pm_status pm_default_options(pm_options* o) {
  if (!o) return PM_E_ARG;
  fill_defaults(o);
  return PM_OK;
}

const char* pm_last_error(const pm_mesh* m) {
  if (!m) return g_create_err.empty() ? "null handle" : g_create_err.c_str();
  return m->err.c_str();
}

pm_status pm_mesh_destroy(pm_mesh* m) {
  if (!m) return PM_OK;
  (void)hipStreamSynchronize(m->s);
  Store& s = m->st;
  dfree(m, s.xy, s.Vcap);
  dfree(m, s.met, s.Vcap);
  dfree(m, s.tag, s.Vcap);
  dfree(m, s.valive, s.Vcap);
  dfree(m, s.hdr, s.Vcap);
  dfree(m, s.cap, s.Vcap);
  dfree(m, s.tri, s.Tcap);
  dfree(m, s.nn, s.nn_pool);
  dfree(m, s.ne, s.ne_pool);
  dfree(m, s.vmesh, s.Vcap);
  dfree(m, s.tmesh, s.Tcap);
  dfree(m, m->ranges, 1);
  dfree(m, m->mdone, 1);
  DBuf<int>* ib[] = {&m->listA, &m->listB, &m->jpU0, &m->jpU1, &m->cls, &m->vt0, &m->vt1, &m->vt2, &m->vt3,
                     &m->vt4, &m->tt0, &m->tt1, &m->tt2, &m->partial, &m->mid, &m->stage, &m->touch, &m->seen, &m->jpB, &m->rtmp,
                     &m->sflag, &m->spos,
                     &m->ctab, &m->ctabs, &m->spart};
  for (auto* b : ib) dfree(m, b->p, b->n);
  DBuf<uint8_t>* ub[] = {&m->nxt, &m->u8tmp};
  dfree(m, m->emet.p, m->emet.n);
  dfree(m, m->vr.p, m->vr.n);
  for (auto* b : ub) dfree(m, b->p, b->n);
  dfree(m, m->qpart.p, m->qpart.n);
  dfree(m, m->upd.p, m->upd.n);
  dfree(m, m->rw.p, m->rw.n);
  dfree(m, m->seeds.p, m->seeds.n);
  dfree(m, m->own.p, m->own.n);
  dfree(m, m->tk.p, m->tk.n);
  dfree(m, m->tgt.p, m->tgt.n);
  dfree(m, m->ops.p, m->ops.n);
  prof_flush(m);
  for (hipEvent_t e : m->prof.pool) (void)hipEventDestroy(e);
  if (m->up_ev) {
    (void)hipEventSynchronize(m->up_ev);
    (void)hipEventDestroy(m->up_ev);
  }
  dfree(m, m->ctr, C_COUNT);
  pinned_put(m);
  for (auto& g : m->dr_graphs) (void)hipGraphExecDestroy(g.second);
  if (m->cap_s) (void)hipStreamDestroy(m->cap_s);
  delete m;
  return PM_OK;
}

pm_status pm_mesh_create(const pm_mesh_desc* d, const pm_options* o, void* stream, pm_mesh** out) {
  if (!out) return PM_E_ARG;
  *out = nullptr;
  if (!d || !d->xy || !d->tri || !d->metric) return PM_E_ARG;
  if (d->V < 3 || d->T < 1 || d->V > (1ll << 30) || d->T > (1ll << 30)) return PM_E_ARG;
  if (d->mem_kind != PM_MEM_HOST && d->mem_kind != PM_MEM_DEVICE) return PM_E_ARG;
  pm_options def;
  fill_defaults(&def);
  if (!o) o = &def;
  if (bad_opts(o)) return PM_E_ARG;
  pm_mesh* m = new (std::nothrow) pm_mesh();
  if (!m) return PM_E_NOMEM;
  m->s = (hipStream_t)stream;
  m->seed = o->seed;
  m->slack = o->slack;
  m->headroom = o->pool_headroom > 0.0 ? o->pool_headroom : 3.0;
  m->st.qk = o->quality;
  if (o->allocator) m->va = *o->allocator;
  g_create_err.clear();
  auto bail = [&](pm_status st) {
    g_create_err = m->err.empty() ? std::string("pm_mesh_create failed") : m->err;
    pm_mesh_destroy(m);
    return st;
  };
  if (dalloc(m, &m->ctr, C_COUNT) != PM_OK || !pinned_get(m)) return bail(PM_E_NOMEM);
  if (scratch_setup(m) != PM_OK) return bail(PM_E_DEVICE);
  zero_ints(m->ctr, C_COUNT, m->s);
  set_int(m->ctr + C_FAILEP, INT_MAX, m->s);
  int V = (int)d->V, T = (int)d->T;
  if (grow_vertices(m, V) != PM_OK || grow_elements(m, T) != PM_OK) return bail(PM_E_NOMEM);
  Store& st = m->st;
  st.V = V;
  st.T = T;
  hipMemcpyKind kind = d->mem_kind == PM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  int* tri3 = nullptr;
  double* xyraw = nullptr;
  if (dalloc(m, &tri3, 3 * (size_t)T) != PM_OK || dalloc(m, &xyraw, 2 * (size_t)V) != PM_OK)
    return bail(PM_E_NOMEM);
  bool ok = hipMemcpyAsync(tri3, d->tri, sizeof(int) * 3 * (size_t)T, kind, m->s) == hipSuccess &&
            hipMemcpyAsync(xyraw, d->xy, sizeof(double) * 2 * (size_t)V, kind, m->s) == hipSuccess &&
            hipMemcpyAsync(st.met, d->metric, sizeof(double) * 3 * (size_t)V, kind, m->s) == hipSuccess;
  if (ok && d->tags) ok = hipMemcpyAsync(st.tag, d->tags, (size_t)V, kind, m->s) == hipSuccess;
  if (!ok) {
    dfree(m, tri3, 3 * (size_t)T);
    dfree(m, xyraw, 2 * (size_t)V);
    return bail(PM_E_DEVICE);
  }
  xy_in(xyraw, V, st.xy, m->s);
  if (!d->tags) tags_from_xy(st.xy, V, st.tag, m->s);
  tri_in(tri3, T, st.tri, m->s);
  fill_u8(st.valive, V, 1, m->s);
  // the staging blocks return to this stream's cache: later work on the
  // stream is ordered after the conversions that read them
  dfree(m, tri3, 3 * (size_t)T);
  dfree(m, xyraw, 2 * (size_t)V);
  if (single_ranges(m) != PM_OK) return bail(PM_E_DEVICE);
  k_validate(st, m->ctr, m->s);
  pm_status r = check_err(m);
  if (r != PM_OK) return bail(r);
  r = build_rows(m);
  if (r != PM_OK) return bail(r);
  *out = m;
  return PM_OK;
}

pm_status pm_mesh_sizes(const pm_mesh* m, int64_t* V, int64_t* T) {
  if (!m) return PM_E_ARG;
  if (V) *V = m->st.V;
  if (T) *T = m->st.T;
  return PM_OK;
}

pm_status pm_mesh_memory(const pm_mesh* m, int64_t* current_bytes, int64_t* peak_bytes) {
  if (!m) return PM_E_ARG;
  if (current_bytes) *current_bytes = m->cur_bytes;
  if (peak_bytes) *peak_bytes = m->peak_bytes;
  return PM_OK;
}

pm_status pm_mesh_export(pm_mesh* m, double* xy, int32_t* tri, double* metric, uint8_t* tags, uint8_t* valive,
                         uint8_t* talive, int32_t mem_kind) {
  if (!m) return PM_E_ARG;
  if (mem_kind != PM_MEM_HOST && mem_kind != PM_MEM_DEVICE) return fail(m, PM_E_ARG, "bad mem_kind");
  Store& st = m->st;
  hipMemcpyKind k = mem_kind == PM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (xy) HIPCHK(hipMemcpyAsync(xy, st.xy, sizeof(double2) * st.V, k, m->s));
  if (metric) HIPCHK(hipMemcpyAsync(metric, st.met, sizeof(Met) * st.V, k, m->s));
  if (tags) HIPCHK(hipMemcpyAsync(tags, st.tag, st.V, k, m->s));
  if (valive) HIPCHK(hipMemcpyAsync(valive, st.valive, st.V, k, m->s));
  if (tri || talive) {
    TRY(ensure(m, m->tt0, 3 * (size_t)st.T));
    TRY(ensure(m, m->u8tmp, (size_t)std::max(st.T, 1)));
    export_tri(st, m->tt0.p, m->u8tmp.p, m->s);
    if (tri) HIPCHK(hipMemcpyAsync(tri, m->tt0.p, sizeof(int) * 3 * (size_t)st.T, k, m->s));
    if (talive) HIPCHK(hipMemcpyAsync(talive, m->u8tmp.p, st.T, k, m->s));
  }
  return sync(m);
}

pm_status pm_mesh_rows(pm_mesh* m, int64_t* nn_total, int64_t* ne_total, int64_t* nn_off, int32_t* nn,
                       int64_t* ne_off, int32_t* ne) {
  if (!m || !nn_total || !ne_total) return PM_E_ARG;
  Store& st = m->st;
  std::vector<Hdr> hdr(st.V);
  std::vector<int2> cap(st.V);
  HIPCHK(hipMemcpyAsync(hdr.data(), st.hdr, sizeof(Hdr) * st.V, hipMemcpyDeviceToHost, m->s));
  HIPCHK(hipMemcpyAsync(cap.data(), st.cap, sizeof(int2) * st.V, hipMemcpyDeviceToHost, m->s));
  TRY(sync(m));
  int64_t a = 0, b = 0;
  for (int v = 0; v < st.V; ++v) {
    a += hdr[v].y;
    b += hdr[v].w;
    // the row layout the kernels rely on: slots start at multiples of four
    // entries, hold a multiple of four, and hold their row
    const Hdr& h = hdr[v];
    const int2& c = cap[v];
    bool ok = h.x % 4 == 0 && h.z % 4 == 0 && c.x % 4 == 0 && c.y % 4 == 0 && h.y <= c.x && h.w <= c.y &&
              (int64_t)h.x + c.x <= st.nn_pool && (int64_t)h.z + c.y <= st.ne_pool;
    if (!ok) return fail(m, PM_E_DEVICE, "row slot of vertex " + std::to_string(v) + " breaks the layout");
  }
  *nn_total = a;
  *ne_total = b;
  if (!nn_off || !nn || !ne_off || !ne) return PM_OK;
  std::vector<int> pnn(st.nn_pool), pne(st.ne_pool);
  HIPCHK(hipMemcpyAsync(pnn.data(), st.nn, sizeof(int) * st.nn_pool, hipMemcpyDeviceToHost, m->s));
  HIPCHK(hipMemcpyAsync(pne.data(), st.ne, sizeof(int) * st.ne_pool, hipMemcpyDeviceToHost, m->s));
  TRY(sync(m));
  a = b = 0;
  for (int v = 0; v < st.V; ++v) {
    nn_off[v] = a;
    ne_off[v] = b;
    for (int k = 0; k < hdr[v].y; ++k) nn[a++] = pnn[hdr[v].x + k];
    for (int k = 0; k < hdr[v].w; ++k) ne[b++] = pne[hdr[v].z + k];
  }
  nn_off[st.V] = a;
  ne_off[st.V] = b;
  return PM_OK;
}

pm_status pm_colour(pm_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out, int32_t* ncolours,
                    int32_t mem_kind) {
  if (!m) return PM_E_ARG;
  if (mem_kind != PM_MEM_HOST && mem_kind != PM_MEM_DEVICE) return fail(m, PM_E_ARG, "bad mem_kind");
  TRY(ensure_phase_scratch(m));
  Store& st = m->st;
  const uint8_t* act_in = nullptr;
  if (active) {
    TRY(ensure(m, m->u8tmp, st.V));
    HIPCHK(hipMemcpyAsync(m->u8tmp.p, active, st.V,
                          mem_kind == PM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, m->s));
    act_in = m->u8tmp.p;
  }
  set_int(m->ctr + C_LIST_B, 0, m->s);
  select_vertices(st, 0, 0.0, act_in, nullptr, m->listA.p, m->ctr, m->sflag.p, m->spos.p, m->spart.p,
                  m->s);
  TRY(read_ctr(m, C_LIST_B, 1));
  int n = m->hctr[C_LIST_B];
  Classes cl;
  TRY(colour_list(m, m->listA.p, n, Round{stream_seed(m->seed, ctx), m->rw.p}, cl));
  if (ncolours) *ncolours = cl.ncol;
  if (colour_out) {
    TRY(ensure(m, m->vt0, st.V));
    pm::colour_out(st, m->rw.p, m->vt0.p, m->s);
    HIPCHK(hipMemcpyAsync(colour_out, m->vt0.p, sizeof(int) * st.V,
                          mem_kind == PM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, m->s));
  }
  clear_round(m->listA.p, n, m->rw.p, m->s);
  return sync(m);
}

pm_status pm_coarsen(pm_mesh* m, const pm_options* o, pm_stats* st) {
  if (!m || !o) return PM_E_ARG;
  if (bad_opts(o)) return fail(m, PM_E_ARG, "bad options");
  ++m->topo;
  pm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  TRY(run_rounds(m, o, st, 0));
  TRY(compact(m));
  return st->v[7] ? PM_OK : PM_W_NOT_CONVERGED;
}

pm_status pm_swap(pm_mesh* m, const pm_options* o, pm_stats* st) {
  if (!m || !o) return PM_E_ARG;
  if (bad_opts(o)) return fail(m, PM_E_ARG, "bad options");
  ++m->topo;
  pm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  TRY(run_rounds(m, o, st, 1));
  return st->v[7] ? PM_OK : PM_W_NOT_CONVERGED;
}

pm_status pm_smooth(pm_mesh* m, const pm_options* o, pm_stats* st) {
  if (!m || !o) return PM_E_ARG;
  if (bad_opts(o)) return fail(m, PM_E_ARG, "bad options");
  pm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  TRY(ensure_phase_scratch(m));
  m->tune = o->tune;
  stats_zero(m);
  set_int(m->ctr + C_LIST_B, 0, m->s);
  select_vertices(m->st, 3, 0.0, nullptr, nullptr, m->listA.p, m->ctr, m->sflag.p, m->spos.p,
                  m->spart.p, m->s);
  TRY(read_ctr(m, C_LIST_B, 1));
  int n = m->hctr[C_LIST_B];
  Classes cl;
  TRY(colour_list(m, m->listA.p, n, Round{stream_seed(m->seed, make_ctx(o->sweep, PH_SMOOTH, 0)), m->rw.p}, cl));
  st->v[1] = n;
  st->v[5] = cl.ncol;
  st->v[12] = cl.jp_iters;
  // topology and metrics stay fixed while smoothing: element tensors once,
  // and kept while the topology does not change
  if (m->emet_topo != m->topo || m->emet.n < (size_t)std::max(m->st.T, 1)) {
    TRY(ensure(m, m->emet, (size_t)std::max(m->st.T, 1)));
    element_metrics(m->st, m->emet.p, m->s);
    m->emet_topo = m->topo;
  }
  m->st.emet = m->emet.p;
  auto sweep_on = [&](hipStream_t q) {
    for (int c = 0; c < cl.ncol; ++c)
      smooth_class(m->st, m->cls.p + cl.off[c], cl.size[c], o->smooth_kind, m->ctr, smooth_lanes(m), q);
  };
  int64_t members = 0;
  for (int c = 0; c < cl.ncol; ++c) members += cl.size[c];
  if (o->smooth_sweeps > 1) {
    // the classes' launches of one sweep, captured once as a graph and
    // replayed for every sweep (they read only the class lists and the store)
    hipGraphExec_t ge = nullptr;
    TRY(capture(m, sweep_on, &ge));
    pm_status r = PM_OK;
    for (int s = 0; s < o->smooth_sweeps && r == PM_OK; ++s) {
      hipError_t e = hipSuccess;
      timed(m, PM_K_SMOOTH, members, [&] { e = hipGraphLaunch(ge, m->s); });
      if (e != hipSuccess) r = fail(m, PM_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    }
    (void)hipGraphExecDestroy(ge);
    TRY(r);
  } else {
    for (int c = 0; c < cl.ncol; ++c)
      timed(m, PM_K_SMOOTH, cl.size[c], [&] {
        smooth_class(m->st, m->cls.p + cl.off[c], cl.size[c], o->smooth_kind, m->ctr, smooth_lanes(m), m->s);
      });
  }
  m->st.emet = nullptr;
  clear_round(m->listA.p, n, m->rw.p, m->s);
  TRY(stats_read(m, st));
  st->v[0] = o->smooth_sweeps;
  st->v[7] = 1;
  return PM_OK;
}

pm_status pm_refine(pm_mesh* m, const pm_options* o, pm_stats* st) {
  if (!m || !o) return PM_E_ARG;
  if (bad_opts(o)) return fail(m, PM_E_ARG, "bad options");
  ++m->topo;
  pm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  stats_zero(m);
  Store& s = m->st;
  int B = s.B;
  int p = 0;
  bool done = false;
  int relayouts = 0;
  // per-mesh flags: a mesh whose pass found nothing to split is finished
  std::vector<int> mdone(B, 0);
  if (B > 1) {
    if (!m->mdone) TRY(dalloc(m, &m->mdone, B));
    HIPCHK(hipMemcpyAsync(m->mdone, mdone.data(), sizeof(int) * B, hipMemcpyHostToDevice, m->s));
    HIPCHK(hipStreamSynchronize(m->s));
    s.mdone = m->mdone;
  }
  while (p < o->refine_passes) {
    int V0 = s.V, T0 = s.T;
    TRY(ensure(m, m->vt0, V0));
    TRY(ensure(m, m->vt1, V0));
    TRY(ensure(m, m->tt0, T0));
    TRY(ensure(m, m->tt1, T0));
    TRY(ensure(m, m->rtmp, 4 * (size_t)B + 4));
    TRY(ensure(m, m->partial, scan_partials_needed(std::max(V0, T0)) + 2));
    stripe_zero(m->ctr, S_EDGES, 1, m->s);
    refine_mark(s, o->L_up2, m->vt0.p, m->ctr, m->s);
    scan_excl(m->vt0.p, m->vt1.p, V0, m->ctr + C_TOTAL, m->partial.p, m->s);
    refine_count(s, o->L_up2, m->tt0.p, m->s);
    scan_excl(m->tt0.p, m->tt1.p, T0, m->ctr + C_TOTAL2, m->partial.p, m->s);
    range_sums(m->vt1.p, m->vt0.p, s.vbase, s.vused, B, m->rtmp.p, m->s);
    range_sums(m->tt1.p, m->tt0.p, s.tbase, s.tused, B, m->rtmp.p + B, m->s);
    // per-mesh needs, totals and tested edges come back in one wait
    std::vector<int> need(2 * B);
    bool aux = 2 * B <= kAuxInts;
    HIPCHK(hipMemcpyAsync(aux ? m->haux : need.data(), m->rtmp.p, sizeof(int) * 2 * B, hipMemcpyDeviceToHost, m->s));
    stripe_sum(m->ctr, S_EDGES, 1, C_EDGES, m->s);
    TRY(read_ctr(m, 0, C_JP));
    TRY(check_err(m, true));  // also the last row build's
    if (aux) std::copy(m->haux, m->haux + 2 * B, need.begin());
    int nv = m->hctr[C_TOTAL], nt = m->hctr[C_TOTAL2];
    int edges = m->hctr[C_EDGES];
    if (nv == 0) {
      st->v[6] += edges;
      done = true;
      break;
    }

    if (B == 1) {
      if ((int64_t)V0 + nv > (1ll << 30) || (int64_t)T0 + nt > (1ll << 30))
        return fail(m, PM_E_NOMEM, "refinement beyond 2^30 vertices or elements");
      TRY(grow_vertices(m, V0 + nv));
      TRY(grow_elements(m, T0 + nt));
    } else {
      bool fits = true;
      for (int i = 0; i < B; ++i)
        fits &= m->vused[i] + need[i] <= m->vbase[i + 1] - m->vbase[i] &&
                m->tused[i] + need[B + i] <= m->tbase[i + 1] - m->tbase[i];
      if (!fits) {
        // a mesh outgrows its range: re-lay the batch out with room, then redo the pass
        if (++relayouts > 1) return fail(m, PM_E_NOMEM, "refinement could not be given room");
        std::vector<int> ev(need.begin(), need.begin() + B), et(need.begin() + B, need.end());
        TRY(compact(m, &ev, &et));
        continue;
      }
    }
    st->v[6] += edges;
    relayouts = 0;
    // meshes whose pass found nothing to split are finished (checked after any relayout)
    bool newly_done = false;
    for (int i = 0; i < B && B > 1; ++i)
      if (!mdone[i] && need[i] == 0) mdone[i] = 1, newly_done = true;
    if (newly_done) {
      HIPCHK(hipMemcpyAsync(m->mdone, mdone.data(), sizeof(int) * B, hipMemcpyHostToDevice, m->s));
      HIPCHK(hipStreamSynchronize(m->s));
    }
    TRY(ensure(m, m->mid, (size_t)s.nn_pool));
    if (B == 1) {
      m->vused[0] = s.V;  // unchanged until the new slots are counted below
      m->tused[0] = s.T;
    }
    refine_mint(s, o->L_up2, m->vt1.p, m->mid.p, m->s);
    refine_split(s, o->L_up2, m->mid.p, m->tt1.p, m->s);
    for (int i = 0; i < B; ++i) {
      m->vused[i] += need[i];
      m->tused[i] += need[B + i];
    }
    if (B == 1) {
      s.V = V0 + nv;
      s.T = T0 + nt;
      m->vbase[1] = s.V;
      m->tbase[1] = s.T;
    }
    TRY(upload_ranges(m));
    st->v[4] += nv;
    st->v[8] += nv;
    st->v[9] += nt;
    ++p;
    // the next pass's read-back checks this build's error bits
    TRY(build_rows(m, p >= o->refine_passes));
  }
  s.mdone = nullptr;
  // the counts above come from the passes' read-backs; the last of those
  // also left the stream drained
  prof_flush(m);
  st->v[0] = p;
  st->v[7] = done ? 1 : 0;
  return done ? PM_OK : PM_W_NOT_CONVERGED;
}

pm_status pm_quality(pm_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM) {
  if (!m) return PM_E_ARG;
  int nparts = quality_parts(m);
  TRY(ensure(m, m->qpart, 2 * (size_t)nparts + 2));
  if (Q || qmin) {
    timed(m, PM_K_QUALITY, m->st.T,
          [&] { quality_sum(m->st, m->qpart.p, m->qpart.p + nparts, nparts, m->qpart.p + 2 * nparts, m->s); });
    HIPCHK(hipMemcpyAsync(m->hq, m->qpart.p + 2 * nparts, 2 * sizeof(double), hipMemcpyDeviceToHost, m->s));
  }
  if (dQdx || dQdM) timed(m, PM_K_ADJOINT, m->st.V, [&] { quality_adjoint(m->st, dQdx, dQdM, m->s); });
  TRY(sync(m));
  prof_flush(m);
  if (Q) *Q = m->hq[0];
  if (qmin) *qmin = m->hq[1];
  return PM_OK;
}

pm_status pm_adapt(pm_mesh* m, const pm_options* o, pm_stats* st) {
  if (!m || !o) return PM_E_ARG;
  if (bad_opts(o)) return fail(m, PM_E_ARG, "bad options");
  pm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  int run = 0;
  for (;;) {
    if (m->ad_phase == PM_PHASE_COARSEN && m->ad_iter >= o->max_iterations) m->ad_phase = PM_PHASE_SMOOTH;
    if (m->ad_phase == PM_PHASE_DONE) return PM_OK;
    if (o->max_phases > 0 && run == o->max_phases) return PM_W_PAUSED;
    pm_options po = *o;
    po.sweep = m->ad_phase == PM_PHASE_SMOOTH ? 0 : m->ad_iter;
    pm_stats ph;
    pm_status r;
    int phase = m->ad_phase;
    if (phase == PM_PHASE_COARSEN) r = pm_coarsen(m, &po, &ph);
    else if (phase == PM_PHASE_SWAP) r = pm_swap(m, &po, &ph);
    else if (phase == PM_PHASE_REFINE) r = pm_refine(m, &po, &ph);
    else r = pm_smooth(m, &po, &ph);
    if (r != PM_OK && r != PM_W_NOT_CONVERGED) return r;
    for (int k = 1; k < 16; ++k)
      if (k != 7) st->v[k] += ph.v[k];
    if (phase != PM_PHASE_SMOOTH && ph.v[4] > 0) m->ad_changed = 1;
    if (phase == PM_PHASE_COARSEN) {
      m->ad_phase = PM_PHASE_SWAP;
    } else if (phase == PM_PHASE_SWAP) {
      m->ad_phase = PM_PHASE_REFINE;
    } else if (phase == PM_PHASE_REFINE) {
      ++m->ad_iter;
      st->v[0] += 1;
      if (!m->ad_changed) st->v[7] = 1;
      m->ad_phase = m->ad_changed ? PM_PHASE_COARSEN : PM_PHASE_SMOOTH;
      m->ad_changed = 0;
    } else {
      m->ad_phase = PM_PHASE_DONE;
    }
    ++run;
  }
}

pm_status pm_get_context(const pm_mesh* m, pm_context* c) {
  if (!m || !c) return PM_E_ARG;
  c->seed = m->seed;
  c->iteration = m->ad_iter;
  c->phase = m->ad_phase;
  c->changed = m->ad_changed;
  c->reserved = 0;
  return PM_OK;
}

pm_status pm_set_context(pm_mesh* m, const pm_context* c) {
  if (!m || !c) return PM_E_ARG;
  if (c->iteration < 0 || c->iteration > 4095 || c->phase < PM_PHASE_COARSEN || c->phase > PM_PHASE_DONE ||
      (c->changed != 0 && c->changed != 1) || c->reserved != 0)
    return fail(m, PM_E_ARG, "bad context");
  m->seed = c->seed;
  m->ad_iter = c->iteration;
  m->ad_phase = c->phase;
  m->ad_changed = c->changed;
  return PM_OK;
}

pm_status pm_mesh_update(pm_mesh* m, const double* xy, const double* metric, int32_t mem_kind) {
  if (!m) return PM_E_ARG;
  if (mem_kind != PM_MEM_HOST && mem_kind != PM_MEM_DEVICE) return fail(m, PM_E_ARG, "bad mem_kind");
  if (m->st.B != 1) return fail(m, PM_E_ARG, "pm_mesh_update takes a single mesh");
  if (!xy && !metric) return PM_OK;
  Store& st = m->st;
  size_t V = (size_t)st.V;
  hipMemcpyKind k = mem_kind == PM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  // the old values, kept until the new ones pass the checks
  TRY(ensure(m, m->upd, 5 * V));
  double2* old_xy = (double2*)m->upd.p;
  Met* old_met = (Met*)(m->upd.p + 2 * V);
  if (xy) {
    HIPCHK(hipMemcpyAsync(old_xy, st.xy, sizeof(double2) * V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(st.xy, xy, sizeof(double2) * V, k, m->s));
  }
  if (metric) {
    HIPCHK(hipMemcpyAsync(old_met, st.met, sizeof(Met) * V, hipMemcpyDeviceToDevice, m->s));
    HIPCHK(hipMemcpyAsync(st.met, metric, sizeof(Met) * V, k, m->s));
  }
  k_validate(st, m->ctr, m->s);
  pm_status r = check_err(m);
  if (r != PM_OK) {
    if (xy) HIPCHK(hipMemcpyAsync(st.xy, old_xy, sizeof(double2) * V, hipMemcpyDeviceToDevice, m->s));
    if (metric) HIPCHK(hipMemcpyAsync(st.met, old_met, sizeof(Met) * V, hipMemcpyDeviceToDevice, m->s));
    TRY(sync(m));
    return r;
  }
  ++m->topo;  // the per-element tensors smoothing keeps follow the metric
  return PM_OK;
}

pm_status pm_quality_noalloc(pm_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM) {
  if (!m) return PM_E_ARG;
  int nparts = quality_parts(m);
  if (nparts > kQualityParts)  // cannot happen for a handle this library made (T < 2^30)
    return fail(m, PM_E_ARG, "pm_quality_noalloc: more than " + std::to_string(kQualityParts) + " partial sums");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (!m->scratch || dev != m->dev)
    return fail(m, PM_E_ARG, "pm_quality_noalloc: call it with the handle's device current");
  double* ps = m->scratch;
  if (Q || qmin) {
    quality_sum(m->st, ps, ps + nparts, nparts, ps + 2 * nparts, m->s);
    HIPCHK(hipMemcpyAsync(m->hq, ps + 2 * nparts, 2 * sizeof(double), hipMemcpyDeviceToHost, m->s));
  }
  if (dQdx || dQdM) quality_adjoint(m->st, dQdx, dQdM, m->s);
  HIPCHK(hipStreamSynchronize(m->s));
  if (Q) *Q = m->hq[0];
  if (qmin) *qmin = m->hq[1];
  return PM_OK;
}

pm_status pm_batch_create(const pm_mesh_desc* meshes, int32_t count, const pm_options* o, void* stream,
                          pm_mesh** out) {
  if (!out) return PM_E_ARG;
  *out = nullptr;
  if (!meshes || count < 1) return PM_E_ARG;
  pm_options def;
  fill_defaults(&def);
  if (!o) o = &def;
  if (bad_opts(o)) return PM_E_ARG;
  std::vector<int> vb(count + 1, 0), tb(count + 1, 0), vu(count), tu(count);
  for (int i = 0; i < count; ++i) {
    const pm_mesh_desc& d = meshes[i];
    if (!d.xy || !d.tri || !d.metric || d.mem_kind != PM_MEM_HOST || d.V < 3 || d.T < 1) return PM_E_ARG;
    int64_t cv = d.V + headroom((int)std::min<int64_t>(d.V, 1 << 29));
    int64_t ct = d.T + headroom((int)std::min<int64_t>(d.T, 1 << 29));
    if (vb[i] + cv > (1ll << 30) || tb[i] + ct > (1ll << 30)) return PM_E_ARG;
    vu[i] = (int)d.V;
    tu[i] = (int)d.T;
    vb[i + 1] = vb[i] + (int)cv;
    tb[i + 1] = tb[i] + (int)ct;
  }
  int nV = vb[count], nT = tb[count];
  // the concatenated store on the host: unused slots are dead (identity metric)
  std::vector<double> xy(2 * (size_t)nV, 0.0), met(3 * (size_t)nV, 0.0);
  std::vector<uint8_t> tag(nV, 0), va(nV, 0);
  std::vector<Elem> tri(nT, make_int4(0, 0, 0, 0));
  std::vector<int> vmesh(nV), tmesh(nT);
  g_create_err.clear();
  for (int i = 0; i < count; ++i) {
    const pm_mesh_desc& d = meshes[i];
    for (int v = vb[i]; v < vb[i + 1]; ++v) {
      vmesh[v] = i;
      met[3 * (size_t)v] = 1.0;
      met[3 * (size_t)v + 2] = 1.0;
    }
    for (int t = tb[i]; t < tb[i + 1]; ++t) tmesh[t] = i;
    for (int64_t v = 0; v < d.V; ++v) {
      size_t g = (size_t)(vb[i] + v);
      double x = d.xy[2 * v], y = d.xy[2 * v + 1];
      xy[2 * g] = x;
      xy[2 * g + 1] = y;
      for (int k = 0; k < 3; ++k) met[3 * g + k] = d.metric[3 * v + k];
      va[g] = 1;
      if (d.tags) {
        tag[g] = d.tags[v];
      } else {
        uint8_t tg = 0;
        if (x == 0.0) tg |= 1;
        if (x == 1.0) tg |= 2;
        if (y == 0.0) tg |= 4;
        if (y == 1.0) tg |= 8;
        tag[g] = tg;
      }
    }
    for (int64_t t = 0; t < d.T; ++t) {
      int a = d.tri[3 * t], b = d.tri[3 * t + 1], c = d.tri[3 * t + 2];
      if (a < 0 || b < 0 || c < 0 || a >= d.V || b >= d.V || c >= d.V) {
        g_create_err = "mesh " + std::to_string(i) + ": element id out of range";
        return PM_E_MESH;
      }
      a += vb[i];
      b += vb[i];
      c += vb[i];
      Elem e;
      if (a < b && a < c) e = make_int4(a, b, c, 1);
      else if (b < a && b < c) e = make_int4(b, c, a, 1);
      else e = make_int4(c, a, b, 1);
      tri[tb[i] + t] = e;
    }
  }
  pm_mesh* m = new (std::nothrow) pm_mesh();
  if (!m) return PM_E_NOMEM;
  m->s = (hipStream_t)stream;
  m->seed = o->seed;
  m->slack = o->slack;
  m->headroom = o->pool_headroom > 0.0 ? o->pool_headroom : 3.0;
  m->st.qk = o->quality;
  if (o->allocator) m->va = *o->allocator;
  auto bail = [&](pm_status st) {
    g_create_err = m->err.empty() ? std::string("pm_batch_create failed") : m->err;
    pm_mesh_destroy(m);
    return st;
  };
  if (dalloc(m, &m->ctr, C_COUNT) != PM_OK || !pinned_get(m)) return bail(PM_E_NOMEM);
  if (scratch_setup(m) != PM_OK) return bail(PM_E_DEVICE);
  zero_ints(m->ctr, C_COUNT, m->s);
  set_int(m->ctr + C_FAILEP, INT_MAX, m->s);
  Store& st = m->st;
  st.B = count;
  if (grow_vertices(m, nV) != PM_OK || grow_elements(m, nT) != PM_OK) return bail(PM_E_NOMEM);
  st.V = nV;
  st.T = nT;
  if (dalloc(m, &st.vmesh, nV) != PM_OK || dalloc(m, &st.tmesh, nT) != PM_OK) return bail(PM_E_NOMEM);
  double* xyraw = nullptr;
  if (dalloc(m, &xyraw, 2 * (size_t)nV) != PM_OK) return bail(PM_E_NOMEM);
  // the copies below do not wait for the stream: let its queued clears (and
  // any earlier user of these cached blocks) finish first
  if (hipStreamSynchronize(m->s) != hipSuccess) return bail(PM_E_DEVICE);
  bool ok = hipMemcpy(xyraw, xy.data(), sizeof(double) * xy.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.met, met.data(), sizeof(double) * met.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.tag, tag.data(), tag.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.valive, va.data(), va.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.tri, tri.data(), sizeof(Elem) * tri.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.vmesh, vmesh.data(), sizeof(int) * vmesh.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.tmesh, tmesh.data(), sizeof(int) * tmesh.size(), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    dfree(m, xyraw, 2 * (size_t)nV);
    return bail(PM_E_DEVICE);
  }
  xy_in(xyraw, nV, st.xy, m->s);
  (void)hipStreamSynchronize(m->s);
  dfree(m, xyraw, 2 * (size_t)nV);
  m->vbase = vb;
  m->tbase = tb;
  m->vused = vu;
  m->tused = tu;
  if (upload_ranges(m) != PM_OK) return bail(PM_E_DEVICE);
  k_validate(st, m->ctr, m->s);
  pm_status r = check_err(m);
  if (r != PM_OK) return bail(r);
  r = build_rows(m);
  if (r != PM_OK) return bail(r);
  *out = m;
  return PM_OK;
}

pm_status pm_batch_count(const pm_mesh* m, int32_t* count) {
  if (!m || !count) return PM_E_ARG;
  *count = m->st.B;
  return PM_OK;
}

pm_status pm_batch_sizes(const pm_mesh* m, int32_t i, int64_t* V, int64_t* T) {
  if (!m || i < 0 || i >= m->st.B) return PM_E_ARG;
  if (V) *V = m->vused[i];
  if (T) *T = m->tused[i];
  return PM_OK;
}

pm_status pm_batch_export(pm_mesh* m, int32_t i, double* xy, int32_t* tri, double* metric, uint8_t* tags,
                          uint8_t* valive, uint8_t* talive) {
  if (!m || i < 0 || i >= m->st.B) return PM_E_ARG;
  Store& st = m->st;
  int v0 = m->vbase[i], nv = m->vused[i], t0 = m->tbase[i], nt = m->tused[i];
  if (xy) HIPCHK(hipMemcpyAsync(xy, st.xy + v0, sizeof(double2) * nv, hipMemcpyDeviceToHost, m->s));
  if (metric) HIPCHK(hipMemcpyAsync(metric, st.met + v0, sizeof(Met) * nv, hipMemcpyDeviceToHost, m->s));
  if (tags) HIPCHK(hipMemcpyAsync(tags, st.tag + v0, nv, hipMemcpyDeviceToHost, m->s));
  if (valive) HIPCHK(hipMemcpyAsync(valive, st.valive + v0, nv, hipMemcpyDeviceToHost, m->s));
  std::vector<Elem> e(nt);
  HIPCHK(hipMemcpyAsync(e.data(), st.tri + t0, sizeof(Elem) * nt, hipMemcpyDeviceToHost, m->s));
  TRY(sync(m));
  for (int t = 0; t < nt; ++t) {
    if (tri) {
      tri[3 * t] = e[t].w ? e[t].x - v0 : e[t].x;
      tri[3 * t + 1] = e[t].w ? e[t].y - v0 : e[t].y;
      tri[3 * t + 2] = e[t].w ? e[t].z - v0 : e[t].z;
    }
    if (talive) talive[t] = e[t].w ? 1 : 0;
  }
  return PM_OK;
}

pm_status pm_batch_quality(pm_mesh* m, double* Q, double* qmin) {
  if (!m) return PM_E_ARG;
  int B = m->st.B;
  TRY(ensure(m, m->qpart, 2 * (size_t)B + 2));
  quality_per_mesh(m->st, m->qpart.p, m->s);
  std::vector<double> h(2 * (size_t)B);
  HIPCHK(hipMemcpyAsync(h.data(), m->qpart.p, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, m->s));
  TRY(sync(m));
  for (int i = 0; i < B; ++i) {
    if (Q) Q[i] = h[2 * i];
    if (qmin) qmin[i] = h[2 * i + 1];
  }
  return PM_OK;
}

pm_status pm_profile(pm_mesh* m, uint32_t mask) {
  if (!m) return PM_E_ARG;
  TRY(sync(m));
  prof_flush(m);
  m->prof.mask = mask;
  for (int k = 0; k < PM_K_COUNT; ++k) {
    m->prof.ms[k] = 0.0;
    m->prof.launches[k] = m->prof.units[k] = 0;
  }
  stripe_zero(m->ctr, S_PJP, 2, m->s);
  stripe_zero(m->ctr, S_POPS, 1, m->s);
  return sync(m);
}

pm_status pm_profile_read(pm_mesh* m, int32_t id, double* ms, int64_t* launches, int64_t* units) {
  if (!m || id < 0 || id > PM_K_COMMIT_OPS) return PM_E_ARG;
  TRY(sync(m));
  prof_flush(m);
  stripe_sum(m->ctr, S_PJP, 2, C_PROF_JP, m->s);
  stripe_sum(m->ctr, S_POPS, 1, C_PROF_OPS, m->s);
  TRY(read_ctr(m, C_PROF_JP, 3));
  int k = id == PM_K_COMMIT_OPS ? PM_K_COMMIT : id;
  if (ms) *ms = m->prof.ms[k];
  if (launches) *launches = m->prof.launches[k];
  if (units) {
    *units = m->prof.units[k];
    if (id == PM_K_JP) *units = m->hctr[C_PROF_JP];
    if (id == PM_K_COMMIT) *units = m->hctr[C_PROF_ROWS];
    if (id == PM_K_COMMIT_OPS) *units = m->hctr[C_PROF_OPS];
  }
  return PM_OK;
}

pm_status pm_fp64_selfcheck(const double* a, const double* b, int64_t n, double* quot, double* root) {
  if (!a || !b || !quot || !root || n < 0 || n > (1ll << 28)) return PM_E_ARG;
  if (n == 0) return PM_OK;
  double* d = nullptr;
  size_t bytes = sizeof(double) * (size_t)n;
  if (hipMalloc((void**)&d, 4 * bytes) != hipSuccess) return PM_E_NOMEM;
  bool ok = hipMemcpy(d, a, bytes, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(d + n, b, bytes, hipMemcpyHostToDevice) == hipSuccess;
  if (ok) {
    fp64_probe(d, d + n, (int)n, d + 2 * n, d + 3 * n, nullptr);
    ok = hipDeviceSynchronize() == hipSuccess &&
         hipMemcpy(quot, d + 2 * n, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemcpy(root, d + 3 * n, bytes, hipMemcpyDeviceToHost) == hipSuccess;
  }
  (void)hipFree(d);
  return ok ? PM_OK : PM_E_DEVICE;
}

}  // extern "C"
