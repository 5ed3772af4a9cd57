// Tetrahedral meshes of the unit cube (Sec. 4's extrusion of the method to
// three dimensions): coarsening, refinement and Laplacian smoothing in the
// metric over Jones-Plassmann colour classes, as independent sets; no swaps.
//
// Layout: per vertex xyz (double4, w unused), the six metric entries, tag and
// live bytes, a row header int4 (nn_off, nn_cnt, ne_off, ne_cnt); per element
// an int4 of vertex ids and a live byte. Rows are rebuilt from the element
// list after every class that changes the topology (count, scan, fill, sort
// per vertex): a class's members are pairwise non-adjacent, so the class
// kernel writes only its members' own elements, and the next class reads the
// current graph. Every floating-point expression is written in one fixed
// order and compiled without contraction, so decisions are the ones a serial
// IEEE-754 program makes from the same inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pm3.h"
#include "common.hpp"
#include "kern.hpp"
#include "blocks.hpp"

namespace pm3 {

using pm::gstride;
using pm::gtid;
using pm::make_ctx;
using pm::stream_seed;
using pm::vkey;
using pm::kWave;

constexpr int kB = 256;
constexpr int kMaxColours = 256;
enum { PH3_COARSEN = 1, PH3_SMOOTH = 3 };

// device counters
enum {
  K_ERR = 0,        // error bits
  K_COLOURED = 1,   // vertices coloured in a JP iteration
  K_NCOL = 2,       // colours used (max + 1)
  K_EVAL = 3,       // members evaluated
  K_DEFER = 4,      // members deferred by re-validation
  K_COMMIT = 5,     // collapses / accepted moves
  K_EDGES = 6,      // edges tested by refinement
  K_TOTAL = 7,      // scan total
  K_CCOMMIT = 8,    // collapses of the class in progress (gates its row commit)
  K_ROOM = 9,       // a row commit ran out of room (pool stripe full, or a row past the wavefront form)
  K_ROOMEP = 10,    // the epoch of the class whose commit ran out of room
  K_NROWS = 11,     // rows stamped by the class in progress (the length of its row list)
  K_COUNT = 16
};
enum { E_MESH = 1, E_METRIC = 2, E_COLOURS = 4, E_LEAVES = 8 };

struct Met6 {
  double a00, a01, a02, a11, a12, a22;
};

struct Store3 {
  int V = 0, T = 0;
  double4* xyz = nullptr;
  Met6* met = nullptr;
  uint8_t* tag = nullptr;
  uint8_t* valive = nullptr;
  int4* tet = nullptr;
  uint8_t* talive = nullptr;
  int4* hdr = nullptr;  // (nn_off, nn_cnt, ne_off, ne_cnt); NN's slot is 3 x NE's
  int* cap = nullptr;   // NE slot capacity of each row (NN's: 3 x)
  int* nn = nullptr;
  int* ne = nullptr;
};

// ---- canonical geometry --------------------------------------------------------------

__device__ __forceinline__ Met6 edge_met(const Met6& p, const Met6& q) {
  return Met6{(p.a00 + q.a00) * 0.5, (p.a01 + q.a01) * 0.5, (p.a02 + q.a02) * 0.5,
              (p.a11 + q.a11) * 0.5, (p.a12 + q.a12) * 0.5, (p.a22 + q.a22) * 0.5};
}

// e^T M e, bitwise the same for -e
__device__ __forceinline__ double qform(const Met6& e, double dx, double dy, double dz) {
  return (((e.a00 * dx) * dx + ((2.0 * e.a01) * dx) * dy) + ((2.0 * e.a02) * dx) * dz) +
         (((e.a11 * dy) * dy + ((2.0 * e.a12) * dy) * dz) + (e.a22 * dz) * dz);
}

__device__ __forceinline__ double len2(const Store3& st, int i, int j) {
  double4 pi = st.xyz[i], pj = st.xyz[j];
  return qform(edge_met(st.met[i], st.met[j]), pj.x - pi.x, pj.y - pi.y, pj.z - pi.z);
}

__device__ __forceinline__ double det3(const Met6& g) {
  return (g.a00 * (g.a11 * g.a22 - g.a12 * g.a12) - g.a01 * (g.a01 * g.a22 - g.a12 * g.a02)) +
         g.a02 * (g.a01 * g.a12 - g.a11 * g.a02);
}

struct Geo3 {
  double4 p[4];
  Met6 m;
};

__device__ __forceinline__ int at4(const int4& t, int k) { return k == 0 ? t.x : (k == 1 ? t.y : (k == 2 ? t.z : t.w)); }
__device__ __forceinline__ bool has4(const int4& t, int v) { return t.x == v || t.y == v || t.z == v || t.w == v; }
__device__ __forceinline__ int4 replace4(int4 t, int v, int u) {
  if (t.x == v) t.x = u;
  else if (t.y == v) t.y = u;
  else if (t.z == v) t.z = u;
  else if (t.w == v) t.w = u;
  return t;
}

// orientation-preserving canonical order: the smallest id first (one of the
// four even permutations that bring a vertex to the front), then the other
// three rotated so that the smallest of them comes second
__device__ __forceinline__ int4 canon4(int4 t) {
  int k = 0, mn = t.x;
  if (t.y < mn) { k = 1; mn = t.y; }
  if (t.z < mn) { k = 2; mn = t.z; }
  if (t.w < mn) { k = 3; }
  int4 r;
  if (k == 0) r = t;
  else if (k == 1) r = make_int4(t.y, t.x, t.w, t.z);
  else if (k == 2) r = make_int4(t.z, t.w, t.x, t.y);
  else r = make_int4(t.w, t.z, t.y, t.x);
  int j = 1;
  int mj = r.y;
  if (r.z < mj) { j = 2; mj = r.z; }
  if (r.w < mj) { j = 3; }
  if (j == 2) r = make_int4(r.x, r.z, r.w, r.y);
  else if (j == 3) r = make_int4(r.x, r.w, r.y, r.z);
  return r;
}

// element t's geometry; vertex ov, if present, placed at q
__device__ __forceinline__ Geo3 geo(const Store3& st, int4 t, int ov, double4 q) {
  Geo3 g;
  int id[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) g.p[k] = id[k] == ov ? q : st.xyz[id[k]];
  Met6 a = st.met[t.x], b = st.met[t.y], c = st.met[t.z], d = st.met[t.w];
  g.m = Met6{(((a.a00 + b.a00) + c.a00) + d.a00) / 4.0, (((a.a01 + b.a01) + c.a01) + d.a01) / 4.0,
             (((a.a02 + b.a02) + c.a02) + d.a02) / 4.0, (((a.a11 + b.a11) + c.a11) + d.a11) / 4.0,
             (((a.a12 + b.a12) + c.a12) + d.a12) / 4.0, (((a.a22 + b.a22) + c.a22) + d.a22) / 4.0};
  return g;
}

__device__ __forceinline__ double vol6(const Geo3& g) {
  double ax = g.p[1].x - g.p[0].x, ay = g.p[1].y - g.p[0].y, az = g.p[1].z - g.p[0].z;
  double bx = g.p[2].x - g.p[0].x, by = g.p[2].y - g.p[0].y, bz = g.p[2].z - g.p[0].z;
  double cx = g.p[3].x - g.p[0].x, cy = g.p[3].y - g.p[0].y, cz = g.p[3].z - g.p[0].z;
  return (ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx)) + az * (bx * cy - by * cx);
}

// sum of the six squared metric edge lengths, edges (01, 02, 03, 12, 13, 23)
__device__ __forceinline__ double edge_sum(const Geo3& g) {
  const int E0[6] = {0, 0, 0, 1, 1, 2}, E1[6] = {1, 2, 3, 2, 3, 3};
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double4 a = g.p[E0[k]], b = g.p[E1[k]];
    s = s + qform(g.m, b.x - a.x, b.y - a.y, b.z - a.z);
  }
  return s;
}

// q^3 = 432 det(M) D^2 / S^3 (decisions)
__device__ __forceinline__ double qual3(const Geo3& g) {
  double D = vol6(g), S = edge_sum(g), det = det3(g.m);
  return (((432.0 * det) * D) * D) / ((S * S) * S);
}

// q = 12 (3 |K|_M)^(2/3) / S (reported)
__device__ __forceinline__ double qual(const Geo3& g) {
  double D = vol6(g), S = edge_sum(g), det = det3(g.m);
  return (12.0 * cbrt(((det * D) * D) * 0.25)) / S;
}

__device__ __forceinline__ bool tag_ok(const Store3& st, int v, int u) { return (st.tag[v] & ~st.tag[u]) == 0; }

__device__ __forceinline__ void stripe_add(int* ctr, int slot, int x) {
  if (x) atomicAdd(&ctr[slot], x);
}

// ---- input, validation ------------------------------------------------------------------

__global__ void k_in(const double* __restrict__ xyz, const int* __restrict__ tet, const double* __restrict__ met,
                     Store3 st, int* ctr) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    st.xyz[v] = make_double4(xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2], 0.0);
    const double* p = met + 6 * v;
    Met6 g{p[0], p[1], p[2], p[3], p[4], p[5]};
    st.met[v] = g;
    st.valive[v] = 1;
    if (!(g.a00 > 0.0) || !(g.a00 * g.a11 - g.a01 * g.a01 > 0.0) || !(det3(g) > 0.0)) atomicOr(&ctr[K_ERR], E_METRIC);
  }
  for (int t = gtid(); t < st.T; t += gstride()) {
    int4 e = make_int4(tet[4 * t], tet[4 * t + 1], tet[4 * t + 2], tet[4 * t + 3]);
    bool bad = e.x < 0 || e.y < 0 || e.z < 0 || e.w < 0 || e.x >= st.V || e.y >= st.V || e.z >= st.V ||
               e.w >= st.V || e.x == e.y || e.x == e.z || e.x == e.w || e.y == e.z || e.y == e.w || e.z == e.w;
    if (bad) {
      atomicOr(&ctr[K_ERR], E_MESH);
      e = make_int4(0, 1, 2, 3);
    }
    st.tet[t] = canon4(e);
    st.talive[t] = 1;
  }
}

__global__ void k_tags(Store3 st) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    double4 p = st.xyz[v];
    uint8_t t = 0;
    if (p.x == 0.0) t |= 1;
    if (p.x == 1.0) t |= 2;
    if (p.y == 0.0) t |= 4;
    if (p.y == 1.0) t |= 8;
    if (p.z == 0.0) t |= 16;
    if (p.z == 1.0) t |= 32;
    st.tag[v] = t;
  }
}

__global__ void k_orient(Store3 st, int* ctr) {
  for (int t = gtid(); t < st.T; t += gstride()) {
    int4 e = st.tet[t];
    if (!(vol6(geo(st, e, -1, make_double4(0, 0, 0, 0))) > 0.0)) atomicOr(&ctr[K_ERR], E_MESH);
  }
}

// ---- rows from the element list ----------------------------------------------------------

__global__ void k_ne_count(Store3 st, int* cnt) {
  for (int t = gtid(); t < st.T; t += gstride()) {
    if (!st.talive[t]) continue;
    int4 e = st.tet[t];
    atomicAdd(&cnt[e.x], 1);
    atomicAdd(&cnt[e.y], 1);
    atomicAdd(&cnt[e.z], 1);
    atomicAdd(&cnt[e.w], 1);
  }
}

__global__ void k_ne_fill(Store3 st, const int* __restrict__ off, int* cur) {
  for (int t = gtid(); t < st.T; t += gstride()) {
    if (!st.talive[t]) continue;
    int4 e = st.tet[t];
    int id[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int pos = atomicAdd(&cur[id[k]], 1);
      st.ne[off[id[k]] + pos] = t;
    }
  }
}

__device__ void isort(int* a, int n) {
  for (int i = 1; i < n; ++i) {
    int x = a[i], j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

// Serial form for rows longer than a wavefront: sort NE(v) in place; NN(v) =
// the sorted distinct other vertices of NE(v)'s elements, inserted one at a
// time into a slot of three entries per NE entry (a binary search finds and
// skips repeats).
__device__ void rows_finish_serial(const Store3& st, int v, int o, int n) {
  int* row = st.ne + o;
  isort(row, n);
  int* nb = st.nn + 3 * o;
  int u = 0;
  for (int i = 0; i < n; ++i) {
    int4 e = st.tet[row[i]];
    int id[4] = {e.x, e.y, e.z, e.w};
    for (int j = 0; j < 4; ++j) {
      int x = id[j];
      if (x == v) continue;
      int lo = 0, hi = u;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (nb[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      if (lo < u && nb[lo] == x) continue;
      for (int q = u; q > lo; --q) nb[q] = nb[q - 1];
      nb[lo] = x;
      ++u;
    }
  }
  st.hdr[v] = make_int4(3 * o, u, o, n);
  st.cap[v] = n;
}

// Bitonic sorting networks across a wavefront, ascending. sort_lanes: one
// value per lane (value i on lane i). sort_lanes_r<R>: R per lane (value i on
// lane i / R, register i % R); pairs R or more apart are exchanged by
// shuffles, nearer ones inside a lane. lanes_at<R>: each lane's value of
// index i (its own i) from the R-per-lane layout.
__device__ __forceinline__ int sort_lanes(int a) {
  int lane = __lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int o = __shfl_xor(a, j);
      bool up = (lane & k) == 0, lo = (lane & j) == 0;
      a = lo == up ? min(a, o) : max(a, o);
    }
  return a;
}
template <int R>
__device__ __forceinline__ void sort_lanes_r(int (&a)[R]) {
  int lane = __lane_id();
#pragma unroll
  for (int k = 2; k <= R * kWave; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i = R * lane + r;
          int o = __shfl_xor(a[r], j / R);
          bool up = (i & k) == 0, lo = (i & j) == 0;
          a[r] = lo == up ? min(a[r], o) : max(a[r], o);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (r & j) continue;
          int r2 = r | j, i = R * lane + r;
          bool up = (i & k) == 0;
          int x = a[r], y = a[r2];
          a[r] = up ? min(x, y) : max(x, y);
          a[r2] = up ? max(x, y) : min(x, y);
        }
      }
    }
}
template <int R>
__device__ __forceinline__ int lanes_at(const int (&a)[R], int i) {
  int src = i / R, q = i % R, out = INT_MAX;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int x = __shfl(a[r], src);
    if (r == q) out = x;
  }
  return out;
}

// Sorted distinct values of the R-per-lane layout `a` (sorted, INT_MAX for
// none) written to dst[0, u) where dst is the same on every lane; returns u.
template <int R>
__device__ __forceinline__ int put_distinct(const int (&a)[R], int* dst) {
  int lane = __lane_id();
  int before = __shfl_up(a[R - 1], 1);
  bool keep[R];
  int mine = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int prev = r > 0 ? a[r - 1] : (lane > 0 ? before : INT_MIN);
    keep[r] = a[r] != INT_MAX && a[r] != prev;
    mine += keep[r] ? 1 : 0;
  }
  int incl = mine;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int x = __shfl_up(incl, d);
    if (lane >= d) incl += x;
  }
  int pos = incl - mine;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (keep[r]) dst[pos++] = a[r];
  return __shfl(incl, kWave - 1);
}

// ---- row commit after a collapse class ---------------------------------------------------------
// The collapse kernel stamps every row its members change with the class
// epoch (own) and records each committed member's target (rec). One
// wavefront per stamped row x rebuilds it: the candidates are NE(x) and the
// NE rows of the members collapsed onto x (neighbours of x whose record
// names x); NE(x) = the sorted distinct candidates that are live and hold x,
// NN(x) = the sorted distinct other vertices of those elements. The row is
// written in place when it fits its slot, else in fresh space from one of
// kTopStripes bump pointers (a stripe per row id modulo the count, each with
// its own range of the pool). Rows past this form (NE above 4 kWave, an
// absorbed row above 2 kWave, more than two absorbed rows) and a full stripe
// set the room counter instead; the later classes of the round then stand
// down and the host rebuilds every row before it runs them again.
constexpr int kTopStripes = 64;
constexpr int kTopStride = 16;  // ints between two stripes' bump pointers

__device__ __forceinline__ void room3(int* ctr, int epoch) {
  ctr[K_ROOMEP] = epoch;
  atomicOr(&ctr[K_ROOM], 1);
}

// Row x from its candidates, RC slots per lane: NE(x) (slot o, count n)
// followed by the rows of the absorbed members (za[j], counts ca[j], j <
// nab), at most RC kWave candidates in all. RN = 2 RC slots per lane hold
// the NN candidates. Writes the row in place when it holds at most capx
// entries, else in fresh space of x's stripe (tops given), and returns
// false, having written nothing, when the row has more than RN/4 kWave
// entries or the stripe is full. Every lane of the wavefront makes this call.
constexpr int kAbsMax = 8;  // absorbed rows a row commit takes
template <int RC, int RN>
__device__ __forceinline__ bool put_row3(const Store3& st, int x, int o, int n, int capx, const int (&za)[kAbsMax],
                                         const int (&ca)[kAbsMax], int nab, int* tops, int64_t base, int64_t per) {
  static_assert(RN == 2 * RC, "three other vertices per element, four slots each");
  int lane = __lane_id();
  int a[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    // candidate idx of the list NE(x), then the absorbed rows in turn
    int idx = r * kWave + lane;
    int src = -1;
    if (idx < n) {
      src = o + idx;
    } else {
      int q = idx - n;
      for (int j = 0; j < nab; ++j) {
        if (q < ca[j]) {
          src = za[j] + q;
          break;
        }
        q -= ca[j];
      }
    }
    a[r] = src >= 0 ? st.ne[src] : -1;
  }
  {
    int4 e[RC];
    uint8_t al[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      e[r] = st.tet[max(a[r], 0)];
      al[r] = st.talive[max(a[r], 0)];
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) a[r] = a[r] >= 0 && al[r] && has4(e[r], x) ? a[r] : INT_MAX;
  }
  sort_lanes_r<RC>(a);
  // repeats out, then sorted again: the distinct entries come first
  {
    int before = __shfl_up(a[RC - 1], 1);
    bool dup[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      int prev = r > 0 ? a[r - 1] : (lane > 0 ? before : INT_MIN);
      dup[r] = a[r] != INT_MAX && a[r] == prev;
    }
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (dup[r]) a[r] = INT_MAX;
  }
  sort_lanes_r<RC>(a);
  int m = 0;
#pragma unroll
  for (int r = 0; r < RC; ++r) m += a[r] != INT_MAX ? 1 : 0;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) m += __shfl_xor(m, d);
  constexpr int K = RN / 4;  // elements per lane
  if (m > K * kWave) return false;
  int el[K];
#pragma unroll
  for (int k = 0; k < K; ++k) el[k] = lanes_at<RC>(a, lane + k * kWave);
  // the slot: in place, else fresh space from the row's stripe
  int off = o, cap = capx;
  if (m > capx) {
    int need = 2 * m;
    int sidx = x % kTopStripes;
    int got = 0;
    if (lane == 0) got = atomicAdd(&tops[sidx * kTopStride], need);
    got = __shfl(got, 0);
    if ((int64_t)got + need > base + (int64_t)(sidx + 1) * per) return false;
    off = got;
    cap = need;
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (lane + k * kWave < m) st.ne[off + k * kWave + lane] = el[k];
  // NN: the other three vertices of each element, four slots per element
  int b[RN];
#pragma unroll
  for (int r = 0; r < RN; ++r) b[r] = INT_MAX;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (lane + k * kWave < m) {
      int4 f = st.tet[el[k]];
      int id[4] = {f.x, f.y, f.z, f.w}, q = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (id[j] != x && q < 3) b[4 * k + q++] = id[j];
    }
  }
  sort_lanes_r<RN>(b);
  int u = put_distinct<RN>(b, st.nn + 3 * (int64_t)off);
  if (lane == 0) {
    st.hdr[x] = make_int4(3 * off, u, off, m);
    st.cap[x] = cap;
  }
  return true;
}

// one stamped row (every lane of the wavefront)
__device__ __forceinline__ void commit_row3(const Store3& st, int x, int epoch, const int2* __restrict__ rec,
                                            int* tops, int64_t base, int64_t per, int* ctr) {
  int lane = __lane_id();
  int4 h = st.hdr[x];
  int capx = st.cap[x];
  if (h.y > 4 * kWave) {
    if (lane == 0) room3(ctr, epoch);
    return;
  }
  // members collapsed onto x: neighbours whose record names x
  int w[4];
  uint64_t bal[4];
  int nab = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int j = k * kWave + lane;
    w[k] = j < h.y ? st.nn[h.x + j] : -1;
    int2 r = w[k] >= 0 ? rec[w[k]] : make_int2(-1, -1);
    bal[k] = __ballot(r.x == epoch && r.y == x);
    nab += __popcll(bal[k]);
  }
  int za[kAbsMax], ca[kAbsMax];
  int tot = h.w;
  if (nab <= kAbsMax) {
    int got = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint64_t b = bal[k];
      while (b) {
        int l = __ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        int z = __shfl(w[k], l);
        int4 hz = st.hdr[z];
        za[got] = hz.z;
        ca[got] = hz.w;
        tot += hz.w;
        ++got;
      }
    }
  }
  // the smaller form when every candidate could be kept in it
  bool ok = false;
  if (nab <= kAbsMax && tot <= 2 * kWave)
    ok = put_row3<4, 8>(st, x, h.z, h.w, capx, za, ca, nab, tops, base, per);
  else if (nab <= kAbsMax && tot <= 8 * kWave)
    ok = put_row3<8, 16>(st, x, h.z, h.w, capx, za, ca, nab, tops, base, per);
  if (!ok && lane == 0) room3(ctr, epoch);
}

// Two launch shapes rebuild the same rows, each once. Vertex order (large
// classes): each wavefront takes a range of vertex slots, reads their stamps
// a wavefront at a time and rebuilds the stamped rows in turn, so
// consecutive wavefronts read nearby rows. Row list (small classes): each
// wavefront takes rows of the class's row list in a wavefront-strided loop,
// and the grid is sized by the class rather than by the mesh.
__global__ void __launch_bounds__(256) k_commit3(Store3 st, int epoch, const int* __restrict__ own,
                                                 const int2* __restrict__ rec, int* tops, int64_t base,
                                                 int64_t per, int* ctr) {
  if (ctr[K_CCOMMIT] == 0 || ctr[K_ROOM]) return;
  int lane = __lane_id();
  int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  int nw = (int)((int64_t)gridDim.x * blockDim.x / kWave);
  int per_wave = (st.V + nw - 1) / nw;
  int x0 = (int)min((int64_t)wid * per_wave, (int64_t)st.V), x1 = min(st.V, x0 + per_wave);
  for (int c0 = x0; c0 < x1; c0 += kWave) {
    int xi = c0 + lane;
    uint64_t dm = __ballot(xi < x1 && own[xi] == epoch);
    while (dm) {
      int l = __ffsll((unsigned long long)dm) - 1;
      dm &= dm - 1;
      commit_row3(st, c0 + l, epoch, rec, tops, base, per, ctr);
    }
  }
}

__global__ void __launch_bounds__(256) k_commit3_list(Store3 st, int epoch, const int* __restrict__ rows,
                                                      const int2* __restrict__ rec, int* tops, int64_t base,
                                                      int64_t per, int* ctr) {
  if (ctr[K_CCOMMIT] == 0 || ctr[K_ROOM]) return;
  int n = ctr[K_NROWS];
  int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  int nw = (int)((int64_t)gridDim.x * blockDim.x / kWave);
  for (int i = wid; i < n; i += nw) commit_row3(st, rows[i], epoch, rec, tops, base, per, ctr);
}

// the start of a class: its collapse count and its row list emptied
__global__ void k_class_start(int* ctr) {
  if (threadIdx.x == 0) {
    ctr[K_CCOMMIT] = 0;
    ctr[K_NROWS] = 0;
  }
}

// Sorted rows from the element lists gathered in build order: NE(v) sorted;
// NN(v) = the sorted distinct other vertices of NE(v)'s elements, in a slot
// of three entries per NE entry. One wavefront per vertex: NE(v) one entry
// per lane through the lane network; the three other vertices of each
// element in four slots per lane (the fourth empty) through the
// four-per-lane network, repeats dropped by comparing each slot with the one
// before it. Rows of more than kWave elements take the serial form on the
// wavefront's first lane.
__global__ void __launch_bounds__(256) k_rows_finish(Store3 st, const int* __restrict__ off, const int* __restrict__ cnt) {
  int lane = __lane_id();
  int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  int nw = (int)((int64_t)gridDim.x * blockDim.x / kWave);
  for (int v = wid; v < st.V; v += nw) {
    int o = off[v], n = cnt[v];
    if (n > kWave) {
      // in place (capacity n), no absorbed rows: the row always fits
      const int none[kAbsMax] = {};
      if (n > 8 * kWave || !put_row3<8, 16>(st, v, o, n, n, none, none, 0, nullptr, 0, 0))
        if (lane == 0) rows_finish_serial(st, v, o, n);
      continue;
    }
    bool has = lane < n;
    int t = has ? st.ne[o + lane] : INT_MAX;
    int4 e = st.tet[has ? t : 0];
    int a[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    if (has) {
      int id[4] = {e.x, e.y, e.z, e.w};
      int q = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (id[j] != v && q < 3) a[q++] = id[j];
    }
    t = sort_lanes(t);
    if (has) st.ne[o + lane] = t;
    sort_lanes_r<4>(a);
    int u = put_distinct<4>(a, st.nn + 3 * o);
    if (lane == 0) {
      st.hdr[v] = make_int4(3 * o, u, o, n);
      st.cap[v] = n;
    }
  }
}

// the stripes' bump pointers after a full row build: stripe s owns
// [base + s per, base + (s + 1) per)
__global__ void k_tops_init(int* tops, int64_t base, int64_t per) {
  int s = (int)threadIdx.x;
  if (s < kTopStripes) tops[s * kTopStride] = (int)(base + (int64_t)s * per);
}

// ---- colouring (Sec. 3.2) -----------------------------------------------------------------
// One Jones-Plassmann iteration `it`: a waiting vertex takes the first colour
// free among its coloured neighbours once every active neighbour with a
// larger key was coloured in an earlier iteration. A colour is stored with
// its iteration, (it << 8) | colour, and a neighbour coloured in this same
// iteration counts as waiting, so the result does not depend on the order in
// which the threads run: the greedy first-fit colouring in descending key
// order. k_jp_strip leaves the colours alone once the colouring is done. A
// vertex that has to wait remembers the neighbour it waits for (blk) and
// reads its row again only once that neighbour has a colour. Counts go to
// the counters once per wavefront.
__device__ __forceinline__ bool coloured_before(int cw, int it) { return cw >= 0 && (cw >> 8) < it; }

// one visit of a waiting vertex v in iteration it: its colour (returned),
// or -1 while a neighbour it has to wait for has none
__device__ __forceinline__ int jp_visit(const Store3& st, int v, const uint8_t* __restrict__ act, int* col, int* blk,
                                        int it, uint64_t sseed, int* ctr) {
  int b = blk[v];
  if (b >= 0 && !coloured_before(col[b], it)) return -1;
  uint64_t kv = vkey(sseed, (uint32_t)v);
  int4 h = st.hdr[v];
  uint64_t used[kMaxColours / 64] = {0, 0, 0, 0};
  // eight neighbours at a time: their ids, then their colours and activity
  // flags, all in flight together; taken in row order as a serial loop
  constexpr int B = 8;
  for (int j0 = 0; j0 < h.y; j0 += B) {
    int w[B], cw[B];
    uint8_t aw[B];
#pragma unroll
    for (int q = 0; q < B; ++q) w[q] = j0 + q < h.y ? st.nn[h.x + j0 + q] : -1;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      cw[q] = w[q] >= 0 ? col[w[q]] : -1;
      aw[q] = w[q] >= 0 ? act[w[q]] : 0;
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (w[q] < 0) continue;
      if (coloured_before(cw[q], it)) {
        int c = cw[q] & 0xFF;
        used[c >> 6] |= 1ull << (c & 63);
      } else if (aw[q] && vkey(sseed, (uint32_t)w[q]) > kv) {
        blk[v] = w[q];
        return -1;
      }
    }
  }
  int c = -1;
  for (int q = 0; q < kMaxColours / 64 && c < 0; ++q)
    if (~used[q]) c = q * 64 + __ffsll((long long)~used[q]) - 1;
  if (c < 0) {
    atomicOr(&ctr[K_ERR], E_COLOURS);
    c = kMaxColours - 1;
  }
  col[v] = (it << 8) | c;
  return c;
}

// a wavefront's counts: vertices coloured and colours used
__device__ __forceinline__ void jp_counts(int coloured, int ncol, int* ctr) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    coloured += __shfl_xor(coloured, d);
    ncol = max(ncol, __shfl_xor(ncol, d));
  }
  if (__lane_id() == 0 && coloured > 0) {
    atomicAdd(&ctr[K_COLOURED], coloured);
    atomicMax(&ctr[K_NCOL], ncol);
  }
}

__global__ void k_jp(Store3 st, const int* __restrict__ A, int n, const uint8_t* __restrict__ act, int* col,
                     int* blk, int it, uint64_t sseed, int* ctr) {
  int coloured = 0, ncol = 0;
  for (int i = gtid(); i < n; i += gstride()) {
    int v = A[i];
    if (col[v] >= 0) continue;
    int c = jp_visit(st, v, act, col, blk, it, sseed, ctr);
    if (c >= 0) {
      ++coloured;
      ncol = max(ncol, c + 1);
    }
  }
  jp_counts(coloured, ncol, ctr);
}

// Lists of at most kJpOne vertices (one per thread): one work-group runs the
// same iterations to completion, separated by block barriers instead of
// launches (at most n + 8 of them, as the host allows one launch each). The
// work-group's waves share one CU's vector L1, which their stores write
// through, so every iteration sees the colours of the ones before it.
constexpr int kJpOne = 1024;
constexpr int kJpOneThreads = 1024;
__global__ void __launch_bounds__(kJpOneThreads) k_jp_one(Store3 st, const int* __restrict__ A, int n,
                                                          const uint8_t* __restrict__ act, int* col, int* blk,
                                                          uint64_t sseed, int* ctr) {
  int coloured = 0, ncol = 0;
  for (int it = 0; it <= n + 8; ++it) {
    bool waiting = false;
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
      int v = A[i];
      if (col[v] >= 0) continue;
      int c = jp_visit(st, v, act, col, blk, it, sseed, ctr);
      if (c >= 0) {
        ++coloured;
        ncol = max(ncol, c + 1);
      } else {
        waiting = true;
      }
    }
    if (!__syncthreads_or(waiting)) break;
  }
  jp_counts(coloured, ncol, ctr);
}

__global__ void k_jp_strip(const int* __restrict__ A, int n, int* col) {
  for (int i = gtid(); i < n; i += gstride()) {
    int v = A[i];
    if (col[v] >= 0) col[v] &= 0xFF;
  }
}

__global__ void k_fill_int(int* p, int n, int x) {
  for (int i = gtid(); i < n; i += gstride()) p[i] = x;
}

__global__ void k_set_act(const int* __restrict__ A, int n, uint8_t* act, uint8_t x) {
  for (int i = gtid(); i < n; i += gstride()) act[A[i]] = x;
}

// the list's vertices active, with no neighbour to wait for yet
__global__ void k_jp_init(const int* __restrict__ A, int n, uint8_t* act, int* blk) {
  for (int i = gtid(); i < n; i += gstride()) {
    act[A[i]] = 1;
    blk[A[i]] = -1;
  }
}

// Class sizes: a histogram of the block's list entries in LDS, then one
// global add per colour and block.
__global__ void k_class_count(const int* __restrict__ A, int n, const int* __restrict__ col, int ncol, int* cnt) {
  __shared__ int h[kMaxColours];
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) h[c] = 0;
  __syncthreads();
  for (int i = gtid(); i < n; i += gstride()) atomicAdd(&h[col[A[i]]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x)
    if (h[c]) atomicAdd(&cnt[c], h[c]);
}

// Class lists: each block ranks its entries per colour in LDS, reserves one
// range per colour with a global add, and writes the entries there. The
// order inside a class is not fixed; the members of a class are pairwise
// non-adjacent and their decisions do not depend on it.
// the classes' first slots: the exclusive prefix sums of the class sizes
// (one work-group of kMaxColours threads)
__global__ void k_class_offsets(const int* __restrict__ cnt, int ncol, int* off) {
  __shared__ int s[kMaxColours];
  int c = (int)threadIdx.x;
  int own = c < ncol ? cnt[c] : 0;
  s[c] = own;
  __syncthreads();
  for (int d = 1; d < kMaxColours; d <<= 1) {
    int t = c >= d ? s[c - d] : 0;
    __syncthreads();
    s[c] += t;
    __syncthreads();
  }
  if (c < ncol) off[c] = s[c] - own;
}

__global__ void k_class_place(const int* __restrict__ A, int n, const int* __restrict__ col, int ncol,
                              const int* __restrict__ off, int* cur, int* out) {
  __shared__ int h[kMaxColours], base[kMaxColours];
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) h[c] = 0;
  __syncthreads();
  int i = (int)((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  int c = -1, r = 0, v = 0;
  if (i < n) {
    v = A[i];
    c = col[v];
    r = atomicAdd(&h[c], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ncol; k += blockDim.x)
    if (h[k]) base[k] = off[k] + atomicAdd(&cur[k], h[k]);
  __syncthreads();
  if (c >= 0) out[base[c] + r] = v;
}

// ---- selection of active vertices ------------------------------------------------------------

__device__ __forceinline__ bool has_candidate(const Store3& st, int v, double L_low2) {
  int4 h = st.hdr[v];
  for (int j = 0; j < h.y; ++j) {
    int u = st.nn[h.x + j];
    if (tag_ok(st, v, u) && len2(st, v, u) < L_low2) return true;
  }
  return false;
}

// mode 0: live vertices with a candidate; 1: flagged ones (flags cleared);
// 2: live interior vertices
__global__ void k_select(Store3 st, int mode, double L_low2, uint8_t* nxt, int* flag) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    bool on = st.valive[v] != 0;
    if (mode == 1) {
      on = on && nxt[v];
      nxt[v] = 0;
    }
    if (mode == 2)
      on = on && st.tag[v] == 0;
    else
      on = on && has_candidate(st, v, L_low2);
    flag[v] = on ? 1 : 0;
  }
}

__global__ void k_compact_list(const int* __restrict__ flag, const int* __restrict__ scan, int n, int* out) {
  for (int v = gtid(); v < n; v += gstride())
    if (flag[v]) out[scan[v]] = v;
}

// ---- coarsening (Sec. 2.4.1) -------------------------------------------------------------------


// One class: re-validation against the current graph, then each kept
// member's collapse, evaluated and applied (members are pairwise
// non-adjacent, so no member reads what another writes). A member runs on a
// group of kL lanes: lane j takes the row entries j, j + kL, ..., so a
// member's neighbours and elements are gathered side by side; the group
// combines its lanes' answers (any beaten, the smallest candidate pair, every
// re-pointed element valid), which are exact, so the decisions are those of a
// serial loop over the rows.
// 32 lanes: rows of 40-70 elements after refinement leave 16 lanes two to
// five elements each per candidate test (psi3 204 -> 192 ms); 8 lanes took 244.
constexpr int kL = 32;

__device__ __forceinline__ bool grp_any(bool p) {
  uint64_t b = __ballot(p);
  int base = __lane_id() & ~(kL - 1);
  constexpr uint64_t mask = kL >= kWave ? ~0ull : ((1ull << kL) - 1);
  return ((b >> base) & mask) != 0;
}

__global__ void __launch_bounds__(256) k_collapse(Store3 st, const int* __restrict__ list, int n,
                                                  const int* __restrict__ col, int c, uint64_t sseed, double L_low2,
                                                  double qmin3, uint8_t* nxt, int epoch, int* own, int* rows,
                                                  int2* rec, int* ctr) {
  // an earlier class's row commit ran out of room: the host rebuilds the
  // rows and runs this class again
  if (ctr[K_ROOM]) return;
  int j0 = __lane_id() & (kL - 1);
  int gid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kL);
  bool act = gid < n;
  int v = act ? list[gid] : 0;
  int4 h = act ? st.hdr[v] : make_int4(0, 0, 0, 0);
  uint64_t kv = vkey(sseed, (uint32_t)v);
  // one pass over the row: re-validation, and each neighbour's metric
  // length kept for the candidate search (rows of up to kC * kL entries;
  // INFINITY marks a neighbour that is no candidate)
  constexpr int kC = 2;
  int cu[kC];
  double cL[kC];
#pragma unroll
  for (int q = 0; q < kC; ++q) {
    cu[q] = -1;
    cL[q] = INFINITY;
  }
  bool b = false;
  for (int jb = 0, q = 0; jb < h.y; jb += kL, ++q) {
    int j = jb + j0;
    if (j < h.y) {
      int w = st.nn[h.x + j];
      b = b || (col[w] == c && vkey(sseed, (uint32_t)w) > kv);
#pragma unroll
      for (int r = 0; r < kC; ++r)
        if (r == q) {
          cu[r] = w;
          if (tag_ok(st, v, w)) {
            double L = len2(st, v, w);
            if (L < L_low2) cL[r] = L;
          }
        }
    }
  }
  bool cached = h.y <= kC * kL;
  bool beaten = grp_any(b);
  int ev = 0, df = 0, cm = 0;
  if (act && beaten) {
    if (j0 == 0) nxt[v] = 1;
    df = 1;
  }
  int target = -1;
  if (act && !beaten) {
    ev = 1;
    // candidates in ascending (L^2, u): each step takes the smallest pair
    // above the previous one
    double pL = -1.0;
    int pu = -1;
    for (;;) {
      double bL = 0.0;
      int bu = -1;
      if (cached) {
#pragma unroll
        for (int q = 0; q < kC; ++q) {
          double L = cL[q];
          int u = cu[q];
          if (u < 0 || !(L < L_low2)) continue;
          bool after = L > pL || (L == pL && u > pu);
          bool before = bu < 0 || L < bL || (L == bL && u < bu);
          if (after && before) {
            bL = L;
            bu = u;
          }
        }
      } else {
        for (int jb = 0; jb < h.y; jb += kL) {
          int j = jb + j0;
          if (j >= h.y) continue;
          int u = st.nn[h.x + j];
          if (!tag_ok(st, v, u)) continue;
          double L = len2(st, v, u);
          if (!(L < L_low2)) continue;
          bool after = L > pL || (L == pL && u > pu);
          bool before = bu < 0 || L < bL || (L == bL && u < bu);
          if (after && before) {
            bL = L;
            bu = u;
          }
        }
      }
#pragma unroll
      for (int d = kL / 2; d > 0; d >>= 1) {
        double oL = __shfl_xor(bL, d);
        int ou = __shfl_xor(bu, d);
        if (ou >= 0 && (bu < 0 || oL < bL || (oL == bL && ou < bu))) {
          bL = oL;
          bu = ou;
        }
      }
      if (bu < 0) break;
      bool bad = false;
      for (int kb = 0; kb < h.w; kb += kL) {
        int k = kb + j0;
        if (k >= h.w) continue;
        int4 e = st.tet[st.ne[h.z + k]];
        if (has4(e, bu)) continue;
        Geo3 g = geo(st, canon4(replace4(e, v, bu)), -1, make_double4(0, 0, 0, 0));
        if (!(vol6(g) > 0.0) || !(qual3(g) >= qmin3)) bad = true;
      }
      if (!grp_any(bad)) {
        target = bu;
        break;
      }
      pL = bL;
      pu = bu;
    }
  }
  if (target >= 0) {
    for (int kb = 0; kb < h.w; kb += kL) {
      int k = kb + j0;
      if (k >= h.w) continue;
      int t = st.ne[h.z + k];
      int4 e = st.tet[t];
      if (has4(e, target))
        st.talive[t] = 0;
      else
        st.tet[t] = canon4(replace4(e, v, target));
    }
    // the changed rows (every neighbour's, the target's among them) for the
    // row commit, stamped with the class epoch; with a row list (rows given)
    // the first stamp of a row in this class also appends it to the list
    // (one add per wavefront); and the member's target
    for (int jb = 0; jb < h.y; jb += kL) {
      int j = jb + j0;
      int w = -1;
      bool fresh = false;
      if (j < h.y) {
        w = st.nn[h.x + j];
        nxt[w] = 1;
        if (rows)
          fresh = atomicExch(&own[w], epoch) != epoch;
        else
          own[w] = epoch;
      }
      if (rows) {
        uint64_t on = __ballot(true), fb = __ballot(fresh);
        int lead = __ffsll((unsigned long long)on) - 1, at = 0;
        if (__lane_id() == lead && fb) at = atomicAdd(&ctr[K_NROWS], __popcll(fb));
        at = __shfl(at, lead);
        if (fresh) rows[at + __popcll(fb & ((1ull << __lane_id()) - 1ull))] = w;
      }
    }
    if (j0 == 0) {
      st.valive[v] = 0;
      rec[v] = make_int2(epoch, target);
    }
    cm = 1;
  }
  if (j0 != 0) ev = df = cm = 0;
  // one add per wavefront and counter
  uint64_t me = __ballot(ev), md = __ballot(df), mc = __ballot(cm);
  if (__lane_id() == 0) {
    stripe_add(ctr, K_EVAL, __popcll(me));
    stripe_add(ctr, K_DEFER, __popcll(md));
    stripe_add(ctr, K_COMMIT, __popcll(mc));
    stripe_add(ctr, K_CCOMMIT, __popcll(mc));
  }
}

// stable renumbering of live vertices and elements (a monotone map keeps the
// elements' canonical order)
__global__ void k_flags(const uint8_t* __restrict__ a, int n, int* f) {
  for (int i = gtid(); i < n; i += gstride()) f[i] = a[i] ? 1 : 0;
}

__global__ void k_compact_v(Store3 st, const int* __restrict__ vmap, double4* xyz, Met6* met, uint8_t* tag) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    if (!st.valive[v]) continue;
    int o = vmap[v];
    xyz[o] = st.xyz[v];
    met[o] = st.met[v];
    tag[o] = st.tag[v];
  }
}

__global__ void k_compact_t(Store3 st, const int* __restrict__ vmap, const int* __restrict__ tmap, int4* tet) {
  for (int t = gtid(); t < st.T; t += gstride()) {
    if (!st.talive[t]) continue;
    int4 e = st.tet[t];
    tet[tmap[t]] = make_int4(vmap[e.x], vmap[e.y], vmap[e.z], vmap[e.w]);
  }
}

__global__ void k_fill_u8(uint8_t* p, int n, uint8_t x) {
  for (int i = gtid(); i < n; i += gstride()) p[i] = x;
}

// ---- refinement (Sec. 2.4.2) ---------------------------------------------------------------------

// marks the long edges (v, w), w > v, per NN entry; counts them per vertex
__global__ void k_mark(Store3 st, double L_up2, int* mark, int* cnt, int* ctr) {
  int edges = 0;
  for (int v = gtid(); v < st.V; v += gstride()) {
    int4 h = st.hdr[v];
    int c = 0;
    for (int j = 0; j < h.y; ++j) {
      int w = st.nn[h.x + j];
      int m = 0;
      if (w > v) {
        ++edges;
        m = len2(st, v, w) > L_up2 ? 1 : 0;
      }
      mark[h.x + j] = m;
      c += m;
    }
    cnt[v] = c;
  }
  stripe_add(ctr, K_EDGES, edges);
}

// new vertex ids V0 + (rank of the edge in (min id, max id) order); the
// midpoint, the edge-mean metric and the AND of the end tags
__global__ void k_mint(Store3 st, int V0, const int* __restrict__ vscan, int* mark) {
  for (int v = gtid(); v < V0; v += gstride()) {
    int4 h = st.hdr[v];
    int k = vscan[v];
    for (int j = 0; j < h.y; ++j) {
      if (!mark[h.x + j]) {
        mark[h.x + j] = -1;
        continue;
      }
      int w = st.nn[h.x + j];
      int id = V0 + k++;
      mark[h.x + j] = id;
      double4 a = st.xyz[v], b = st.xyz[w];
      st.xyz[id] = make_double4((a.x + b.x) * 0.5, (a.y + b.y) * 0.5, (a.z + b.z) * 0.5, 0.0);
      st.met[id] = edge_met(st.met[v], st.met[w]);
      st.tag[id] = st.tag[v] & st.tag[w];
      st.valive[id] = 1;
    }
  }
}

struct Split {
  int a, b, mid;
  double L2;
};

__device__ __forceinline__ bool split_before(const Split& p, const Split& q) {
  if (p.L2 != q.L2) return p.L2 > q.L2;
  return p.a != q.a ? p.a < q.a : p.b < q.b;
}

// the midpoint id of edge (a, b) (a < b): b's position in NN(a)
__device__ __forceinline__ int mid_of(const Store3& st, const int* mark, int a, int b) {
  int4 h = st.hdr[a];
  int lo = 0, hi = h.y - 1;
  while (lo <= hi) {
    int m = (lo + hi) >> 1;
    int w = st.nn[h.x + m];
    if (w == b) return mark[h.x + m];
    if (w < b) lo = m + 1;
    else hi = m - 1;
  }
  return -1;
}

// the element's split edges in the global order
__device__ int own_splits(const Store3& st, const int* mark, int4 e, Split* s) {
  int id[4] = {e.x, e.y, e.z, e.w};
  int n = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      int a = min(id[i], id[j]), b = max(id[i], id[j]);
      int m = mid_of(st, mark, a, b);
      if (m < 0) continue;
      Split x{a, b, m, len2(st, a, b)};
      int k = n++;
      while (k > 0 && split_before(x, s[k - 1])) {
        s[k] = s[k - 1];
        --k;
      }
      s[k] = x;
    }
  return n;
}

// Bisection along the first split edge (in the global order) each piece
// holds, children depth first (the child keeping the edge's smaller id
// first). A piece needs only the splits after the one that made it, since it
// lies inside its parent. count_only: returns the number of leaves; else
// writes them (the first into slot t, the rest from base).
constexpr int kMaxLeaves = 64;
__device__ int bisect(Store3 st, const Split* s, int ns, int4 e, bool count_only, int t, int base) {
  int4 stk_t[8];
  int stk_k[8];
  int top = 0;
  stk_t[0] = e;
  stk_k[0] = 0;
  int leaves = 0;
  while (top >= 0) {
    int4 x = stk_t[top];
    int k = stk_k[top];
    --top;
    while (k < ns && !(has4(x, s[k].a) && has4(x, s[k].b))) ++k;
    if (k == ns) {
      if (!count_only) {
        int slot = leaves == 0 ? t : base + leaves - 1;
        st.tet[slot] = canon4(x);
        st.talive[slot] = 1;
      }
      ++leaves;
      continue;
    }
    int4 ca = replace4(x, s[k].b, s[k].mid);  // keeps a
    int4 cb = replace4(x, s[k].a, s[k].mid);  // keeps b
    // depth first, child a first: push b, then a
    ++top;
    stk_t[top] = cb;
    stk_k[top] = k + 1;
    ++top;
    stk_t[top] = ca;
    stk_k[top] = k + 1;
  }
  return leaves;
}

__global__ void k_split_count(Store3 st, int T0, const int* __restrict__ mark, int* tcnt, int* ctr) {
  for (int t = gtid(); t < T0; t += gstride()) {
    int c = 0;
    if (st.talive[t]) {
      Split s[6];
      int4 e = st.tet[t];
      int ns = own_splits(st, mark, e, s);
      if (ns > 0) {
        int l = bisect(st, s, ns, e, true, t, 0);
        if (l > kMaxLeaves) atomicOr(&ctr[K_ERR], E_LEAVES);
        c = l - 1;
      }
    }
    tcnt[t] = c;
  }
}

__global__ void k_split_write(Store3 st, int T0, const int* __restrict__ mark, const int* __restrict__ tscan) {
  for (int t = gtid(); t < T0; t += gstride()) {
    if (!st.talive[t]) continue;
    Split s[6];
    int4 e = st.tet[t];
    int ns = own_splits(st, mark, e, s);
    if (ns > 0) bisect(st, s, ns, e, false, t, T0 + tscan[t]);
  }
}

// ---- smoothing (Sec. 2.4.4) -------------------------------------------------------------------------

// One class of Laplacian moves with kSL lanes per member: lane j takes the
// row entries j, j + kSL, ... . The group adds the neighbour terms in row
// order by shuffles, so each sum is the serial loop's; each lane gathers an
// element's geometry once for its old and its moved quality; the patch
// minima fold as the serial loop folds them (the first element's value
// taken as it is, later ones only when smaller, so a NaN counts only as the
// first), and the moved patch's validity is a group AND.
constexpr int kSL = 8;
__global__ void __launch_bounds__(256) k_smooth(Store3 st, const int* __restrict__ list, int n, int* ctr) {
  int lane = __lane_id();
  int j0 = lane & (kSL - 1), base = lane & ~(kSL - 1);
  int64_t ng = (int64_t)gridDim.x * blockDim.x / kSL;
  int ev = 0, cm = 0;
  // every branch below is uniform over a group (its member's data)
  for (int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSL; gi < n; gi += ng) {
    int v = list[gi];
    int4 h = st.hdr[v];
    double4 pv = st.xyz[v];
    Met6 mv = st.met[v];
    Met6 G{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rx = 0.0, ry = 0.0, rz = 0.0;
    for (int jb = 0; jb < h.y; jb += kSL) {
      int j = jb + j0;
      Met6 e{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      double tx = 0.0, ty = 0.0, tz = 0.0;
      if (j < h.y) {
        int w = st.nn[h.x + j];
        e = edge_met(mv, st.met[w]);
        double4 pw = st.xyz[w];
        double dx = pw.x - pv.x, dy = pw.y - pv.y, dz = pw.z - pv.z;
        tx = (e.a00 * dx + e.a01 * dy) + e.a02 * dz;
        ty = (e.a01 * dx + e.a11 * dy) + e.a12 * dz;
        tz = (e.a02 * dx + e.a12 * dy) + e.a22 * dz;
      }
      int cnt = min(kSL, h.y - jb);
#pragma unroll
      for (int k = 0; k < kSL; ++k) {
        int src = base + k;
        double s00 = __shfl(e.a00, src), s01 = __shfl(e.a01, src), s02 = __shfl(e.a02, src);
        double s11 = __shfl(e.a11, src), s12 = __shfl(e.a12, src), s22 = __shfl(e.a22, src);
        double sx = __shfl(tx, src), sy = __shfl(ty, src), sz = __shfl(tz, src);
        if (k < cnt) {
          G.a00 = G.a00 + s00;
          G.a01 = G.a01 + s01;
          G.a02 = G.a02 + s02;
          G.a11 = G.a11 + s11;
          G.a12 = G.a12 + s12;
          G.a22 = G.a22 + s22;
          rx = rx + sx;
          ry = ry + sy;
          rz = rz + sz;
        }
      }
    }
    double det = det3(G);
    double c00 = G.a11 * G.a22 - G.a12 * G.a12, c01 = G.a02 * G.a12 - G.a01 * G.a22,
           c02 = G.a01 * G.a12 - G.a02 * G.a11, c11 = G.a00 * G.a22 - G.a02 * G.a02,
           c12 = G.a01 * G.a02 - G.a00 * G.a12, c22 = G.a00 * G.a11 - G.a01 * G.a01;
    double4 p = make_double4(pv.x + ((c00 * rx + c01 * ry) + c02 * rz) / det,
                             pv.y + ((c01 * rx + c11 * ry) + c12 * rz) / det,
                             pv.z + ((c02 * rx + c12 * ry) + c22 * rz) / det, 0.0);
    if (j0 == 0) ++ev;
    bool vn = true;
    double mo = INFINITY, mn = INFINITY;
    for (int kb = 0; kb < h.w; kb += kSL) {
      int k = kb + j0;
      if (k >= h.w) continue;
      int4 t = st.tet[st.ne[h.z + k]];
      Geo3 go = geo(st, t, v, pv);
      Geo3 gn = go;
      int id[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (id[q] == v) gn.p[q] = p;
      if (!(vol6(gn) > 0.0)) vn = false;
      double qo = qual3(go), qn = qual3(gn);
      if (k == 0 || qo < mo) mo = qo;
      if (k == 0 || qn < mn) mn = qn;
    }
    uint64_t gm = ((1ull << kSL) - 1ull) << base;
    vn = (__ballot(!vn) & gm) == 0;
    double oldmin = __shfl(mo, base), newmin = __shfl(mn, base);
#pragma unroll
    for (int k = 1; k < kSL; ++k) {
      double a = __shfl(mo, base + k), b = __shfl(mn, base + k);
      if (a < oldmin) oldmin = a;
      if (b < newmin) newmin = b;
    }
    if (!(vn && newmin >= oldmin)) continue;
    if (j0 == 0) {
      st.xyz[v] = p;
      ++cm;
    }
  }
  stripe_add(ctr, K_EVAL, ev);
  stripe_add(ctr, K_COMMIT, cm);
}

// ---- quality ----------------------------------------------------------------------------------------

constexpr int QB = 256;
__global__ void k_quality(Store3 st, double* psum, double* pmin) {
  __shared__ double ls[QB], lm[QB];
  double s = 0.0, mn = INFINITY;
  for (int t = gtid(); t < st.T; t += gstride()) {
    if (!st.talive[t]) continue;
    double q = qual(geo(st, st.tet[t], -1, make_double4(0, 0, 0, 0)));
    s = s + q;
    mn = fmin(mn, q);
  }
  ls[threadIdx.x] = s;
  lm[threadIdx.x] = mn;
  __syncthreads();
  for (int k = QB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + k];
      lm[threadIdx.x] = fmin(lm[threadIdx.x], lm[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = ls[0];
    pmin[blockIdx.x] = lm[0];
  }
}

__global__ void k_quality_final(const double* __restrict__ psum, const double* __restrict__ pmin, int n,
                                double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0, mn = INFINITY;
  for (int i = 0; i < n; ++i) {
    s = s + psum[i];
    mn = fmin(mn, pmin[i]);
  }
  out[0] = s;
  out[1] = mn;
}

__global__ void k_export(Store3 st, double* xyz, int* tet, double* met) {
  for (int v = gtid(); v < st.V; v += gstride()) {
    double4 p = st.xyz[v];
    if (xyz) {
      xyz[3 * v] = p.x;
      xyz[3 * v + 1] = p.y;
      xyz[3 * v + 2] = p.z;
    }
    if (met) {
      Met6 g = st.met[v];
      double* q = met + 6 * v;
      q[0] = g.a00;
      q[1] = g.a01;
      q[2] = g.a02;
      q[3] = g.a11;
      q[4] = g.a12;
      q[5] = g.a22;
    }
  }
  if (tet)
    for (int t = gtid(); t < st.T; t += gstride()) {
      int4 e = st.tet[t];
      tet[4 * t] = e.x;
      tet[4 * t + 1] = e.y;
      tet[4 * t + 2] = e.z;
      tet[4 * t + 3] = e.w;
    }
}

inline int grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kB - 1) / kB, 16384)); }

}  // namespace pm3

using namespace pm3;

// ---- host side ------------------------------------------------------------------------------------------

struct pm3_mesh {
  hipStream_t s = nullptr;
  uint64_t seed = 0;
  std::string err;
  Store3 st;
  int Vcap = 0, Tcap = 0;
  int64_t nncap = 0, necap = 0;
  int* ctr = nullptr;   // device counters
  int* hctr = nullptr;  // pinned mirror
  // scratch
  int *cnt = nullptr, *off = nullptr, *cur = nullptr, *flag = nullptr, *scan = nullptr, *partial = nullptr;
  int *A = nullptr, *cls = nullptr, *col = nullptr, *blk = nullptr, *mark = nullptr,
      *tcnt = nullptr, *tscan = nullptr, *ccount = nullptr, *coff = nullptr;
  uint8_t *act = nullptr, *nxt = nullptr;
  double* qbuf = nullptr;
  int scap = 0, tscap = 0, pcap = 0;
  int64_t mcap = 0;
  // row commit: per-vertex class stamps and member records, the stripes'
  // bump pointers, the epoch of the last class, and the pool range above
  // the last full build that the stripes share
  int* own = nullptr;
  int* rows = nullptr;  // the rows stamped by the class in progress, each once
  int2* rec = nullptr;
  int* tops = nullptr;
  int epoch = 0;
  int64_t top_base = 0, top_per = 0;
  double headroom = 3.0;  // pool_headroom of the creation options
};

namespace {

thread_local std::string g3_create_err;

pm_status fail3(pm3_mesh* m, pm_status st, const std::string& msg) {
  if (m) m->err = msg;
  return st;
}

#define H3(call)                                                                    \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail3(m, PM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define T3(call)                     \
  do {                               \
    pm_status s_ = (call);           \
    if (s_ != PM_OK) return s_;      \
  } while (0)

// Device blocks come from the library's stream-ordered block cache: a block
// freed on the handle's stream is reused only by later work on that stream,
// so growing an array needs no wait before the old block is released.
template <class T>
pm_status dgrow(pm3_mesh* m, T** p, int64_t old_n, int64_t n, bool keep) {
  if (n <= old_n && *p) return PM_OK;
  T* q = nullptr;
  if (pm::block_alloc(m->s, (void**)&q, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail3(m, PM_E_NOMEM, "device allocation failed");
  }
  if (keep && *p && old_n > 0) H3(hipMemcpyAsync(q, *p, sizeof(T) * (size_t)old_n, hipMemcpyDeviceToDevice, m->s));
  if (*p) pm::block_free(*p);
  *p = q;
  return PM_OK;
}

template <class T>
void dfree3(T*& p) {
  if (p) pm::block_free(p);
  p = nullptr;
}

pm_status read_ctr(pm3_mesh* m) {
  H3(hipMemcpyAsync(m->hctr, m->ctr, sizeof(int) * K_COUNT, hipMemcpyDeviceToHost, m->s));
  H3(hipStreamSynchronize(m->s));
  return PM_OK;
}

pm_status zero_ctr(pm3_mesh* m) {
  k_fill_int<<<1, kB, 0, m->s>>>(m->ctr, K_COUNT, 0);
  H3(hipGetLastError());
  return PM_OK;
}

// capacity for V vertices and T elements (kept contents)
pm_status reserve(pm3_mesh* m, int V, int T) {
  Store3& st = m->st;
  if (V > m->Vcap) {
    int nc = std::max(V, m->Vcap + m->Vcap / 2);
    T3(dgrow(m, &st.xyz, m->Vcap, nc, true));
    T3(dgrow(m, &st.met, m->Vcap, nc, true));
    T3(dgrow(m, &st.tag, m->Vcap, nc, true));
    T3(dgrow(m, &st.valive, m->Vcap, nc, true));
    // growth happens in the middle of a refinement pass, whose rows, vertex
    // scan and element scan must survive it: every array keeps its contents
    T3(dgrow(m, &st.hdr, m->Vcap, nc, true));
    T3(dgrow(m, &m->cnt, m->Vcap + 1, nc + 1, true));
    T3(dgrow(m, &m->off, m->Vcap + 1, nc + 1, true));
    T3(dgrow(m, &m->cur, m->Vcap + 1, nc + 1, true));
    T3(dgrow(m, &m->flag, m->Vcap + 1, nc + 1, true));
    T3(dgrow(m, &m->scan, m->Vcap + 1, nc + 1, true));
    T3(dgrow(m, &m->A, m->Vcap, nc, true));
    T3(dgrow(m, &m->cls, m->Vcap, nc, true));
    T3(dgrow(m, &m->col, m->Vcap, nc, true));
    T3(dgrow(m, &m->blk, m->Vcap, nc, true));
    T3(dgrow(m, &m->act, m->Vcap, nc, true));
    T3(dgrow(m, &m->nxt, m->Vcap, nc, true));
    T3(dgrow(m, &st.cap, m->Vcap, nc, true));
    T3(dgrow(m, &m->own, m->Vcap, nc, true));
    T3(dgrow(m, &m->rec, m->Vcap, nc, true));
    T3(dgrow(m, &m->rows, m->Vcap, nc, false));
    // new vertex slots carry no class stamp or record
    k_fill_int<<<grid(nc - m->Vcap), kB, 0, m->s>>>(m->own + m->Vcap, nc - m->Vcap, -1);
    k_fill_int<<<grid(2 * (int64_t)(nc - m->Vcap)), kB, 0, m->s>>>((int*)(m->rec + m->Vcap), 2 * (nc - m->Vcap), -1);
    H3(hipGetLastError());
    m->Vcap = nc;
  }
  if (T > m->Tcap) {
    int nc = std::max(T, m->Tcap + m->Tcap / 2);
    T3(dgrow(m, &st.tet, m->Tcap, nc, true));
    T3(dgrow(m, &st.talive, m->Tcap, nc, true));
    T3(dgrow(m, &m->tcnt, m->Tcap + 1, nc + 1, true));
    T3(dgrow(m, &m->tscan, m->Tcap + 1, nc + 1, true));
    m->Tcap = nc;
  }
  int need = pm::scan_partials_needed(std::max(m->Vcap, m->Tcap) + 1);
  if (need > m->pcap) {
    T3(dgrow(m, &m->partial, m->pcap, need, false));
    m->pcap = need;
  }
  return PM_OK;
}

// exclusive scan of n ints into out; returns the total
// the scan's total, with every counter (the host copy is then as current as
// after read_ctr)
pm_status scan_total(pm3_mesh* m, const int* in, int* out, int n, int* total) {
  pm::scan_excl(in, out, n, m->ctr + K_TOTAL, m->partial, m->s);
  H3(hipGetLastError());
  H3(hipMemcpyAsync(m->hctr, m->ctr, sizeof(int) * K_COUNT, hipMemcpyDeviceToHost, m->s));
  H3(hipStreamSynchronize(m->s));
  *total = m->hctr[K_TOTAL];
  return PM_OK;
}

// every row from the live elements; sorted rows, or loose ones inside a
// coarsening phase
// Every row from the element list, packed and sorted; the pools keep the
// headroom times the packed size free above it for the row commits of a
// coarsening phase (a row that outgrows its slot moves, with twice the room,
// and its old slot stays unused until the next full build), split into the
// stripes' ranges. Clears the room counters.
pm_status build_rows(pm3_mesh* m) {
  Store3& st = m->st;
  int V = st.V;
  k_fill_int<<<grid(V + 1), kB, 0, m->s>>>(m->cnt, V + 1, 0);
  k_ne_count<<<grid(st.T), kB, 0, m->s>>>(st, m->cnt);
  int total = 0;
  T3(scan_total(m, m->cnt, m->off, V, &total));
  int64_t want = total + (int64_t)(m->headroom * (double)total) + kTopStripes * 64;
  if (want > m->necap) {
    int64_t nc = std::max<int64_t>(want, m->necap + m->necap / 2);
    if (3 * nc > INT32_MAX) return fail3(m, PM_E_NOMEM, "adjacency pool beyond 2^31 entries");
    T3(dgrow(m, &st.ne, m->necap, nc, false));
    T3(dgrow(m, &st.nn, m->nncap, 3 * nc, false));
    m->necap = nc;
    m->nncap = 3 * nc;
  }
  // refinement marks NN entries of packed rows only
  if (3 * (int64_t)total + 3 > m->mcap) {
    int64_t nc = std::max<int64_t>(3 * (int64_t)total + 3, m->mcap + m->mcap / 2);
    T3(dgrow(m, &m->mark, m->mcap, nc, false));
    m->mcap = nc;
  }
  if (!m->tops) T3(dgrow(m, &m->tops, 0, kTopStripes * kTopStride, false));
  k_fill_int<<<grid(V + 1), kB, 0, m->s>>>(m->cur, V + 1, 0);
  k_ne_fill<<<grid(st.T), kB, 0, m->s>>>(st, m->off, m->cur);
  k_rows_finish<<<grid((int64_t)V * kWave), kB, 0, m->s>>>(st, m->off, m->cnt);
  m->top_base = total;
  m->top_per = (m->necap - total) / kTopStripes;
  k_tops_init<<<1, kTopStripes, 0, m->s>>>(m->tops, m->top_base, m->top_per);
  k_fill_int<<<1, kB, 0, m->s>>>(m->ctr + K_ROOM, 2, 0);
  H3(hipGetLastError());
  return PM_OK;
}

// list of the vertices selected by mode (ascending); returns its length
pm_status select_list(pm3_mesh* m, int mode, double L_low2, int* n) {
  Store3& st = m->st;
  k_select<<<grid(st.V), kB, 0, m->s>>>(st, mode, L_low2, m->nxt, m->flag);
  int total = 0;
  T3(scan_total(m, m->flag, m->scan, st.V, &total));
  k_compact_list<<<grid(st.V), kB, 0, m->s>>>(m->flag, m->scan, st.V, m->A);
  H3(hipGetLastError());
  *n = total;
  return PM_OK;
}

// Jones-Plassmann colouring of the list A[0, n); col holds the colours
// (-1 elsewhere); returns the colour count
pm_status colour_list(pm3_mesh* m, int n, uint32_t ctx, int* ncol) {
  Store3& st = m->st;
  uint64_t sseed = stream_seed(m->seed, ctx);
  k_fill_int<<<grid(st.V), kB, 0, m->s>>>(m->col, st.V, -1);
  k_fill_u8<<<grid(st.V), kB, 0, m->s>>>(m->act, st.V, 0);
  k_jp_init<<<grid(n), kB, 0, m->s>>>(m->A, n, m->act, m->blk);
  T3(zero_ctr(m));
  int done = 0;
  if (n > 0 && n <= kJpOne) {
    k_jp_one<<<1, kJpOneThreads, 0, m->s>>>(st, m->A, n, m->act, m->col, m->blk, sseed, m->ctr);
    H3(hipGetLastError());
    T3(read_ctr(m));
    if (m->hctr[K_ERR] & E_COLOURS) return fail3(m, PM_E_DEVICE, "more than 256 colours");
    if (m->hctr[K_COLOURED] != n) return fail3(m, PM_E_DEVICE, "colouring made no progress");
    done = n;
  }
  // iterations in batches of kJpBatch between read-backs (an iteration after
  // the last vertex has its colour changes nothing)
  constexpr int kJpBatch = 4;
  for (int it = 0; done < n;) {
    // the stamp keeps 23 bits of the iteration
    if (it > n + 8 || it + kJpBatch >= (1 << 23)) return fail3(m, PM_E_DEVICE, "colouring made no progress");
    for (int b = 0; b < kJpBatch; ++b, ++it)
      k_jp<<<grid(n), kB, 0, m->s>>>(st, m->A, n, m->act, m->col, m->blk, it, sseed, m->ctr);
    H3(hipGetLastError());
    T3(read_ctr(m));
    if (m->hctr[K_ERR] & E_COLOURS) return fail3(m, PM_E_DEVICE, "more than 256 colours");
    done = m->hctr[K_COLOURED];
  }
  if (n > 0) k_jp_strip<<<grid(n), kB, 0, m->s>>>(m->A, n, m->col);
  H3(hipGetLastError());
  *ncol = n > 0 ? m->hctr[K_NCOL] : 0;
  return PM_OK;
}

// class lists of the coloured list: m->cls, offsets and sizes on the host
pm_status class_lists(pm3_mesh* m, int n, int ncol, std::vector<int>& off, std::vector<int>& size) {
  if (!m->ccount) {
    T3(dgrow(m, &m->ccount, 0, 2 * kMaxColours, false));
    T3(dgrow(m, &m->coff, 0, kMaxColours, false));
  }
  // sizes, offsets and placement on the device; one read-back of the sizes
  // (the host computes the same offsets from them)
  k_fill_int<<<1, 2 * kMaxColours, 0, m->s>>>(m->ccount, 2 * kMaxColours, 0);
  k_class_count<<<grid(n), kB, 0, m->s>>>(m->A, n, m->col, ncol, m->ccount);
  k_class_offsets<<<1, kMaxColours, 0, m->s>>>(m->ccount, ncol, m->coff);
  k_class_place<<<std::max(1, (n + kB - 1) / kB), kB, 0, m->s>>>(m->A, n, m->col, ncol, m->coff,
                                                                   m->ccount + kMaxColours, m->cls);
  H3(hipGetLastError());
  H3(hipMemcpyAsync(m->hctr + K_COUNT, m->ccount, sizeof(int) * ncol, hipMemcpyDeviceToHost, m->s));
  H3(hipStreamSynchronize(m->s));
  size.assign(ncol, 0);
  off.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) {
    size[c] = m->hctr[K_COUNT + c];
    off[c + 1] = off[c] + size[c];
  }
  return PM_OK;
}

pm_status compact(pm3_mesh* m) {
  Store3& st = m->st;
  int V = st.V, T = st.T;
  k_flags<<<grid(V), kB, 0, m->s>>>(st.valive, V, m->flag);
  int nv = 0, nt = 0;
  T3(scan_total(m, m->flag, m->scan, V, &nv));
  k_flags<<<grid(T), kB, 0, m->s>>>(st.talive, T, m->tcnt);
  T3(scan_total(m, m->tcnt, m->tscan, T, &nt));
  double4* xyz = nullptr;
  Met6* met = nullptr;
  uint8_t* tag = nullptr;
  int4* tet = nullptr;
  T3(dgrow(m, &xyz, 0, m->Vcap, false));
  T3(dgrow(m, &met, 0, m->Vcap, false));
  T3(dgrow(m, &tag, 0, m->Vcap, false));
  T3(dgrow(m, &tet, 0, m->Tcap, false));
  k_compact_v<<<grid(V), kB, 0, m->s>>>(st, m->scan, xyz, met, tag);
  k_compact_t<<<grid(T), kB, 0, m->s>>>(st, m->scan, m->tscan, tet);
  H3(hipGetLastError());
  dfree3(st.xyz);
  dfree3(st.met);
  dfree3(st.tag);
  dfree3(st.tet);
  st.xyz = xyz;
  st.met = met;
  st.tag = tag;
  st.tet = tet;
  st.V = nv;
  st.T = nt;
  k_fill_u8<<<grid(nv), kB, 0, m->s>>>(st.valive, nv, 1);
  k_fill_u8<<<grid(nt), kB, 0, m->s>>>(st.talive, nt, 1);
  k_fill_u8<<<grid(nv), kB, 0, m->s>>>(m->nxt, nv, 0);
  H3(hipGetLastError());
  return build_rows(m);
}

void put_stats(pm_stats* out, const int64_t* v) {
  if (!out) return;
  for (int i = 0; i < 16; ++i) out->v[i] = v[i];
}

}  // namespace

extern "C" {

pm_status pm3_mesh_create(const pm3_mesh_desc* d, const pm_options* o, void* stream, pm3_mesh** out) {
  if (!out) return PM_E_ARG;
  *out = nullptr;
  if (!d || !d->xyz || !d->tet || !d->metric) return PM_E_ARG;
  if (d->V < 4 || d->T < 1 || d->V > (1ll << 29) || d->T > (1ll << 29)) return PM_E_ARG;
  if (d->mem_kind != PM_MEM_HOST && d->mem_kind != PM_MEM_DEVICE) return PM_E_ARG;
  pm_options def;
  if (!o) {
    pm_default_options(&def);
    o = &def;
  }
  pm3_mesh* m = new (std::nothrow) pm3_mesh();
  if (!m) return PM_E_NOMEM;
  m->s = (hipStream_t)stream;
  m->seed = o->seed;
  if (!(o->pool_headroom == 0.0 || (o->pool_headroom >= 1.0 && o->pool_headroom <= 64.0))) {
    delete m;
    g3_create_err = "pool_headroom: 0 (the default) or within [1, 64]";
    return PM_E_ARG;
  }
  m->headroom = o->pool_headroom > 0.0 ? o->pool_headroom : 3.0;
  auto bail = [&](pm_status s) {
    g3_create_err = m->err.empty() ? std::string("pm3_mesh_create failed") : m->err;
    pm3_mesh_destroy(m);
    return s;
  };
  int V = (int)d->V, T = (int)d->T;
  if (pm::block_alloc(m->s, (void**)&m->ctr, sizeof(int) * K_COUNT) != hipSuccess ||
      hipHostMalloc((void**)&m->hctr, sizeof(int) * (K_COUNT + 2 * kMaxColours), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return bail(PM_E_NOMEM);
  }
  if (reserve(m, V, T) != PM_OK) return bail(PM_E_NOMEM);
  Store3& st = m->st;
  st.V = V;
  st.T = T;
  double *xyz = nullptr, *met = nullptr;
  int* tet = nullptr;
  uint8_t* tags = nullptr;
  hipMemcpyKind kind = d->mem_kind == PM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if (dgrow(m, &xyz, 0, 3 * (int64_t)V, false) != PM_OK || dgrow(m, &met, 0, 6 * (int64_t)V, false) != PM_OK ||
      dgrow(m, &tet, 0, 4 * (int64_t)T, false) != PM_OK)
    return bail(PM_E_NOMEM);
  bool ok = hipMemcpyAsync(xyz, d->xyz, sizeof(double) * 3 * V, kind, m->s) == hipSuccess &&
            hipMemcpyAsync(met, d->metric, sizeof(double) * 6 * V, kind, m->s) == hipSuccess &&
            hipMemcpyAsync(tet, d->tet, sizeof(int) * 4 * T, kind, m->s) == hipSuccess;
  if (ok && d->tags) ok = hipMemcpyAsync(st.tag, d->tags, (size_t)V, kind, m->s) == hipSuccess;
  if (!ok) return bail(PM_E_DEVICE);
  if (zero_ctr(m) != PM_OK) return bail(PM_E_DEVICE);
  k_in<<<grid(std::max(V, T)), kB, 0, m->s>>>(xyz, tet, met, st, m->ctr);
  if (!d->tags) k_tags<<<grid(V), kB, 0, m->s>>>(st);
  k_orient<<<grid(T), kB, 0, m->s>>>(st, m->ctr);
  if (read_ctr(m) != PM_OK) return bail(PM_E_DEVICE);
  dfree3(xyz);
  dfree3(met);
  dfree3(tet);
  if (m->hctr[K_ERR]) {
    m->err = "invalid mesh: ids, orientation or metric";
    return bail(PM_E_MESH);
  }
  k_fill_u8<<<grid(V), kB, 0, m->s>>>(m->nxt, V, 0);
  if (build_rows(m) != PM_OK) return bail(PM_E_DEVICE);
  if (hipStreamSynchronize(m->s) != hipSuccess) return bail(PM_E_DEVICE);
  *out = m;
  return PM_OK;
}

pm_status pm3_mesh_destroy(pm3_mesh* m) {
  if (!m) return PM_OK;
  (void)hipStreamSynchronize(m->s);
  Store3& st = m->st;
  dfree3(st.xyz);
  dfree3(st.met);
  dfree3(st.tag);
  dfree3(st.valive);
  dfree3(st.tet);
  dfree3(st.talive);
  dfree3(st.hdr);
  dfree3(st.nn);
  dfree3(st.ne);
  for (int** p : {&m->cnt, &m->off, &m->cur, &m->flag, &m->scan, &m->partial, &m->A, &m->cls, &m->col,
                  &m->blk, &m->mark, &m->tcnt, &m->tscan, &m->ccount, &m->coff, &m->ctr})
    dfree3(*p);
  dfree3(m->act);
  dfree3(m->nxt);
  dfree3(m->qbuf);
  dfree3(st.cap);
  dfree3(m->own);
  dfree3(m->rows);
  dfree3(m->rec);
  dfree3(m->tops);
  if (m->hctr) (void)hipHostFree(m->hctr);
  delete m;
  return PM_OK;
}

pm_status pm3_mesh_sizes(const pm3_mesh* m, int64_t* V, int64_t* T) {
  if (!m) return PM_E_ARG;
  if (V) *V = m->st.V;
  if (T) *T = m->st.T;
  return PM_OK;
}

pm_status pm3_mesh_export(pm3_mesh* m, double* xyz, int32_t* tet, double* metric, uint8_t* tags, uint8_t* valive,
                          uint8_t* talive, int32_t mem_kind) {
  if (!m) return PM_E_ARG;
  if (mem_kind != PM_MEM_HOST && mem_kind != PM_MEM_DEVICE) return fail3(m, PM_E_ARG, "bad mem_kind");
  Store3& st = m->st;
  int V = st.V, T = st.T;
  bool host = mem_kind == PM_MEM_HOST;
  double *dx = nullptr, *dm = nullptr;
  int* dt = nullptr;
  if (host) {
    if (xyz) T3(dgrow(m, &dx, 0, 3 * (int64_t)V, false));
    if (metric) T3(dgrow(m, &dm, 0, 6 * (int64_t)V, false));
    if (tet) T3(dgrow(m, &dt, 0, 4 * (int64_t)T, false));
  } else {
    dx = xyz;
    dm = metric;
    dt = tet;
  }
  k_export<<<grid(std::max(V, T)), kB, 0, m->s>>>(st, dx, dt, dm);
  H3(hipGetLastError());
  hipMemcpyKind k = host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (host) {
    if (xyz) H3(hipMemcpyAsync(xyz, dx, sizeof(double) * 3 * V, k, m->s));
    if (metric) H3(hipMemcpyAsync(metric, dm, sizeof(double) * 6 * V, k, m->s));
    if (tet) H3(hipMemcpyAsync(tet, dt, sizeof(int) * 4 * T, k, m->s));
  }
  if (tags) H3(hipMemcpyAsync(tags, st.tag, (size_t)V, k, m->s));
  if (valive) H3(hipMemcpyAsync(valive, st.valive, (size_t)V, k, m->s));
  if (talive) H3(hipMemcpyAsync(talive, st.talive, (size_t)T, k, m->s));
  H3(hipStreamSynchronize(m->s));
  if (host) {  // staging blocks (for device exports they are the caller's arrays)
    dfree3(dx);
    dfree3(dm);
    dfree3(dt);
  }
  return PM_OK;
}

pm_status pm3_mesh_rows(pm3_mesh* m, int64_t* nn_total, int64_t* ne_total, int64_t* nn_off, int32_t* nn,
                        int64_t* ne_off, int32_t* ne) {
  if (!m) return PM_E_ARG;
  Store3& st = m->st;
  int V = st.V;
  std::vector<int4> hdr(V);
  H3(hipMemcpyAsync(hdr.data(), st.hdr, sizeof(int4) * V, hipMemcpyDeviceToHost, m->s));
  H3(hipStreamSynchronize(m->s));
  int64_t a = 0, b = 0;
  for (int v = 0; v < V; ++v) {
    a += hdr[v].y;
    b += hdr[v].w;
  }
  if (nn_total) *nn_total = a;
  if (ne_total) *ne_total = b;
  if (!nn_off || !nn || !ne_off || !ne) return PM_OK;
  std::vector<int> hnn(m->nncap > 0 ? (size_t)std::min<int64_t>(m->nncap, 3 * b + 3) : 1),
      hne((size_t)std::max<int64_t>(b, 1));
  if (b > 0) {
    H3(hipMemcpyAsync(hnn.data(), st.nn, sizeof(int) * (size_t)(3 * b), hipMemcpyDeviceToHost, m->s));
    H3(hipMemcpyAsync(hne.data(), st.ne, sizeof(int) * (size_t)b, hipMemcpyDeviceToHost, m->s));
    H3(hipStreamSynchronize(m->s));
  }
  int64_t pa = 0, pb = 0;
  for (int v = 0; v < V; ++v) {
    nn_off[v] = pa;
    ne_off[v] = pb;
    for (int j = 0; j < hdr[v].y; ++j) nn[pa++] = hnn[hdr[v].x + j];
    for (int j = 0; j < hdr[v].w; ++j) ne[pb++] = hne[hdr[v].z + j];
  }
  nn_off[V] = pa;
  ne_off[V] = pb;
  return PM_OK;
}

pm_status pm3_colour(pm3_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out, int32_t* ncolours) {
  if (!m) return PM_E_ARG;
  Store3& st = m->st;
  int n = 0;
  if (active) {
    std::vector<int> f(st.V);
    std::vector<uint8_t> va(st.V);
    H3(hipMemcpyAsync(va.data(), st.valive, (size_t)st.V, hipMemcpyDeviceToHost, m->s));
    H3(hipStreamSynchronize(m->s));
    for (int v = 0; v < st.V; ++v) f[v] = (active[v] && va[v]) ? 1 : 0;
    H3(hipMemcpyAsync(m->flag, f.data(), sizeof(int) * st.V, hipMemcpyHostToDevice, m->s));
    int total = 0;
    T3(scan_total(m, m->flag, m->scan, st.V, &total));
    k_compact_list<<<grid(st.V), kB, 0, m->s>>>(m->flag, m->scan, st.V, m->A);
    n = total;
  } else {
    k_flags<<<grid(st.V), kB, 0, m->s>>>(st.valive, st.V, m->flag);
    int total = 0;
    T3(scan_total(m, m->flag, m->scan, st.V, &total));
    k_compact_list<<<grid(st.V), kB, 0, m->s>>>(m->flag, m->scan, st.V, m->A);
    n = total;
  }
  int ncol = 0;
  T3(colour_list(m, n, ctx, &ncol));
  if (ncolours) *ncolours = ncol;
  if (colour_out) {
    H3(hipMemcpyAsync(colour_out, m->col, sizeof(int) * st.V, hipMemcpyDeviceToHost, m->s));
    H3(hipStreamSynchronize(m->s));
  }
  return PM_OK;
}

pm_status pm3_coarsen(pm3_mesh* m, const pm_options* o, pm_stats* out) {
  if (!m || !o) return PM_E_ARG;
  if (!(o->L_low2 > 0.0) || !(o->q_min >= 0.0) || o->coarsen_rounds < 0) return fail3(m, PM_E_ARG, "bad options");
  Store3& st = m->st;
  int64_t sv[16] = {};
  double qmin3 = (o->q_min * o->q_min) * o->q_min;
  int n = 0;
  T3(select_list(m, 0, o->L_low2, &n));
  k_fill_u8<<<grid(st.V), kB, 0, m->s>>>(m->nxt, st.V, 0);
  int r = 0;
  std::vector<int> off, size;
  while (n > 0 && r < o->coarsen_rounds) {
    uint32_t ctx = make_ctx(o->sweep, PH3_COARSEN, r);
    uint64_t sseed = stream_seed(m->seed, ctx);
    int ncol = 0;
    T3(colour_list(m, n, ctx, &ncol));
    sv[PM_S_COLOURED] += n;
    sv[PM_S_COLOURS] += ncol;
    T3(class_lists(m, n, ncol, off, size));
    // the colouring zeroed the counters: the round's stats accumulate on the
    // device and come back with the next list's length. Each class: the
    // collapses, then the commit of the rows they changed. A commit that runs
    // out of room makes the round's later classes stand down; the host then
    // rebuilds every row from the elements and runs those classes again.
    std::vector<int> class_epoch(ncol, -1);
    int c0 = 0;
    for (;;) {
      for (int c = c0; c < ncol; ++c) {
        if (size[c] == 0) continue;
        int ep = ++m->epoch;
        class_epoch[c] = ep;
        k_class_start<<<1, kWave, 0, m->s>>>(m->ctr);
        // the row list while the class can stamp at most about an eighth of
        // the rows (a wavefront for about every row a member's neighbours
        // give, at most one grid's worth), else vertex order
        int64_t reach = (int64_t)size[c] * 16;
        bool listed = reach * 8 <= st.V;
        int nb = (int)(((int64_t)size[c] * kL + kB - 1) / kB);
        k_collapse<<<nb, kB, 0, m->s>>>(st, m->cls + off[c], size[c], m->col, c, sseed, o->L_low2, qmin3,
                                         m->nxt, ep, m->own, listed ? m->rows : nullptr, m->rec, m->ctr);
        if (listed)
          k_commit3_list<<<grid(reach * kWave), kB, 0, m->s>>>(st, ep, m->rows, m->rec, m->tops, m->top_base,
                                                              m->top_per, m->ctr);
        else
          k_commit3<<<grid((int64_t)st.V * kWave), kB, 0, m->s>>>(st, ep, m->own, m->rec, m->tops, m->top_base,
                                                                   m->top_per, m->ctr);
        H3(hipGetLastError());
      }
      T3(read_ctr(m));
      if (!m->hctr[K_ROOM]) break;
      int failed = -1;
      for (int c = 0; c < ncol; ++c)
        if (class_epoch[c] == m->hctr[K_ROOMEP]) failed = c;
      if (failed < c0) return fail3(m, PM_E_DEVICE, "row commit: room counter names no class of this round");
      T3(build_rows(m));
      ++sv[13];
      c0 = failed + 1;
    }
    T3(select_list(m, 1, o->L_low2, &n));  // its read-back returns the round's counters too
    sv[PM_S_EVALUATED] += m->hctr[K_EVAL];
    sv[PM_S_DEFERRED] += m->hctr[K_DEFER];
    sv[PM_S_COMMITTED] += m->hctr[K_COMMIT];
    ++r;
  }
  sv[PM_S_ROUNDS] = r;
  sv[PM_S_CONVERGED] = n == 0 ? 1 : 0;
  T3(compact(m));
  H3(hipStreamSynchronize(m->s));
  put_stats(out, sv);
  return n == 0 ? PM_OK : PM_W_NOT_CONVERGED;
}

pm_status pm3_refine(pm3_mesh* m, const pm_options* o, pm_stats* out) {
  if (!m || !o) return PM_E_ARG;
  if (!(o->L_up2 > 0.0) || o->refine_passes < 0) return fail3(m, PM_E_ARG, "bad options");
  Store3& st = m->st;
  int64_t sv[16] = {};
  int p = 0;
  bool done = false;
  for (; p < o->refine_passes; ++p) {
    int V0 = st.V, T0 = st.T;
    T3(zero_ctr(m));
    k_mark<<<grid(V0), kB, 0, m->s>>>(st, o->L_up2, m->mark, m->cnt, m->ctr);
    int nv = 0;
    T3(scan_total(m, m->cnt, m->scan, V0, &nv));
    sv[PM_S_EDGES] += m->hctr[K_EDGES];
    if (nv == 0) {
      done = true;
      break;
    }
    T3(reserve(m, V0 + nv, T0));
    k_mint<<<grid(V0), kB, 0, m->s>>>(st, V0, m->scan, m->mark);
    st.V = V0 + nv;
    k_split_count<<<grid(T0), kB, 0, m->s>>>(st, T0, m->mark, m->tcnt, m->ctr);
    int nt = 0;
    T3(scan_total(m, m->tcnt, m->tscan, T0, &nt));
    if (m->hctr[K_ERR] & E_LEAVES) return fail3(m, PM_E_DEVICE, "an element split into too many pieces");
    T3(reserve(m, V0 + nv, T0 + nt));
    k_split_write<<<grid(T0), kB, 0, m->s>>>(st, T0, m->mark, m->tscan);
    st.T = T0 + nt;
    H3(hipGetLastError());
    sv[PM_S_NEWV] += nv;
    sv[PM_S_NEWT] += nt;
    sv[PM_S_COMMITTED] += nv;
    T3(build_rows(m));
  }
  H3(hipStreamSynchronize(m->s));
  sv[PM_S_ROUNDS] = p;
  sv[PM_S_CONVERGED] = done ? 1 : 0;
  put_stats(out, sv);
  return done ? PM_OK : PM_W_NOT_CONVERGED;
}

pm_status pm3_smooth(pm3_mesh* m, const pm_options* o, pm_stats* out) {
  if (!m || !o) return PM_E_ARG;
  if (o->smooth_sweeps < 0) return fail3(m, PM_E_ARG, "bad options");
  Store3& st = m->st;
  int64_t sv[16] = {};
  int n = 0;
  T3(select_list(m, 2, 0.0, &n));
  int ncol = 0;
  T3(colour_list(m, n, make_ctx(o->sweep, PH3_SMOOTH, 0), &ncol));
  sv[PM_S_COLOURED] += n;
  sv[PM_S_COLOURS] += ncol;
  std::vector<int> off, size;
  T3(class_lists(m, n, ncol, off, size));
  T3(zero_ctr(m));
  for (int s = 0; s < o->smooth_sweeps; ++s)
    for (int c = 0; c < ncol; ++c)
      if (size[c] > 0) k_smooth<<<grid((int64_t)size[c] * kSL), kB, 0, m->s>>>(st, m->cls + off[c], size[c], m->ctr);
  H3(hipGetLastError());
  T3(read_ctr(m));
  sv[PM_S_EVALUATED] = m->hctr[K_EVAL];
  sv[PM_S_COMMITTED] = m->hctr[K_COMMIT];
  sv[PM_S_ROUNDS] = o->smooth_sweeps;
  sv[PM_S_CONVERGED] = 1;
  put_stats(out, sv);
  return PM_OK;
}

pm_status pm3_quality(pm3_mesh* m, double* Q, double* qmin) {
  if (!m) return PM_E_ARG;
  constexpr int NB = 1024;
  if (!m->qbuf) T3(dgrow(m, &m->qbuf, 0, 2 * NB + 2, false));
  k_quality<<<NB, QB, 0, m->s>>>(m->st, m->qbuf, m->qbuf + NB);
  k_quality_final<<<1, 64, 0, m->s>>>(m->qbuf, m->qbuf + NB, NB, m->qbuf + 2 * NB);
  double h[2];
  H3(hipMemcpyAsync(h, m->qbuf + 2 * NB, sizeof(double) * 2, hipMemcpyDeviceToHost, m->s));
  H3(hipStreamSynchronize(m->s));
  if (Q) *Q = h[0];
  if (qmin) *qmin = h[1];
  return PM_OK;
}

const char* pm3_last_error(const pm3_mesh* m) { return m ? m->err.c_str() : g3_create_err.c_str(); }

}  // extern "C"
