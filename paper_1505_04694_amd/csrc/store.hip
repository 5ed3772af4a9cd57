// Device mesh store: ordered scan, input validation, slack-padded CSR rows
// built from the element list, stable compaction, and template refinement.
//
// Rows: NE(v) = live elements holding v, NN(v) = the other vertices of those
// elements (Sec. 3.1: per-vertex adjacency lists). Every row is a sorted id
// set stored in a slack-padded slot of its pool, so the commit can grow it in
// place; a row that outgrows its slot moves to the pool's bump region.
#include "kern.hpp"

namespace pm {

// ---- ordered exclusive scan --------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_B = SCAN_T * SCAN_I;

// exclusive scan over the block; returns the thread's prefix, sets *tot
__device__ int block_excl(int v, int* lds, int* tot) {
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int nw = blockDim.x / kWave;
  int incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  if (lane == kWave - 1) lds[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      int t = lds[w];
      lds[w] = acc;
      acc += t;
    }
    lds[nw] = acc;
  }
  __syncthreads();
  int r = lds[wid] + incl - v;
  *tot = lds[nw];
  __syncthreads();
  return r;
}

__global__ void k_scan_reduce(const int* __restrict__ in, int n, int* __restrict__ partial) {
  __shared__ int lds[SCAN_T / kWave + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_B;
  int s = 0;
  for (int i = threadIdx.x; i < SCAN_B; i += SCAN_T) {
    int64_t j = base + i;
    if (j < n) s += in[j];
  }
  int tot;
  block_excl(s, lds, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_scan_partials(int* __restrict__ partial, int nb, int* __restrict__ total) {
  __shared__ int lds[1024 / kWave + 1];
  int per = (nb + blockDim.x - 1) / blockDim.x;
  int lo = threadIdx.x * per;
  int hi = min(nb, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += partial[i];
  int tot;
  int acc = block_excl(s, lds, &tot);
  for (int i = lo; i < hi; ++i) {
    int t = partial[i];
    partial[i] = acc;
    acc += t;
  }
  if (threadIdx.x == 0) *total = tot;
}

__global__ void k_scan_apply(const int* __restrict__ in, int* __restrict__ out, int n,
                             const int* __restrict__ partial) {
  __shared__ int lds[SCAN_T / kWave + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
  int v[SCAN_I];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_I; ++k) {
    int64_t j = base + k;
    v[k] = j < n ? in[j] : 0;
    s += v[k];
  }
  int tot;
  int acc = block_excl(s, lds, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_I; ++k) {
    int64_t j = base + k;
    if (j < n) out[j] = acc;
    acc += v[k];
  }
}

int scan_partials_needed(int n) { return (n + SCAN_B - 1) / SCAN_B + 1; }

// short arrays: one block of 1024 threads, each scanning a contiguous piece
// of at most eight entries (its loads are serial, two passes: longer pieces
// made a 65536-entry scan take 100 us, against a few for the three-kernel
// form)
constexpr int kScanSingle = 8192;
__global__ void __launch_bounds__(1024) k_scan_single(const int* __restrict__ in, int* __restrict__ out, int n,
                                                      int* __restrict__ total) {
  __shared__ int lds[1024 / kWave + 1];
  int per = (n + 1023) / 1024;
  int lo = (int)threadIdx.x * per;
  int hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += in[i];
  int tot;
  int acc = block_excl(s, lds, &tot);
  for (int i = lo; i < hi; ++i) {
    int t = in[i];
    out[i] = acc;
    acc += t;
  }
  if (threadIdx.x == 0) *total = tot;
}

void scan_excl(const int* in, int* out, int n, int* total, int* partial, hipStream_t s) {
  if (n <= kScanSingle) {
    k_scan_single<<<1, 1024, 0, s>>>(in, out, n, total);
    return;
  }
  int nb = (n + SCAN_B - 1) / SCAN_B;
  if (nb < 1) nb = 1;
  k_scan_reduce<<<nb, SCAN_T, 0, s>>>(in, n, partial);
  k_scan_partials<<<1, 1024, 0, s>>>(partial, nb, total);
  k_scan_apply<<<nb, SCAN_T, 0, s>>>(in, out, n, partial);
}

// ---- validation ---------------------------------------------------------------------
// elements arrive already rotated (smallest id first) by the creation kernel
__global__ void k_validate_elems(const Elem* __restrict__ tri, int T, int V, const double2* __restrict__ xy,
                                 int* ctr) {
  for (int t = gtid(); t < T; t += gstride()) {
    Elem e = tri[t];
    if (!e.w) continue;  // unused slot of a mesh's range
    if (e.x < 0 || e.y < 0 || e.z < 0 || e.x >= V || e.y >= V || e.z >= V || e.x == e.y || e.y == e.z ||
        e.x == e.z) {
      atomicOr(&ctr[C_ERR], E_MESH_ID);
      continue;
    }
    double2 p0 = xy[e.x], p1 = xy[e.y], p2 = xy[e.z];
    double D = (p1.x - p0.x) * (p2.y - p0.y) - (p2.x - p0.x) * (p1.y - p0.y);
    if (!(D > 0.0)) atomicOr(&ctr[C_ERR], E_MESH_ORIENT);
  }
}

__global__ void k_validate_verts(const double2* __restrict__ xy, const Met* __restrict__ met,
                                 const uint8_t* __restrict__ valive, int V, int* ctr) {
  for (int v = gtid(); v < V; v += gstride()) {
    if (!valive[v]) continue;
    Met m = met[v];
    double2 p = xy[v];
    bool ok = (m.a > 0.0) && (m.a * m.c - m.b * m.b > 0.0) && isfinite(m.a) && isfinite(m.b) &&
              isfinite(m.c) && isfinite(p.x) && isfinite(p.y);
    if (!ok) atomicOr(&ctr[C_ERR], E_MESH_METRIC);
  }
}

void k_validate(const Store& st, int* ctr, hipStream_t s) {
  k_validate_elems<<<grid_for(st.T), kBlock, 0, s>>>(st.tri, st.T, st.V, st.xy, ctr);
  k_validate_verts<<<grid_for(st.V), kBlock, 0, s>>>(st.xy, st.met, st.valive, st.V, ctr);
}

// ---- row build ----------------------------------------------------------------------
// Element-to-vertex incidence counts and fills. A block takes a contiguous
// chunk of kIncChunk elements; when the chunk's vertices span at most
// kIncSpan ids (meshes numbered with locality), it counts in LDS and makes
// one global atomic per vertex it touches instead of one per incidence.
constexpr int kIncPer = 4;
constexpr int kIncChunk = kBlock * kIncPer;
constexpr int kIncSpan = 4096;
__device__ __forceinline__ void chunk_span(const Elem* __restrict__ tri, int t0, int t1, int& vmin, int& vmax,
                                           int* red) {
  int lo = INT_MAX, hi = -1;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
    Elem e = tri[t];
    if (!e.w) continue;
    lo = min(lo, min(e.x, min(e.y, e.z)));
    hi = max(hi, max(e.x, max(e.y, e.z)));
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    lo = min(lo, __shfl_xor(lo, d));
    hi = max(hi, __shfl_xor(hi, d));
  }
  int wv = (int)threadIdx.x / kWave;
  if (__lane_id() == 0) {
    red[2 * wv] = lo;
    red[2 * wv + 1] = hi;
  }
  __syncthreads();
  vmin = INT_MAX;
  vmax = -1;
#pragma unroll
  for (int q = 0; q < kBlock / kWave; ++q) {
    vmin = min(vmin, red[2 * q]);
    vmax = max(vmax, red[2 * q + 1]);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_ne_count(const Elem* __restrict__ tri, int T, int* __restrict__ cnt) {
  __shared__ int loc[kIncSpan];
  __shared__ int red[2 * kBlock / kWave];
  int t0 = blockIdx.x * kIncChunk, t1 = min(T, t0 + kIncChunk);
  int vmin, vmax;
  chunk_span(tri, t0, t1, vmin, vmax, red);
  if (vmax < 0) return;
  int span = vmax - vmin + 1;
  if (span > kIncSpan) {
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
      Elem e = tri[t];
      if (!e.w) continue;
      atomicAdd(&cnt[e.x], 1);
      atomicAdd(&cnt[e.y], 1);
      atomicAdd(&cnt[e.z], 1);
    }
    return;
  }
  for (int i = (int)threadIdx.x; i < span; i += kBlock) loc[i] = 0;
  __syncthreads();
  for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
    Elem e = tri[t];
    if (!e.w) continue;
    atomicAdd(&loc[e.x - vmin], 1);
    atomicAdd(&loc[e.y - vmin], 1);
    atomicAdd(&loc[e.z - vmin], 1);
  }
  __syncthreads();
  for (int i = (int)threadIdx.x; i < span; i += kBlock)
    if (loc[i]) atomicAdd(&cnt[vmin + i], loc[i]);
}

void build_count(const Store& st, int* ne_cnt, hipStream_t s) {
  int nb = (st.T + kIncChunk - 1) / kIncChunk;
  if (nb > 0) k_ne_count<<<nb, kBlock, 0, s>>>(st.tri, st.T, ne_cnt);
}

__device__ __forceinline__ int round4(int x) { return (x + 3) & ~3; }

__global__ void k_caps(const int* __restrict__ ne_cnt, int V, double slack, int* __restrict__ nn_cap,
                       int* __restrict__ ne_cap) {
  for (int v = gtid(); v < V; v += gstride()) {
    int c = ne_cnt[v];
    if (c == 0) {
      nn_cap[v] = 0;
      ne_cap[v] = 0;
      continue;
    }
    int a = (int)ceil((double)c * slack);
    int b = (int)ceil((double)(c + 1) * slack);
    ne_cap[v] = round4(max(c + 2, a));
    nn_cap[v] = round4(max(c + 3, b));
  }
}

void build_caps(const Store& st, const int* ne_cnt, double slack, int* nn_cap, int* ne_cap, hipStream_t s) {
  k_caps<<<grid_for(st.V), kBlock, 0, s>>>(ne_cnt, st.V, slack, nn_cap, ne_cap);
}

__global__ void k_set_headers(Hdr* __restrict__ hdr, int2* __restrict__ cap, int V, const int* __restrict__ nn_off,
                              const int* __restrict__ ne_off, const int* __restrict__ nn_cap,
                              const int* __restrict__ ne_cap) {
  for (int v = gtid(); v < V; v += gstride()) {
    hdr[v] = make_int4(nn_off[v], 0, ne_off[v], 0);
    cap[v] = make_int2(nn_cap[v], ne_cap[v]);
  }
}

void set_headers(const Store& st, const int* nn_off, const int* ne_off, const int* nn_cap, const int* ne_cap,
                 hipStream_t s) {
  k_set_headers<<<grid_for(st.V), kBlock, 0, s>>>(st.hdr, st.cap, st.V, nn_off, ne_off, nn_cap, ne_cap);
}

// Fill: each incidence takes a slot of its vertex's NE row (rows are sorted
// by the row finish, so the order of filling does not matter). In the LDS
// path an incidence takes its rank among the chunk's incidences of that
// vertex, and one global atomic per vertex reserves the chunk's slots.
__global__ void __launch_bounds__(256) k_ne_fill(const Elem* __restrict__ tri, int T, Hdr* hdr, int* __restrict__ ne) {
  __shared__ int loc[kIncSpan];
  __shared__ int red[2 * kBlock / kWave];
  int t0 = blockIdx.x * kIncChunk, t1 = min(T, t0 + kIncChunk);
  int vmin, vmax;
  chunk_span(tri, t0, t1, vmin, vmax, red);
  if (vmax < 0) return;
  int span = vmax - vmin + 1;
  if (span > kIncSpan) {
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
      Elem e = tri[t];
      if (!e.w) continue;
      int vs[3] = {e.x, e.y, e.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        int* c = reinterpret_cast<int*>(&hdr[vs[k]]) + 3;
        int pos = atomicAdd(c, 1);
        ne[hdr[vs[k]].z + pos] = t;
      }
    }
    return;
  }
  for (int i = (int)threadIdx.x; i < span; i += kBlock) loc[i] = 0;
  __syncthreads();
  int rank[kIncPer][3];
#pragma unroll
  for (int r = 0; r < kIncPer; ++r) {
    int t = t0 + r * kBlock + (int)threadIdx.x;
    Elem e = t < t1 ? tri[t] : make_int4(0, 0, 0, 0);
    rank[r][0] = rank[r][1] = rank[r][2] = -1;
    if (t < t1 && e.w) {
      rank[r][0] = atomicAdd(&loc[e.x - vmin], 1);
      rank[r][1] = atomicAdd(&loc[e.y - vmin], 1);
      rank[r][2] = atomicAdd(&loc[e.z - vmin], 1);
    }
  }
  __syncthreads();
  // reserve the chunk's slots: loc[i] becomes the first slot of the chunk in
  // row vmin + i; a thread's reservations are all in flight before it uses one
  constexpr int R = kIncSpan / kBlock;
  int cnt[R], at[R], z[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int i = q * kBlock + (int)threadIdx.x;
    cnt[q] = i < span ? loc[i] : 0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int i = q * kBlock + (int)threadIdx.x;
    z[q] = cnt[q] ? hdr[vmin + i].z : 0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int i = q * kBlock + (int)threadIdx.x;
    at[q] = cnt[q] ? atomicAdd(reinterpret_cast<int*>(&hdr[vmin + i]) + 3, cnt[q]) : 0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int i = q * kBlock + (int)threadIdx.x;
    if (cnt[q]) loc[i] = z[q] + at[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kIncPer; ++r) {
    int t = t0 + r * kBlock + (int)threadIdx.x;
    if (rank[r][0] < 0) continue;
    Elem e = tri[t];
    ne[loc[e.x - vmin] + rank[r][0]] = t;
    ne[loc[e.y - vmin] + rank[r][1]] = t;
    ne[loc[e.z - vmin] + rank[r][2]] = t;
  }
}

void build_fill(const Store& st, int* fill, hipStream_t s) {
  (void)fill;
  int nb = (st.T + kIncChunk - 1) / kIncChunk;
  if (nb > 0) k_ne_fill<<<nb, kBlock, 0, s>>>(st.tri, st.T, st.hdr, st.ne);
}

__device__ void isort(int* a, int n) {
  for (int i = 1; i < n; ++i) {
    int x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

// sort NE(v); NN(v) = sorted "next" vertices of v's elements, plus the one
// "previous" vertex that is not a next (boundary vertices). A repeated next
// means a directed edge is used twice: inconsistent orientation or a
// non-manifold edge; more than one unmatched previous is a pinched vertex.
// Rows of up to 16 elements are finished in registers: sorting networks,
// and every previous looked up among all nexts (8-wide when a wavefront's
// rows all fit, 16-wide otherwise).
constexpr int kFinishReg = 16;
template <int N>
__device__ __forceinline__ void row_finish_reg(const Elem* __restrict__ tri, Hdr* __restrict__ hdr, int ncap,
                                               int* __restrict__ nn, int* __restrict__ ne, int v, Hdr h,
                                               int* ctr) {
  int c = h.w;
  int r[N];
  if constexpr (N == 8) {
    row8(ne, h.z, c, r);
#pragma unroll
    for (int k = 0; k < N; ++k)
      if (k >= c) r[k] = INT_MAX;
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) r[k] = k < c ? ne[h.z + k] : INT_MAX;
  }
  bitonic<N>(r);
  // the elements' loads go out together (an empty slot loads the first
  // element again rather than branch around its load)
  int nx[N], pv[N];
  if constexpr (N == 8) {
    // the sorted row, four entries per store (the slot holds a multiple of four)
    *(int4*)(ne + h.z) = make_int4(r[0], r[1], r[2], r[3]);
    if (c > 4) *(int4*)(ne + h.z + 4) = make_int4(r[4], r[5], r[6], r[7]);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (N != 8 && k < c) ne[h.z + k] = r[k];
    Elem e = tri[k < c ? r[k] : r[0]];
    int s = slot_of(e, v);
    nx[k] = k < c ? at(e, s == 2 ? 0 : s + 1) : INT_MAX;
    pv[k] = k < c ? at(e, s == 0 ? 2 : s - 1) : INT_MAX;
  }
  bitonic<N>(nx);
  bool bad = false;
#pragma unroll
  for (int k = 1; k < N; ++k) bad |= nx[k] != INT_MAX && nx[k] == nx[k - 1];
  int extra = INT_MAX, nextra = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (pv[k] == INT_MAX) continue;
    bool found = false;
#pragma unroll
    for (int q = 0; q < N; ++q) found |= nx[q] == pv[k];
    if (!found) {
      extra = pv[k];
      ++nextra;
    }
  }
  int n = c + nextra;
  if (nextra > 1 || n > ncap) bad = true;
  if (bad) {
    atomicOr(&ctr[C_ERR], E_MESH_MANIFOLD);
    n = c;
    nextra = 0;
  }
  int w = 0;
  bool put = nextra == 0;
  int* out = nn + h.x;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int x = nx[k];
    if (x == INT_MAX) continue;
    if (!put && extra < x) {
      out[w++] = extra;
      put = true;
    }
    out[w++] = x;
  }
  if (!put) out[w++] = extra;
  reinterpret_cast<int*>(&hdr[v])[1] = n;
}

__global__ void k_row_finish(const Elem* __restrict__ tri, Hdr* __restrict__ hdr, const int2* __restrict__ cap,
                             int* __restrict__ nn, int* __restrict__ ne, int V, int* ctr) {
  for (int v = gtid(); v < V; v += gstride()) {
    Hdr h = hdr[v];
    int c = h.w;
    if (c == 0) continue;
    if (c <= kFinishReg) {
      if (__all(c <= 8)) row_finish_reg<8>(tri, hdr, cap[v].x, nn, ne, v, h, ctr);
      else row_finish_reg<kFinishReg>(tri, hdr, cap[v].x, nn, ne, v, h, ctr);
      continue;
    }
    int* row = ne + h.z;
    isort(row, c);
    int* out = nn + h.x;
    int ncap = cap[v].x;
    for (int i = 0; i < c; ++i) {
      Elem e = tri[row[i]];
      int k = slot_of(e, v);
      out[i] = at(e, k == 2 ? 0 : k + 1);
    }
    isort(out, c);
    bool bad = false;
    for (int i = 1; i < c; ++i)
      if (out[i] == out[i - 1]) bad = true;
    int n = c, extra = 0;
    for (int i = 0; i < c && !bad; ++i) {
      Elem e = tri[row[i]];
      int k = slot_of(e, v);
      int p = at(e, k == 0 ? 2 : k - 1);
      // binary search in the current sorted row out[0..n)
      int lo = 0, hi = n;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (out[mid] < p) lo = mid + 1;
        else hi = mid;
      }
      if (lo < n && out[lo] == p) continue;
      if (++extra > 1 || n + 1 > ncap) {
        bad = true;
        break;
      }
      // insert p into out[0..n)
      int j = n - 1;
      while (j >= 0 && out[j] > p) {
        out[j + 1] = out[j];
        --j;
      }
      out[j + 1] = p;
      ++n;
    }
    if (bad) atomicOr(&ctr[C_ERR], E_MESH_MANIFOLD);
    reinterpret_cast<int*>(&hdr[v])[1] = n;
  }
}

void build_finish(const Store& st, int* ctr, hipStream_t s) {
  k_row_finish<<<grid_for(st.V), kBlock, 0, s>>>(st.tri, st.hdr, st.cap, st.nn, st.ne, st.V, ctr);
}

// ---- compaction --------------------------------------------------------------------------
__global__ void k_flag_v(const uint8_t* __restrict__ valive, int V, int* __restrict__ f) {
  for (int v = gtid(); v < V; v += gstride()) f[v] = valive[v] ? 1 : 0;
}
__global__ void k_flag_t(const Elem* __restrict__ tri, int T, int* __restrict__ f) {
  for (int t = gtid(); t < T; t += gstride()) f[t] = tri[t].w ? 1 : 0;
}
void flag_live_vertices(const Store& st, int* flag, hipStream_t s) {
  k_flag_v<<<grid_for(st.V), kBlock, 0, s>>>(st.valive, st.V, flag);
}
void flag_live_elements(const Store& st, int* flag, hipStream_t s) {
  k_flag_t<<<grid_for(st.T), kBlock, 0, s>>>(st.tri, st.T, flag);
}

__global__ void k_compact_v(const double2* __restrict__ xy, const Met* __restrict__ met,
                            const uint8_t* __restrict__ tag, const uint8_t* __restrict__ valive, int V,
                            const int* __restrict__ vmap, double2* __restrict__ xy2, Met* __restrict__ met2,
                            uint8_t* __restrict__ tag2, uint8_t* __restrict__ va2) {
  for (int v = gtid(); v < V; v += gstride()) {
    if (!valive[v]) continue;
    int n = vmap[v];
    xy2[n] = xy[v];
    met2[n] = met[v];
    tag2[n] = tag[v];
    va2[n] = 1;
  }
}
void compact_vertices(const Store& st, const int* vmap, double2* xy2, Met* met2, uint8_t* tag2, uint8_t* va2,
                      hipStream_t s) {
  k_compact_v<<<grid_for(st.V), kBlock, 0, s>>>(st.xy, st.met, st.tag, st.valive, st.V, vmap, xy2, met2, tag2, va2);
}

__global__ void k_range_sums(const int* __restrict__ scan, const int* __restrict__ src, const int* __restrict__ base,
                             const int* __restrict__ used, int B, int* __restrict__ out) {
  for (int i = gtid(); i < B; i += gstride()) {
    int lo = base[i], hi = base[i] + used[i];
    // inclusive value at hi - 1 minus exclusive value at lo
    out[i] = hi > lo ? scan[hi - 1] + src[hi - 1] - scan[lo] : 0;
  }
}
void range_sums(const int* scan, const int* src, const int* base, const int* used, int B, int* out, hipStream_t s) {
  k_range_sums<<<grid_for(B), kBlock, 0, s>>>(scan, src, base, used, B, out);
}

__global__ void k_mesh_maps(const int* __restrict__ flag, const int* __restrict__ scan, const int* __restrict__ mesh,
                            const int* __restrict__ base, const int* __restrict__ nbase, int n, int* __restrict__ map) {
  for (int x = gtid(); x < n; x += gstride()) {
    if (!flag[x]) continue;
    int i = mesh ? mesh[x] : 0;
    map[x] = nbase[i] + scan[x] - scan[base[i]];
  }
}
void mesh_maps(const int* flag, const int* scan, const int* mesh, const int* base, const int* nbase, int n, int* map,
               hipStream_t s) {
  k_mesh_maps<<<grid_for(n), kBlock, 0, s>>>(flag, scan, mesh, base, nbase, n, map);
}

__global__ void k_fill_mesh_ids(const int* __restrict__ base, int B, int n, int* __restrict__ mesh) {
  for (int x = gtid(); x < n; x += gstride()) {
    int lo = 0, hi = B;  // last i with base[i] <= x
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (base[mid] <= x) lo = mid;
      else hi = mid;
    }
    mesh[x] = lo;
  }
}
void fill_mesh_ids(const int* base, int B, int n, int* mesh, hipStream_t s) {
  k_fill_mesh_ids<<<grid_for(n), kBlock, 0, s>>>(base, B, n, mesh);
}

__global__ void k_compact_t(const Elem* __restrict__ tri, int T, const int* __restrict__ vmap,
                            const int* __restrict__ tmap, Elem* __restrict__ tri2) {
  for (int t = gtid(); t < T; t += gstride()) {
    Elem e = tri[t];
    if (!e.w) continue;
    // the renumbering is monotone, so the smallest id stays first
    tri2[tmap[t]] = make_int4(vmap[e.x], vmap[e.y], vmap[e.z], 1);
  }
}
void compact_elements(const Store& st, const int* vmap, const int* tmap, Elem* tri2, hipStream_t s) {
  k_compact_t<<<grid_for(st.T), kBlock, 0, s>>>(st.tri, st.T, vmap, tmap, tri2);
}

// ---- refinement (Sec. 2.4.2) ------------------------------------------------------------
__device__ __forceinline__ double elen2(const double2* xy, const Met* met, int i, int j) {
  return len2(xy[i], met[i], xy[j], met[j]);
}

// count long edges (a, b > a) per vertex; also counts tested edges. Meshes of
// a batch that have finished refining are skipped.
__global__ void k_refine_mark(Store st, double L_up2, int* __restrict__ cnt, int* ctr) {
  const double2* xy = st.xy;
  const Met* met = st.met;
  const Hdr* hdr = st.hdr;
  const int* nn = st.nn;
  int V = st.V;
  int stride = gstride();
  for (int v0 = blockIdx.x * blockDim.x; v0 < V; v0 += stride) {
    int a = v0 + (int)threadIdx.x;
    int tested = 0, c = 0;
    if (a < V) {
      bool skip = st.mdone && st.mdone[st.vmesh ? st.vmesh[a] : 0];
      if (st.valive[a] && !skip) {
        Hdr h = hdr[a];
        for (int j = 0; j < h.y; ++j) {
          int b = nn[h.x + j];
          if (b <= a) continue;
          ++tested;
          if (elen2(xy, met, a, b) > L_up2) ++c;
        }
      }
      cnt[a] = c;
    }
    wave_add_full(stripe_ptr(ctr, S_EDGES), tested);
  }
}
void refine_mark(const Store& st, double L_up2, int* cnt, int* ctr, hipStream_t s) {
  k_refine_mark<<<grid_for(st.V), kBlock, 0, s>>>(st, L_up2, cnt, ctr);
}

// new vertex ids inside the vertex's mesh range: base + used + (long edges of
// the mesh before a, in (a, b) order) + rank in a's row
__global__ void k_refine_mint(Store st, double L_up2, const int* __restrict__ vscan, int* __restrict__ mid) {
  for (int a = gtid(); a < st.V; a += gstride()) {
    if (!st.valive[a]) continue;
    int i = st.vmesh ? st.vmesh[a] : 0;
    if (a >= st.vbase[i] + st.vused[i]) continue;  // minted in this pass
    Hdr h = st.hdr[a];
    int first = st.vbase[i] + st.vused[i] + vscan[a] - vscan[st.vbase[i]];
    int k = 0;
    for (int j = 0; j < h.y; ++j) {
      int b = st.nn[h.x + j];
      if (b <= a) continue;
      if (!(elen2(st.xy, st.met, a, b) > L_up2)) continue;
      int id = first + k++;
      mid[h.x + j] = id;
      double2 pa = st.xy[a], pb = st.xy[b];
      Met ma = st.met[a], mb = st.met[b];
      st.xy[id] = make_double2((pa.x + pb.x) * 0.5, (pa.y + pb.y) * 0.5);
      Met mm;
      mm.a = (ma.a + mb.a) * 0.5;
      mm.b = (ma.b + mb.b) * 0.5;
      mm.c = (ma.c + mb.c) * 0.5;
      st.met[id] = mm;
      st.tag[id] = st.tag[a] & st.tag[b];
      st.valive[id] = 1;
    }
  }
}
void refine_mint(const Store& st, double L_up2, const int* vscan, int* mid, hipStream_t s) {
  k_refine_mint<<<grid_for(st.V), kBlock, 0, s>>>(st, L_up2, vscan, mid);
}

__global__ void k_refine_count(const double2* __restrict__ xy, const Met* __restrict__ met,
                               const Elem* __restrict__ tri, int T, double L_up2, int* __restrict__ ecnt) {
  for (int t = gtid(); t < T; t += gstride()) {
    Elem e = tri[t];
    int c = 0;
    if (e.w) {
      c += elen2(xy, met, e.x, e.y) > L_up2;
      c += elen2(xy, met, e.y, e.z) > L_up2;
      c += elen2(xy, met, e.z, e.x) > L_up2;
    }
    ecnt[t] = c;
  }
}
void refine_count(const Store& st, double L_up2, int* ecnt, hipStream_t s) {
  k_refine_count<<<grid_for(st.T), kBlock, 0, s>>>(st.xy, st.met, st.tri, st.T, L_up2, ecnt);
}

__device__ int midpoint_of(const Hdr* hdr, const int* nn, const int* mid, int p, int q) {
  int a = min(p, q), b = max(p, q);
  Hdr h = hdr[a];
  int lo = 0, hi = h.y;
  while (lo < hi) {
    int m = (lo + hi) >> 1;
    if (nn[h.x + m] < b) lo = m + 1;
    else hi = m;
  }
  return mid[h.x + lo];
}

__device__ __forceinline__ Elem mk(int a, int b, int c) {
  int3 r = rot_min(a, b, c);
  return make_int4(r.x, r.y, r.z, 1);
}

// children by template; the first keeps the parent id, the others take ids
// inside the element's mesh range: base + used + (new children of the mesh
// before t) + (child index - 1)
__global__ void k_refine_split(Store st, double L_up2, const int* __restrict__ mid, const int* __restrict__ escan) {
  const double2* xy = st.xy;
  const Met* met = st.met;
  Elem* tri = st.tri;
  const Hdr* hdr = st.hdr;
  const int* nn = st.nn;
  int T = st.T;
  for (int t = gtid(); t < T; t += gstride()) {
    Elem e = tri[t];
    if (!e.w) continue;
    int i = st.tmesh ? st.tmesh[t] : 0;
    if (t >= st.tbase[i] + st.tused[i]) continue;  // a child written in this pass
    int m0 = elen2(xy, met, e.x, e.y) > L_up2 ? midpoint_of(hdr, nn, mid, e.x, e.y) : -1;
    int m1 = elen2(xy, met, e.y, e.z) > L_up2 ? midpoint_of(hdr, nn, mid, e.y, e.z) : -1;
    int m2 = elen2(xy, met, e.z, e.x) > L_up2 ? midpoint_of(hdr, nn, mid, e.z, e.x) : -1;
    int ns = (m0 >= 0) + (m1 >= 0) + (m2 >= 0);
    if (ns == 0) continue;
    Elem ch[4];
    if (ns == 1) {
      // the split edge k runs P -> Q with mid-point M, R opposite
      int k = m0 >= 0 ? 0 : (m1 >= 0 ? 1 : 2);
      int P = at(e, k), Q = at(e, k == 2 ? 0 : k + 1), R = at(e, k == 0 ? 2 : k - 1);
      int M = k == 0 ? m0 : (k == 1 ? m1 : m2);
      ch[0] = mk(P, M, R);
      ch[1] = mk(M, Q, R);
    } else if (ns == 2) {
      // the unsplit edge k runs P -> Q; M1 on Q-R, M2 on R-P
      int k = m0 < 0 ? 0 : (m1 < 0 ? 1 : 2);
      int P = at(e, k), Q = at(e, k == 2 ? 0 : k + 1), R = at(e, k == 0 ? 2 : k - 1);
      int M1 = k == 0 ? m1 : (k == 1 ? m2 : m0);
      int M2 = k == 0 ? m2 : (k == 1 ? m0 : m1);
      ch[0] = mk(M1, R, M2);
      double dP = elen2(xy, met, P, M1), dQ = elen2(xy, met, Q, M2);
      if (dP <= dQ) {
        ch[1] = mk(P, Q, M1);
        ch[2] = mk(P, M1, M2);
      } else {
        ch[1] = mk(P, Q, M2);
        ch[2] = mk(Q, M1, M2);
      }
    } else {
      ch[0] = mk(e.x, m0, m2);
      ch[1] = mk(m0, e.y, m1);
      ch[2] = mk(m2, m1, e.z);
      ch[3] = mk(m0, m1, m2);
    }
    tri[t] = ch[0];
    int base = st.tbase[i] + st.tused[i] + escan[t] - escan[st.tbase[i]];
    tri[base] = ch[1];
    if (ns >= 2) tri[base + 1] = ch[2];
    if (ns == 3) tri[base + 2] = ch[3];
  }
}
void refine_split(const Store& st, double L_up2, const int* mid, const int* escan, hipStream_t s) {
  k_refine_split<<<grid_for(st.T), kBlock, 0, s>>>(st, L_up2, mid, escan);
}

// ---- small utilities ---------------------------------------------------------------------------
// (plain kernels rather than memset nodes, so the sequences stay graph-safe)
__global__ void k_zero(int* __restrict__ p, int n) {
  for (int i = gtid(); i < n; i += gstride()) p[i] = 0;
}
void zero_ints(int* p, int n, hipStream_t s) {
  if (n > 0) k_zero<<<grid_for(n, 1024), kBlock, 0, s>>>(p, n);
}
__global__ void k_fill_u8(uint8_t* __restrict__ p, int n, uint8_t v) {
  for (int i = gtid(); i < n; i += gstride()) p[i] = v;
}
void fill_u8(uint8_t* p, int n, uint8_t v, hipStream_t s) {
  if (n > 0) k_fill_u8<<<grid_for(n, 1024), kBlock, 0, s>>>(p, n, v);
}
__global__ void k_set_int(int* p, int v) { *p = v; }
void set_int(int* p, int v, hipStream_t s) { k_set_int<<<1, 1, 0, s>>>(p, v); }

// input triangles (T x 3) to stored elements: rotated smallest-id first, live
__global__ void k_tri_in(const int* __restrict__ tri3, int T, Elem* __restrict__ tri) {
  for (int t = gtid(); t < T; t += gstride()) {
    int a = tri3[3 * t], b = tri3[3 * t + 1], c = tri3[3 * t + 2];
    int3 r = rot_min(a, b, c);
    tri[t] = make_int4(r.x, r.y, r.z, 1);
  }
}
void tri_in(const int* tri3, int T, Elem* tri, hipStream_t s) {
  k_tri_in<<<grid_for(T), kBlock, 0, s>>>(tri3, T, tri);
}
__global__ void k_xy_in(const double* __restrict__ xy, int V, double2* __restrict__ out) {
  for (int v = gtid(); v < V; v += gstride()) out[v] = make_double2(xy[2 * v], xy[2 * v + 1]);
}
void xy_in(const double* xy, int V, double2* out, hipStream_t s) {
  k_xy_in<<<grid_for(V), kBlock, 0, s>>>(xy, V, out);
}
// unit-square side tags from exact coordinates
__global__ void k_tags(const double2* __restrict__ xy, int V, uint8_t* __restrict__ tag) {
  for (int v = gtid(); v < V; v += gstride()) {
    double2 p = xy[v];
    uint8_t t = 0;
    if (p.x == 0.0) t |= 1;
    if (p.x == 1.0) t |= 2;
    if (p.y == 0.0) t |= 4;
    if (p.y == 1.0) t |= 8;
    tag[v] = t;
  }
}
void tags_from_xy(const double2* xy, int V, uint8_t* tag, hipStream_t s) {
  k_tags<<<grid_for(V), kBlock, 0, s>>>(xy, V, tag);
}

// ---- export --------------------------------------------------------------------------------
__global__ void k_export_tri(const Elem* __restrict__ tri, int T, int* __restrict__ tri3, uint8_t* talive) {
  for (int t = gtid(); t < T; t += gstride()) {
    Elem e = tri[t];
    if (tri3) {
      tri3[3 * t] = e.x;
      tri3[3 * t + 1] = e.y;
      tri3[3 * t + 2] = e.z;
    }
    if (talive) talive[t] = e.w ? 1 : 0;
  }
}
void export_tri(const Store& st, int* tri3, uint8_t* talive, hipStream_t s) {
  k_export_tri<<<grid_for(st.T), kBlock, 0, s>>>(st.tri, st.T, tri3, talive);
}

}  // namespace pm
