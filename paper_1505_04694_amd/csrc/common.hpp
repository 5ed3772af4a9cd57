// Device-side building blocks shared by the adaptation kernels: the canonical
// FP64 arithmetic of the metric geometry, the vertex priority hash, element
// rotation, and wavefront-aggregated list appends.
//
// Every floating-point expression is written in one fixed order and compiled
// with -ffp-contract=off, so a decision taken here (L^2 < 0.5, area > 0,
// q^2 >= q_min^2, ...) is the same decision a serial IEEE-754 program makes
// from the same inputs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

struct Met {
  double a, b, c;  // [[a, b], [b, c]]
};

// a vertex's coordinates, metric and boundary tag in one 64-byte line, for
// the kernels that gather them for many neighbours at once
struct alignas(64) VRec {
  double x, y;
  double a, b, c;
  int tag;
  int pad0;
  double pad1, pad2;
};

// element: three vertex ids, counter-clockwise, smallest id first; w = 1 live
typedef int4 Elem;

// vertex row headers: NN row (offset, count), NE row (offset, count)
typedef int4 Hdr;

constexpr int kWave = 64;
constexpr double kK4R3 = 6.928203230275509;  // the double nearest 4 sqrt(3)
constexpr double kK12R3 = 20.784609690826528;  // the double nearest 12 sqrt(3)

// ---- metric geometry (Sec. 2.2) ---------------------------------------------

// squared length of edge i-j in the mean tensor of its end points
__device__ __forceinline__ double len2(double2 pi, Met mi, double2 pj, Met mj) {
  double a = (mi.a + mj.a) * 0.5;
  double b = (mi.b + mj.b) * 0.5;
  double c = (mi.c + mj.c) * 0.5;
  double dx = pj.x - pi.x;
  double dy = pj.y - pi.y;
  return ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
}

// an element's geometry: vertex coordinates in stored order and the mean tensor
struct Geo {
  double x[3], y[3];
  double a, b, c;
};

__device__ __forceinline__ Geo make_geo(double2 p0, double2 p1, double2 p2, Met m0, Met m1, Met m2) {
  Geo g;
  g.x[0] = p0.x; g.y[0] = p0.y;
  g.x[1] = p1.x; g.y[1] = p1.y;
  g.x[2] = p2.x; g.y[2] = p2.y;
  g.a = ((m0.a + m1.a) + m2.a) / 3.0;
  g.b = ((m0.b + m1.b) + m2.b) / 3.0;
  g.c = ((m0.c + m1.c) + m2.c) / 3.0;
  return g;
}

__device__ __forceinline__ double area2(const Geo& g) {
  return (g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]);
}

struct Parts {
  double D, A, S, det;
  double ex[3], ey[3];
};

__device__ __forceinline__ Parts parts(const Geo& g) {
  Parts p;
  p.D = area2(g);
  p.A = 0.5 * p.D;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int k1 = k == 2 ? 0 : k + 1;
    p.ex[k] = g.x[k1] - g.x[k];
    p.ey[k] = g.y[k1] - g.y[k];
  }
  double l0 = ((g.a * p.ex[0]) * p.ex[0] + ((2.0 * g.b) * p.ex[0]) * p.ey[0]) + (g.c * p.ey[0]) * p.ey[0];
  double l1 = ((g.a * p.ex[1]) * p.ex[1] + ((2.0 * g.b) * p.ex[1]) * p.ey[1]) + (g.c * p.ey[1]) * p.ey[1];
  double l2 = ((g.a * p.ex[2]) * p.ex[2] + ((2.0 * g.b) * p.ex[2]) * p.ey[2]) + (g.c * p.ey[2]) * p.ey[2];
  p.S = (l0 + l1) + l2;
  p.det = g.a * g.c - g.b * g.b;
  return p;
}

// q^2 = 48 det(M) A^2 / S^2: every decision uses this square-root-free form
__device__ __forceinline__ double qual2(const Geo& g) {
  Parts p = parts(g);
  return (((48.0 * p.det) * p.A) * p.A) / (p.S * p.S);
}

__device__ __forceinline__ double qual(const Geo& g) {
  Parts p = parts(g);
  return ((kK4R3 * sqrt(p.det)) * p.A) / p.S;
}

// value of slot k of a 3-array without dynamic indexing (keeps it in registers)
__device__ __forceinline__ double sel3(double a0, double a1, double a2, int k) {
  return k == 0 ? a0 : (k == 1 ? a1 : a2);
}

// dq/dx for the vertex in slot k
__device__ __forceinline__ void qual_grad_x(const Geo& g, int k, double& gx, double& gy) {
  Parts p = parts(g);
  double s = sqrt(p.det);
  // slots k+1 and k+2 (= k-1), cyclically
  double x1 = sel3(g.x[1], g.x[2], g.x[0], k), x2 = sel3(g.x[2], g.x[0], g.x[1], k);
  double y1 = sel3(g.y[1], g.y[2], g.y[0], k), y2 = sel3(g.y[2], g.y[0], g.y[1], k);
  double exk = sel3(p.ex[0], p.ex[1], p.ex[2], k), exm = sel3(p.ex[2], p.ex[0], p.ex[1], k);
  double eyk = sel3(p.ey[0], p.ey[1], p.ey[2], k), eym = sel3(p.ey[2], p.ey[0], p.ey[1], k);
  double dAx = 0.5 * (y1 - y2);
  double dAy = 0.5 * (x2 - x1);
  double ux = exm - exk;
  double uy = eym - eyk;
  double dSx = 2.0 * (g.a * ux + g.b * uy);
  double dSy = 2.0 * (g.b * ux + g.c * uy);
  double Ks = kK4R3 * s;
  double SS = p.S * p.S;
  gx = (Ks * (dAx * p.S - p.A * dSx)) / SS;
  gy = (Ks * (dAy * p.S - p.A * dSy)) / SS;
}

// dq/d(mean tensor entries); b is the stored off-diagonal entry
__device__ __forceinline__ void qual_grad_m(const Geo& g, double& da, double& db, double& dc) {
  Parts p = parts(g);
  double s = sqrt(p.det);
  double Sxx = (p.ex[0] * p.ex[0] + p.ex[1] * p.ex[1]) + p.ex[2] * p.ex[2];
  double Sxy = (p.ex[0] * p.ey[0] + p.ex[1] * p.ey[1]) + p.ex[2] * p.ey[2];
  double Syy = (p.ey[0] * p.ey[0] + p.ey[1] * p.ey[1]) + p.ey[2] * p.ey[2];
  double KA = kK4R3 * p.A;
  double SS = p.S * p.S;
  da = (KA * ((g.c * p.S) / (2.0 * s) - s * Sxx)) / SS;
  db = (KA * (-(g.b * p.S) / s - (2.0 * s) * Sxy)) / SS;
  dc = (KA * ((g.a * p.S) / (2.0 * s) - s * Syy)) / SS;
}

// ---- Vasilevskii's functional with its size factor (Sec. 2.2) ---------------------
// Q_V = 12 sqrt(3) sqrt(det M) A / P^2 * F(P / 3), P the sum of the three metric
// edge lengths, F(x) = (m (2 - m))^3 with m = min(x, 1/x): 1 exactly for the
// equilateral triangle with unit metric edges. Decisions compare Q_V^2 (the
// product rounded once) with q_min^2, as the mean ratio's compare q^2.

struct VParts {
  double A, s, P;
  double L[3], ex[3], ey[3];
};

__device__ __forceinline__ VParts vparts(const Geo& g) {
  VParts v;
  v.A = 0.5 * area2(g);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int k1 = k == 2 ? 0 : k + 1;
    v.ex[k] = g.x[k1] - g.x[k];
    v.ey[k] = g.y[k1] - g.y[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    v.L[k] = sqrt(((g.a * v.ex[k]) * v.ex[k] + ((2.0 * g.b) * v.ex[k]) * v.ey[k]) + (g.c * v.ey[k]) * v.ey[k]);
  v.P = (v.L[0] + v.L[1]) + v.L[2];
  v.s = sqrt(g.a * g.c - g.b * g.b);
  return v;
}

// G(P) = F(P / 3) / P^2 and dG/dP
__device__ __forceinline__ void vas_size(double P, double& G, double& dG) {
  double x = P / 3.0;
  bool below = x < 1.0;
  double mm = below ? x : 1.0 / x;
  double f = mm * (2.0 - mm);
  double F = (f * f) * f;
  double dm = below ? 1.0 : -1.0 / (x * x);
  double dF = ((3.0 * (f * f)) * (2.0 - 2.0 * mm)) * dm;
  double P2 = P * P;
  G = F / P2;
  dG = dF / (3.0 * P2) - (2.0 * F) / (P2 * P);
}

__device__ __forceinline__ double vas_q(const Geo& g) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, G, dG);
  return ((kK12R3 * v.s) * v.A) * G;
}

__device__ __forceinline__ void vas_grad_x(const Geo& g, int k, double& gx, double& gy) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, G, dG);
  double x1 = sel3(g.x[1], g.x[2], g.x[0], k), x2 = sel3(g.x[2], g.x[0], g.x[1], k);
  double y1 = sel3(g.y[1], g.y[2], g.y[0], k), y2 = sel3(g.y[2], g.y[0], g.y[1], k);
  double exk = sel3(v.ex[0], v.ex[1], v.ex[2], k), exm = sel3(v.ex[2], v.ex[0], v.ex[1], k);
  double eyk = sel3(v.ey[0], v.ey[1], v.ey[2], k), eym = sel3(v.ey[2], v.ey[0], v.ey[1], k);
  double Lk = sel3(v.L[0], v.L[1], v.L[2], k), Lm = sel3(v.L[2], v.L[0], v.L[1], k);
  double dAx = 0.5 * (y1 - y2);
  double dAy = 0.5 * (x2 - x1);
  // x_k ends edge k-1 and starts edge k: dP/dx_k = M e_{k-1} / L_{k-1} - M e_k / L_k
  double dPx = (g.a * exm + g.b * eym) / Lm - (g.a * exk + g.b * eyk) / Lk;
  double dPy = (g.b * exm + g.c * eym) / Lm - (g.b * exk + g.c * eyk) / Lk;
  double Ks = kK12R3 * v.s;
  gx = Ks * (dAx * G + (v.A * dG) * dPx);
  gy = Ks * (dAy * G + (v.A * dG) * dPy);
}

__device__ __forceinline__ void vas_grad_m(const Geo& g, double& da, double& db, double& dc) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, G, dG);
  double Pa = 0.0, Pb = 0.0, Pc = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Pa = Pa + (v.ex[j] * v.ex[j]) / (2.0 * v.L[j]);
    Pb = Pb + (v.ex[j] * v.ey[j]) / v.L[j];
    Pc = Pc + (v.ey[j] * v.ey[j]) / (2.0 * v.L[j]);
  }
  double KA = kK12R3 * v.A;
  da = KA * ((g.c / (2.0 * v.s)) * G + (v.s * dG) * Pa);
  db = KA * (-(g.b / v.s) * G + (v.s * dG) * Pb);
  dc = KA * ((g.a / (2.0 * v.s)) * G + (v.s * dG) * Pc);
}

// The element functional a handle was created with (qk: 0 the mean ratio,
// 1 Vasilevskii's): the squared value every decision compares, the reported
// value, and its derivatives.
__device__ __forceinline__ double qd2(const Geo& g, int qk) {
  if (qk) {
    double q = vas_q(g);
    return q * q;
  }
  return qual2(g);
}
__device__ __forceinline__ double qval(const Geo& g, int qk) { return qk ? vas_q(g) : qual(g); }
__device__ __forceinline__ void qgrad_x(const Geo& g, int k, int qk, double& gx, double& gy) {
  if (qk)
    vas_grad_x(g, k, gx, gy);
  else
    qual_grad_x(g, k, gx, gy);
}
__device__ __forceinline__ void qgrad_m(const Geo& g, int qk, double& da, double& db, double& dc) {
  if (qk)
    vas_grad_m(g, da, db, dc);
  else
    qual_grad_m(g, da, db, dc);
}

// ---- ids ----------------------------------------------------------------------

// counter-clockwise rotation with the smallest id first
__device__ __forceinline__ int3 rot_min(int a, int b, int c) {
  if (a < b && a < c) return make_int3(a, b, c);
  if (b < a && b < c) return make_int3(b, c, a);
  return make_int3(c, a, b);
}

__device__ __forceinline__ int slot_of(const Elem& e, int v) { return e.x == v ? 0 : (e.y == v ? 1 : 2); }
__device__ __forceinline__ int at(const Elem& e, int k) { return k == 0 ? e.x : (k == 1 ? e.y : e.z); }
__device__ __forceinline__ bool holds(const Elem& e, int v) { return e.x == v || e.y == v || e.z == v; }

// ---- priorities (Sec. 3.2) -------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014) taken as a counter-based generator: the
// i-th output of the stream seeded with s is mix(s + (i + 1) * gamma). A round's
// stream seed is the first output of the stream seeded with seed ^ (ctx << 32);
// a vertex's priority is the high half of that stream's id-th output.
__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream_seed(uint64_t seed, uint32_t ctx) {
  uint64_t z = (seed ^ ((uint64_t)ctx << 32)) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// 64-bit key: priority in the high half, id in the low half; larger wins
__device__ __forceinline__ uint64_t vkey(uint64_t sseed, uint32_t id) {
  uint64_t p = sm_mix(sseed + ((uint64_t)id + 1ull) * 0x9E3779B97F4A7C15ull) >> 32;
  return (p << 32) | (uint64_t)id;
}

__host__ __device__ __forceinline__ uint32_t make_ctx(int sweep, int phase, int round) {
  return ((uint32_t)sweep << 20) | ((uint32_t)phase << 16) | (uint32_t)round;
}
enum { PH_COARSEN = 1, PH_SWAP = 2, PH_SMOOTH = 3 };

// ---- wavefront-aggregated appends (Sec. 3.4) --------------------------------------
// The lanes that reach this call together take one fetch-and-add on the list
// counter, then each writes at base + its rank among them.
__device__ __forceinline__ int wave_append_slot(int* counter) {
  uint64_t mask = __ballot(1);
  int lane = __lane_id();
  int leader = __ffsll((unsigned long long)mask) - 1;
  int rank = __popcll(mask & ((1ull << lane) - 1ull));
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + rank;
}

// add a per-lane amount with one atomic per wavefront; all 64 lanes of the
// wavefront must make this call together (amount 0 for idle lanes)
__device__ __forceinline__ int wave_add_full(int* counter, int amount) {
  int lane = __lane_id();
  int incl = amount;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  int total = __shfl(incl, kWave - 1);
  int base = 0;
  if (lane == kWave - 1 && total > 0) base = atomicAdd(counter, total);
  base = __shfl(base, kWave - 1);
  return base + incl - amount;
}

// Entries [off, off + 8) of a row slot holding cnt entries there (-1 past
// them), as two 16-byte loads: slots start at multiples of four entries and
// hold a multiple of four, so neither load leaves the slot.
__device__ __forceinline__ void row8(const int* pool, int off, int cnt, int (&t)[8]) {
  int4 a = make_int4(-1, -1, -1, -1), b = a;
  if (cnt > 0) a = *(const int4*)(pool + off);
  if (cnt > 4) b = *(const int4*)(pool + off + 4);
  t[0] = a.x;
  t[1] = a.y;
  t[2] = a.z;
  t[3] = a.w;
  t[4] = b.x;
  t[5] = b.y;
  t[6] = b.z;
  t[7] = b.w;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (q >= cnt) t[q] = -1;
}

// XCD-aware block order. Work-groups are dealt to the 8 XCDs in turn (block b
// runs on XCD b % 8), and each XCD has its own L2. Renumbering blocks so that
// every XCD receives one contiguous eighth of the grid keeps neighbouring work
// items (neighbouring vertices, when lists are in vertex order) in one L2.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_block() {
  int nb = gridDim.x, b = blockIdx.x;
  int per = nb / kXcd, rem = nb % kXcd;
  int x = b % kXcd, k = b / kXcd;
  return x * per + min(x, rem) + k;
}
__device__ __forceinline__ int xtid() { return xcd_block() * blockDim.x + threadIdx.x; }

// sorting network on a register array (all indices are compile-time constants)
template <int N>
__device__ __forceinline__ void bitonic(int (&a)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        int l = i ^ j;
        if (l > i) {
          int x = a[i], y = a[l];
          int lo = min(x, y), hi = max(x, y);
          bool up = (i & k) == 0;
          a[i] = up ? lo : hi;
          a[l] = up ? hi : lo;
        }
      }
    }
  }
}

// grid-stride helpers
__device__ __forceinline__ int gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int gstride() { return gridDim.x * blockDim.x; }

}  // namespace pm
