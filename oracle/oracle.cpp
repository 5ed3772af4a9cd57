// CPU oracle: plain serial FP64 definition of the adaptation path.
// TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing); the HIP
// library never includes, links or calls this file.
//
// Built with g++ -O2 -ffp-contract=off so that every floating-point operation
// below is one IEEE-754 binary64 operation rounded to nearest.
//
// Paper sections followed (arXiv:1505.04694):
//   Sec. 2.2  element quality: the ideal element is equilateral with unit
//             edges in metric space (mean-ratio functional q = 4 sqrt(3) A_M / sum l_M^2)
//   Sec. 2.3  Algorithm 1: coarsen, swap, refine, then smooth
//   Sec. 2.4  the four kernels (collapse, split with templates, flip, smoothing)
//             and propagation to the neighbourhood until nothing changes
//   Sec. 3.1  hazards: topological hazards and adjacency-list races
//   Sec. 3.2  colouring: independent sets of the vertex graph, recoloured
//             after topology changes
//   Sec. 3.3  deferred update: one owner per adjacency list, committed after
//             every independent set
//   Sec. 3.4  worklists of touched items for the next sweep
// Readings of points the paper leaves open are listed beside each function.
//
// Pins: every rule here is checked by the CPU tests against closed forms, hand
// cases in exact arithmetic, and an independent re-derivation of each class
// member's decision. Parity unpinned: the strictness of the gradient
// smoother's two acceptance comparisons (patch minimum "not lower", patch sum
// "strictly higher"). They differ from their alternatives only when a
// continuous functional takes exactly equal values at two points of the
// search line, which no test case reaches; the HIP path takes the same
// comparisons.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <random>
#include <utility>
#include <vector>

namespace {

// the double nearest 4*sqrt(3) (4 * RN(sqrt 3) is exact scaling)
const double K4R3 = 6.928203230275509;
// the double nearest 12*sqrt(3)
const double K12R3 = 20.784609690826528;
const uint8_t TX0 = 1, TX1 = 2, TY0 = 4, TY1 = 8;
enum { PH_COARSEN = 1, PH_SWAP = 2, PH_SMOOTH = 3 };

using Tri = std::array<int32_t, 3>;

struct Mesh {
  int64_t V = 0, T = 0;
  std::vector<double> x, y, ma, mb, mc;
  std::vector<uint8_t> tag, valive;
  std::vector<Tri> tri;
  std::vector<uint8_t> talive;
  std::vector<std::vector<int32_t>> NN, NE;
  uint64_t seed = 0;
  orc_hook hook = nullptr;
  void* hook_user = nullptr;
  uint64_t order_seed = 0;
  std::vector<int32_t> cur_members;  // the class being processed, for the hook
  std::vector<int32_t> cur_class;    // the same class before re-validation
  // Algorithm 1's loop state: outer iteration, next phase, whether the
  // iteration has changed the mesh so far
  int32_t ad_iter = 0, ad_phase = ORC_PHASE_COARSEN, ad_changed = 0;
  // element quality functional: ORC_QUALITY_MEAN_RATIO or ORC_QUALITY_VASILEVSKII
  int32_t qk = ORC_QUALITY_MEAN_RATIO;
};

// ---- sorted-set rows ---------------------------------------------------------
void set_insert(std::vector<int32_t>& s, int32_t v) {
  auto it = std::lower_bound(s.begin(), s.end(), v);
  if (it == s.end() || *it != v) s.insert(it, v);
}
void set_erase(std::vector<int32_t>& s, int32_t v) {
  auto it = std::lower_bound(s.begin(), s.end(), v);
  if (it != s.end() && *it == v) s.erase(it);
}
bool set_has(const std::vector<int32_t>& s, int32_t v) {
  return std::binary_search(s.begin(), s.end(), v);
}

// counter-clockwise order kept, smallest id first
Tri canon(int32_t a, int32_t b, int32_t c) {
  if (a < b && a < c) return {a, b, c};
  if (b < a && b < c) return {b, c, a};
  return {c, a, b};
}
bool has_vertex(const Tri& t, int32_t v) { return t[0] == v || t[1] == v || t[2] == v; }

// NE(v) = live elements containing v; NN(v) = the other vertices of those
void rebuild_rows(Mesh& m) {
  m.NN.assign(m.V, {});
  m.NE.assign(m.V, {});
  for (int64_t t = 0; t < m.T; ++t) {
    if (!m.talive[t]) continue;
    for (int k = 0; k < 3; ++k) m.NE[m.tri[t][k]].push_back((int32_t)t);
  }
  for (int64_t v = 0; v < m.V; ++v) {
    std::vector<int32_t> nb;
    for (int32_t t : m.NE[v])
      for (int k = 0; k < 3; ++k)
        if (m.tri[t][k] != v) nb.push_back(m.tri[t][k]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    m.NN[v] = nb;
  }
}

// ---- metric geometry (Sec. 2.2) ---------------------------------------------
// Edge metric = mean of the two end-point tensors; element metric = mean of
// the three vertex tensors in the element's stored (canonical) order. The
// expression order written here is the definition used for every decision.

// squared metric length of edge i-j
double len2(const Mesh& m, int32_t i, int32_t j) {
  double a = (m.ma[i] + m.ma[j]) * 0.5;
  double b = (m.mb[i] + m.mb[j]) * 0.5;
  double c = (m.mc[i] + m.mc[j]) * 0.5;
  double dx = m.x[j] - m.x[i];
  double dy = m.y[j] - m.y[i];
  return ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
}

struct Geo {
  double x[3], y[3];
  double a, b, c;  // element metric
};

// geometry of element t (ids in stored order); vertex ov, if present, is placed at (ox, oy)
Geo geo(const Mesh& m, const Tri& t, int32_t ov = -1, double ox = 0.0, double oy = 0.0) {
  Geo g;
  for (int k = 0; k < 3; ++k) {
    int32_t v = t[k];
    if (v == ov) {
      g.x[k] = ox;
      g.y[k] = oy;
    } else {
      g.x[k] = m.x[v];
      g.y[k] = m.y[v];
    }
  }
  g.a = ((m.ma[t[0]] + m.ma[t[1]]) + m.ma[t[2]]) / 3.0;
  g.b = ((m.mb[t[0]] + m.mb[t[1]]) + m.mb[t[2]]) / 3.0;
  g.c = ((m.mc[t[0]] + m.mc[t[1]]) + m.mc[t[2]]) / 3.0;
  return g;
}

// twice the signed Euclidean area
double area2(const Geo& g) {
  return (g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]);
}

struct Parts {
  double D, A, S, det;
  double ex[3], ey[3];  // edge k runs from vertex k to vertex k+1
};

Parts parts(const Geo& g) {
  Parts p;
  p.D = area2(g);
  p.A = 0.5 * p.D;
  for (int k = 0; k < 3; ++k) {
    int k1 = (k + 1) % 3;
    p.ex[k] = g.x[k1] - g.x[k];
    p.ey[k] = g.y[k1] - g.y[k];
  }
  double l[3];
  for (int k = 0; k < 3; ++k)
    l[k] = ((g.a * p.ex[k]) * p.ex[k] + ((2.0 * g.b) * p.ex[k]) * p.ey[k]) + (g.c * p.ey[k]) * p.ey[k];
  p.S = (l[0] + l[1]) + l[2];
  p.det = g.a * g.c - g.b * g.b;
  return p;
}

// squared quality, used for every decision (no square root involved)
double qual2(const Geo& g) {
  Parts p = parts(g);
  return (((48.0 * p.det) * p.A) * p.A) / (p.S * p.S);
}

// reported quality q = 4 sqrt(3) sqrt(det M) A / S
double qual(const Geo& g) {
  Parts p = parts(g);
  return ((K4R3 * std::sqrt(p.det)) * p.A) / p.S;
}

// dq/d(x_k, y_k) for the vertex in position k of the element
void qual_grad_x(const Geo& g, int k, double* gx, double* gy) {
  Parts p = parts(g);
  double s = std::sqrt(p.det);
  int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
  double dAx = 0.5 * (g.y[k1] - g.y[k2]);
  double dAy = 0.5 * (g.x[k2] - g.x[k1]);
  // x_k enters edge k-1 (+) and edge k (-): dS/dx_k = 2 M (e_{k-1} - e_k)
  double ux = p.ex[k2] - p.ex[k];
  double uy = p.ey[k2] - p.ey[k];
  double dSx = 2.0 * (g.a * ux + g.b * uy);
  double dSy = 2.0 * (g.b * ux + g.c * uy);
  double Ks = K4R3 * s;
  double SS = p.S * p.S;
  *gx = (Ks * (dAx * p.S - p.A * dSx)) / SS;
  *gy = (Ks * (dAy * p.S - p.A * dSy)) / SS;
}

// dq/d(element metric entries a, b, c); b is the stored off-diagonal entry
void qual_grad_m(const Geo& g, double* da, double* db, double* dc) {
  Parts p = parts(g);
  double s = std::sqrt(p.det);
  double Sxx = (p.ex[0] * p.ex[0] + p.ex[1] * p.ex[1]) + p.ex[2] * p.ex[2];
  double Sxy = (p.ex[0] * p.ey[0] + p.ex[1] * p.ey[1]) + p.ex[2] * p.ey[2];
  double Syy = (p.ey[0] * p.ey[0] + p.ey[1] * p.ey[1]) + p.ey[2] * p.ey[2];
  double KA = K4R3 * p.A;
  double SS = p.S * p.S;
  *da = (KA * ((g.c * p.S) / (2.0 * s) - s * Sxx)) / SS;
  *db = (KA * (-(g.b * p.S) / s - (2.0 * s) * Sxy)) / SS;
  *dc = (KA * ((g.a * p.S) / (2.0 * s) - s * Syy)) / SS;
}

// ---- Vasilevskii's functional with its size factor (Sec. 2.2) ---------------
// Q_V = 12 sqrt(3) |K|_M / P^2 * F(P / 3), P the perimeter in the metric (sum
// of the three edge lengths in the element metric), |K|_M = sqrt(det M) A, and
// F(x) = (m (2 - m))^3 with m = min(x, 1/x). Q_V = 1 exactly for the
// equilateral triangle with unit metric edges; F penalises any other size.
// Decisions compare Q_V^2 (the product rounded once) with q_min^2, as the mean
// ratio's decisions compare q^2.
struct VParts {
  double A, s, P;
  double L[3], ex[3], ey[3];
};

VParts vparts(const Geo& g) {
  VParts v;
  v.A = 0.5 * area2(g);
  for (int k = 0; k < 3; ++k) {
    int k1 = (k + 1) % 3;
    v.ex[k] = g.x[k1] - g.x[k];
    v.ey[k] = g.y[k1] - g.y[k];
  }
  for (int k = 0; k < 3; ++k)
    v.L[k] = std::sqrt(((g.a * v.ex[k]) * v.ex[k] + ((2.0 * g.b) * v.ex[k]) * v.ey[k]) + (g.c * v.ey[k]) * v.ey[k]);
  v.P = (v.L[0] + v.L[1]) + v.L[2];
  v.s = std::sqrt(g.a * g.c - g.b * g.b);
  return v;
}

// size factor F at x = P / 3 and the derivative of G(P) = F(P/3) / P^2
void vas_size(double P, double* G, double* dG) {
  double x = P / 3.0;
  bool below = x < 1.0;
  double mm = below ? x : 1.0 / x;
  double f = mm * (2.0 - mm);
  double F = (f * f) * f;
  double dm = below ? 1.0 : -1.0 / (x * x);
  double dF = ((3.0 * (f * f)) * (2.0 - 2.0 * mm)) * dm;
  double P2 = P * P;
  *G = F / P2;
  *dG = dF / (3.0 * P2) - (2.0 * F) / (P2 * P);
}

double qual_vas(const Geo& g) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, &G, &dG);
  return ((K12R3 * v.s) * v.A) * G;
}

void vas_grad_x(const Geo& g, int k, double* gx, double* gy) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, &G, &dG);
  int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
  double dAx = 0.5 * (g.y[k1] - g.y[k2]);
  double dAy = 0.5 * (g.x[k2] - g.x[k1]);
  // x_k ends edge k-1 and starts edge k: dP/dx_k = M e_{k-1} / L_{k-1} - M e_k / L_k
  double dPx = (g.a * v.ex[k2] + g.b * v.ey[k2]) / v.L[k2] - (g.a * v.ex[k] + g.b * v.ey[k]) / v.L[k];
  double dPy = (g.b * v.ex[k2] + g.c * v.ey[k2]) / v.L[k2] - (g.b * v.ex[k] + g.c * v.ey[k]) / v.L[k];
  double Ks = K12R3 * v.s;
  *gx = Ks * (dAx * G + (v.A * dG) * dPx);
  *gy = Ks * (dAy * G + (v.A * dG) * dPy);
}

void vas_grad_m(const Geo& g, double* da, double* db, double* dc) {
  VParts v = vparts(g);
  double G, dG;
  vas_size(v.P, &G, &dG);
  double Pa = 0.0, Pb = 0.0, Pc = 0.0;
  for (int j = 0; j < 3; ++j) {
    Pa = Pa + (v.ex[j] * v.ex[j]) / (2.0 * v.L[j]);
    Pb = Pb + (v.ex[j] * v.ey[j]) / v.L[j];
    Pc = Pc + (v.ey[j] * v.ey[j]) / (2.0 * v.L[j]);
  }
  double KA = K12R3 * v.A;
  *da = KA * ((g.c / (2.0 * v.s)) * G + (v.s * dG) * Pa);
  *db = KA * (-(g.b / v.s) * G + (v.s * dG) * Pb);
  *dc = KA * ((g.a / (2.0 * v.s)) * G + (v.s * dG) * Pc);
}

// the handle's functional: value used by decisions (squared), reported value,
// and its derivatives
double dq2(const Mesh& m, const Geo& g) {
  if (m.qk == ORC_QUALITY_VASILEVSKII) {
    double q = qual_vas(g);
    return q * q;
  }
  return qual2(g);
}
double qval(const Mesh& m, const Geo& g) { return m.qk == ORC_QUALITY_VASILEVSKII ? qual_vas(g) : qual(g); }
void qgrad_x(const Mesh& m, const Geo& g, int k, double* gx, double* gy) {
  if (m.qk == ORC_QUALITY_VASILEVSKII)
    vas_grad_x(g, k, gx, gy);
  else
    qual_grad_x(g, k, gx, gy);
}
void qgrad_m(const Mesh& m, const Geo& g, double* da, double* db, double* dc) {
  if (m.qk == ORC_QUALITY_VASILEVSKII)
    vas_grad_m(g, da, db, dc);
  else
    qual_grad_m(g, da, db, dc);
}

int pos_in(const Tri& t, int32_t v) { return t[0] == v ? 0 : (t[1] == v ? 1 : 2); }

// ---- priorities (Sec. 3.2: colouring from random priorities) ----------------
const uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
uint64_t splitmix_at(uint64_t s, uint64_t i) { return mix64(s + (i + 1) * GAMMA); }
uint32_t prio(uint64_t seed, uint32_t ctx, uint32_t id) {
  uint64_t stream = splitmix_at(seed ^ ((uint64_t)ctx << 32), 0);
  return (uint32_t)(splitmix_at(stream, id) >> 32);
}
uint32_t make_ctx(int sweep, int phase, int round) {
  return ((uint32_t)sweep << 20) | ((uint32_t)phase << 16) | (uint32_t)round;
}
// key order: (priority, id) lexicographic, larger wins
bool key_greater(uint32_t pa, int32_t a, uint32_t pb, int32_t b) {
  return pa != pb ? pa > pb : a > b;
}

// ---- colouring (Sec. 3.2) -----------------------------------------------------
// Reading: Jones-Plassmann with first-fit colours, whose result is exactly the
// sequential greedy colouring of the active-induced subgraph taken in
// descending key order; that greedy order is what is written here.
int32_t colour(const Mesh& m, const std::vector<int32_t>& A, uint32_t ctx, std::vector<int32_t>& col) {
  col.assign(m.V, -1);
  std::vector<std::pair<uint32_t, int32_t>> order;
  order.reserve(A.size());
  for (int32_t v : A) order.push_back({prio(m.seed, ctx, (uint32_t)v), v});
  std::sort(order.begin(), order.end(), [](const auto& p, const auto& q) {
    return key_greater(p.first, p.second, q.first, q.second);
  });
  int32_t ncol = 0;
  std::vector<char> used;
  for (auto& pv : order) {
    int32_t v = pv.second;
    used.assign(m.NN[v].size() + 2, 0);
    for (int32_t w : m.NN[v]) {
      int32_t c = col[w];
      if (c >= 0 && c < (int32_t)used.size()) used[c] = 1;
    }
    int32_t c = 0;
    while (used[c]) ++c;
    col[v] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// Sec. 3.2 re-colours after topology changes; several classes share one
// colouring, so before a class runs, a member adjacent in the current graph
// to a same-class member with a larger key is deferred to the next round.
void revalidate(const Mesh& m, const std::vector<int32_t>& members, const std::vector<int32_t>& col,
                int32_t c, uint32_t ctx, std::vector<int32_t>& kept, std::vector<int32_t>& deferred) {
  kept.clear();
  deferred.clear();
  for (int32_t v : members) {
    uint32_t pv = prio(m.seed, ctx, (uint32_t)v);
    bool beaten = false;
    for (int32_t w : m.NN[v])
      if (col[w] == c && key_greater(prio(m.seed, ctx, (uint32_t)w), w, pv, v)) {
        beaten = true;
        break;
      }
    (beaten ? deferred : kept).push_back(v);
  }
}

void shuffle_members(Mesh& m, std::vector<int32_t>& v, uint64_t salt) {
  if (!m.order_seed) return;
  std::mt19937_64 rng(m.order_seed * 1000003ULL + salt);
  std::shuffle(v.begin(), v.end(), rng);
}

void run_hook(Mesh& m, int phase, int round, int cls, int stage, const std::vector<int32_t>& members,
              const std::vector<int32_t>& whole) {
  if (!m.hook) return;
  m.cur_members = members;
  m.cur_class = whole;
  m.hook(m.hook_user, phase, round, cls, stage);
}

std::vector<std::vector<int32_t>> classes_of(const std::vector<int32_t>& A, const std::vector<int32_t>& col,
                                             int32_t ncol) {
  std::vector<std::vector<int32_t>> cls(ncol);
  for (int32_t v : A) cls[col[v]].push_back(v);  // A is ascending, so each class is too
  return cls;
}

// ---- coarsening (Sec. 2.4.1) ---------------------------------------------------
// Reading: v may collapse onto a neighbour u when the edge is short
// (L^2 < L_low^2) and u lies on every boundary side v lies on (corners never
// move; side vertices move only along their side). Candidates are tried in
// ascending (L^2, u); the first one whose re-pointed elements all keep a
// positive area and quality >= q_min is taken.
bool tag_ok(const Mesh& m, int32_t v, int32_t u) { return (m.tag[v] & ~m.tag[u]) == 0; }

bool has_candidate(const Mesh& m, int32_t v, double L_low2) {
  for (int32_t u : m.NN[v])
    if (tag_ok(m, v, u) && len2(m, v, u) < L_low2) return true;
  return false;
}

int32_t eval_collapse(const Mesh& m, int32_t v, double L_low2, double qmin2) {
  std::vector<std::pair<double, int32_t>> cand;
  for (int32_t u : m.NN[v]) {
    if (!tag_ok(m, v, u)) continue;
    double L2 = len2(m, v, u);
    if (L2 < L_low2) cand.push_back({L2, u});
  }
  std::sort(cand.begin(), cand.end());
  for (auto& cu : cand) {
    int32_t u = cu.second;
    bool ok = true;
    for (int32_t t : m.NE[v]) {
      const Tri& e = m.tri[t];
      if (has_vertex(e, u)) continue;  // removed with the edge
      Tri r = e;
      r[pos_in(e, v)] = u;
      Tri rc = canon(r[0], r[1], r[2]);
      Geo g = geo(m, rc);
      if (!(area2(g) > 0.0) || !(dq2(m, g) >= qmin2)) {
        ok = false;
        break;
      }
    }
    if (ok) return u;
  }
  return -1;
}

void apply_collapse(Mesh& m, int32_t v, int32_t u) {
  std::vector<int32_t> nv = m.NN[v], ne = m.NE[v];
  for (int32_t t : ne) {
    Tri& e = m.tri[t];
    if (has_vertex(e, u)) {
      m.talive[t] = 0;
      for (int k = 0; k < 3; ++k)
        if (e[k] != v) set_erase(m.NE[e[k]], t);
    } else {
      e[pos_in(e, v)] = u;
      e = canon(e[0], e[1], e[2]);
      set_insert(m.NE[u], t);
    }
  }
  for (int32_t w : nv) {
    set_erase(m.NN[w], v);
    if (w != u) {
      set_insert(m.NN[w], u);
      set_insert(m.NN[u], w);
    }
  }
  m.NN[v].clear();
  m.NE[v].clear();
  m.valive[v] = 0;
}

// ---- swapping (Sec. 2.4.3) -------------------------------------------------------
// Reading: member v looks at every interior edge (v, w); the flip replaces
// (v,w,a), (w,v,b) by (v,b,a), (w,a,b), is valid when both new areas are
// positive, and is wanted when the smaller new quality beats the smaller old
// one strictly. The best new minimum wins, ties to the smaller w. The new
// element holding v keeps the smaller of the two element ids.
struct Flip {
  int32_t w, T1, T2, a, b;
  double newmin;
};

bool eval_flip(const Mesh& m, int32_t v, Flip& best) {
  bool found = false;
  for (int32_t w : m.NN[v]) {
    int32_t T1 = -1, T2 = -1;
    for (int32_t t : m.NE[v]) {
      const Tri& e = m.tri[t];
      int k = pos_in(e, v);
      if (e[(k + 1) % 3] == w) T1 = t;       // edge runs v -> w
      else if (e[(k + 2) % 3] == w) T2 = t;  // edge runs w -> v
    }
    if (T1 < 0 || T2 < 0) continue;  // boundary edge
    const Tri& e1 = m.tri[T1];
    const Tri& e2 = m.tri[T2];
    int32_t a = e1[(pos_in(e1, v) + 2) % 3];
    int32_t b = e2[(pos_in(e2, v) + 1) % 3];
    Tri tv = canon(v, b, a), tw = canon(w, a, b);
    Geo gv = geo(m, tv), gw = geo(m, tw);
    if (!(area2(gv) > 0.0) || !(area2(gw) > 0.0)) continue;
    double qv = dq2(m, gv), qw = dq2(m, gw);
    double q1 = dq2(m, geo(m, e1)), q2 = dq2(m, geo(m, e2));
    double nmin = qw < qv ? qw : qv;
    double omin = q2 < q1 ? q2 : q1;
    if (!(nmin > omin)) continue;
    if (!found || nmin > best.newmin) {
      best = Flip{w, T1, T2, a, b, nmin};
      found = true;
    }
  }
  return found;
}

bool apply_flip(Mesh& m, int32_t v, const Flip& f) {
  if (set_has(m.NN[f.a], f.b)) return false;  // impossible for a valid mesh
  int32_t lo = std::min(f.T1, f.T2), hi = std::max(f.T1, f.T2);
  m.tri[lo] = canon(v, f.b, f.a);
  m.tri[hi] = canon(f.w, f.a, f.b);
  set_erase(m.NN[v], f.w);
  set_erase(m.NN[f.w], v);
  set_insert(m.NN[f.a], f.b);
  set_insert(m.NN[f.b], f.a);
  set_erase(m.NE[v], hi);
  set_erase(m.NE[f.w], lo);
  set_insert(m.NE[f.a], f.T2);
  set_insert(m.NE[f.b], f.T1);
  return true;
}

// ---- smoothing (Sec. 2.4.4) --------------------------------------------------------
// Reading: the metric travels with the vertex. A move is kept when every
// element around v keeps a positive area and the smallest q^2 around v does
// not drop.
double patch_min_q2(const Mesh& m, int32_t v, double px, double py, bool& valid) {
  valid = true;
  double mn = 0.0;
  bool first = true;
  for (int32_t t : m.NE[v]) {
    Geo g = geo(m, m.tri[t], v, px, py);
    if (!(area2(g) > 0.0)) valid = false;
    double q2 = dq2(m, g);
    if (first || q2 < mn) mn = q2;
    first = false;
  }
  return mn;
}

double patch_q(const Mesh& m, int32_t v, double px, double py) {
  double s = 0.0;
  for (int32_t t : m.NE[v]) s = s + qval(m, geo(m, m.tri[t], v, px, py));
  return s;
}

// Laplacian in the metric: the point p minimising sum_j (x_j - p)^T M_vj (x_j - p)
bool smooth_laplace(Mesh& m, int32_t v) {
  double Ga = 0.0, Gb = 0.0, Gc = 0.0, rx = 0.0, ry = 0.0;
  double xv = m.x[v], yv = m.y[v];
  for (int32_t j : m.NN[v]) {
    double ea = (m.ma[v] + m.ma[j]) * 0.5;
    double eb = (m.mb[v] + m.mb[j]) * 0.5;
    double ec = (m.mc[v] + m.mc[j]) * 0.5;
    double dx = m.x[j] - xv, dy = m.y[j] - yv;
    Ga = Ga + ea;
    Gb = Gb + eb;
    Gc = Gc + ec;
    rx = rx + (ea * dx + eb * dy);
    ry = ry + (eb * dx + ec * dy);
  }
  double det = Ga * Gc - Gb * Gb;
  double px = xv + (Gc * rx - Gb * ry) / det;
  double py = yv + (Ga * ry - Gb * rx) / det;
  bool vo, vn;
  double oldmin = patch_min_q2(m, v, xv, yv, vo);
  double newmin = patch_min_q2(m, v, px, py, vn);
  if (vn && newmin >= oldmin) {
    m.x[v] = px;
    m.y[v] = py;
    return true;
  }
  return false;
}

// Gradient step on the local functional Q_v = sum over the elements of v of q,
// direction normalised in the max-norm, step h/2, h/4, h/8, h/16 with h the
// smallest max-norm distance to a neighbour.
bool smooth_gradient(Mesh& m, int32_t v) {
  double xv = m.x[v], yv = m.y[v];
  double gx = 0.0, gy = 0.0;
  for (int32_t t : m.NE[v]) {
    const Tri& e = m.tri[t];
    double ex, ey;
    qgrad_x(m, geo(m, e), pos_in(e, v), &ex, &ey);
    gx = gx + ex;
    gy = gy + ey;
  }
  if (gx == 0.0 && gy == 0.0) return false;
  double ax = std::fabs(gx), ay = std::fabs(gy);
  double nrm = ax < ay ? ay : ax;
  double dx = gx / nrm, dy = gy / nrm;
  double h = 0.0;
  bool first = true;
  for (int32_t j : m.NN[v]) {
    double hx = std::fabs(m.x[j] - xv), hy = std::fabs(m.y[j] - yv);
    double hj = hx < hy ? hy : hx;
    if (first || hj < h) h = hj;
    first = false;
  }
  bool vo;
  double oldmin = patch_min_q2(m, v, xv, yv, vo);
  double Qold = patch_q(m, v, xv, yv);
  double step = h;
  for (int k = 1; k <= 4; ++k) {
    step = step * 0.5;
    double px = xv + step * dx, py = yv + step * dy;
    bool vn;
    double newmin = patch_min_q2(m, v, px, py, vn);
    if (!vn || !(newmin >= oldmin)) continue;
    if (!(patch_q(m, v, px, py) > Qold)) continue;
    m.x[v] = px;
    m.y[v] = py;
    return true;
  }
  return false;
}

// Min-max optimisation smoothing (Sec. 2.4.4 cites optimisation-based
// smoothing, which aims at the worst element). Reading: ascent on the
// patch's minimum quality. The worst element is the one of smallest q
// (ties: the first in NE(v), ascending ids), the second worst likewise among
// the rest. Direction: the gradient of the worst element's q in x_v; when the
// second worst is within 1% (q2 <= 1.01 q1), the point nearest the origin on
// the segment between the two gradients (the ascent direction of the smaller
// of the two). Normalised in the max-norm; steps h/2 .. h/16 with h as in the
// gradient step; the first step that keeps every area positive and raises
// the patch minimum of q^2 strictly is taken.
bool smooth_minmax(Mesh& m, int32_t v) {
  double xv = m.x[v], yv = m.y[v];
  int32_t t1 = -1, t2 = -1;
  double q1 = 0.0, q2 = 0.0;
  for (int32_t t : m.NE[v]) {
    double q = qval(m, geo(m, m.tri[t]));
    if (t1 < 0 || q < q1) {
      t2 = t1;
      q2 = q1;
      t1 = t;
      q1 = q;
    } else if (t2 < 0 || q < q2) {
      t2 = t;
      q2 = q;
    }
  }
  if (t1 < 0) return false;
  double ax, ay;
  qgrad_x(m, geo(m, m.tri[t1]), pos_in(m.tri[t1], v), &ax, &ay);
  double gx = ax, gy = ay;
  if (t2 >= 0 && q2 <= q1 * 1.01) {
    double bx, by;
    qgrad_x(m, geo(m, m.tri[t2]), pos_in(m.tri[t2], v), &bx, &by);
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
  double nx = std::fabs(gx), ny = std::fabs(gy);
  double nrm = nx < ny ? ny : nx;
  double dx = gx / nrm, dy = gy / nrm;
  double h = 0.0;
  bool first = true;
  for (int32_t j : m.NN[v]) {
    double hx = std::fabs(m.x[j] - xv), hy = std::fabs(m.y[j] - yv);
    double hj = hx < hy ? hy : hx;
    if (first || hj < h) h = hj;
    first = false;
  }
  bool vo;
  double oldmin = patch_min_q2(m, v, xv, yv, vo);
  double step = h;
  for (int k = 1; k <= 4; ++k) {
    step = step * 0.5;
    double px = xv + step * dx, py = yv + step * dy;
    bool vn;
    double newmin = patch_min_q2(m, v, px, py, vn);
    if (!vn || !(newmin > oldmin)) continue;
    m.x[v] = px;
    m.y[v] = py;
    return true;
  }
  return false;
}

}  // namespace

struct orc_mesh : Mesh {};

extern "C" {

uint64_t orc_splitmix(uint64_t s, uint64_t i) { return splitmix_at(s, i); }
uint32_t orc_prio(uint64_t seed, uint32_t ctx, uint32_t id) { return prio(seed, ctx, id); }

orc_mesh* orc_create(int64_t V, int64_t T, const double* xy, const int32_t* tri, const double* metric,
                     const uint8_t* tags, uint64_t seed) {
  if (V <= 0 || T <= 0 || !xy || !tri || !metric) return nullptr;
  orc_mesh* m = new orc_mesh();
  m->V = V;
  m->T = T;
  m->seed = seed;
  m->x.resize(V);
  m->y.resize(V);
  m->ma.resize(V);
  m->mb.resize(V);
  m->mc.resize(V);
  m->tag.resize(V);
  m->valive.assign(V, 1);
  for (int64_t v = 0; v < V; ++v) {
    m->x[v] = xy[2 * v];
    m->y[v] = xy[2 * v + 1];
    m->ma[v] = metric[3 * v];
    m->mb[v] = metric[3 * v + 1];
    m->mc[v] = metric[3 * v + 2];
    if (!(m->ma[v] > 0.0) || !(m->ma[v] * m->mc[v] - m->mb[v] * m->mb[v] > 0.0)) {
      delete m;
      return nullptr;
    }
    if (tags) {
      m->tag[v] = tags[v];
    } else {
      uint8_t t = 0;
      if (m->x[v] == 0.0) t |= TX0;
      if (m->x[v] == 1.0) t |= TX1;
      if (m->y[v] == 0.0) t |= TY0;
      if (m->y[v] == 1.0) t |= TY1;
      m->tag[v] = t;
    }
  }
  m->tri.resize(T);
  m->talive.assign(T, 1);
  for (int64_t t = 0; t < T; ++t) {
    int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= V || b >= V || c >= V || a == b || b == c || a == c) {
      delete m;
      return nullptr;
    }
    m->tri[t] = canon(a, b, c);
    if (!(area2(geo(*m, m->tri[t])) > 0.0)) {
      delete m;
      return nullptr;
    }
  }
  rebuild_rows(*m);
  return m;
}

void orc_destroy(orc_mesh* m) { delete m; }

void orc_sizes(const orc_mesh* m, int64_t* V, int64_t* T) {
  if (V) *V = m->V;
  if (T) *T = m->T;
}

void orc_export(const orc_mesh* m, double* xy, int32_t* tri, double* metric, uint8_t* tags, uint8_t* valive,
                uint8_t* talive) {
  for (int64_t v = 0; v < m->V; ++v) {
    if (xy) {
      xy[2 * v] = m->x[v];
      xy[2 * v + 1] = m->y[v];
    }
    if (metric) {
      metric[3 * v] = m->ma[v];
      metric[3 * v + 1] = m->mb[v];
      metric[3 * v + 2] = m->mc[v];
    }
    if (tags) tags[v] = m->tag[v];
    if (valive) valive[v] = m->valive[v];
  }
  for (int64_t t = 0; t < m->T; ++t) {
    if (tri)
      for (int k = 0; k < 3; ++k) tri[3 * t + k] = m->tri[t][k];
    if (talive) talive[t] = m->talive[t];
  }
}

void orc_row_totals(const orc_mesh* m, int64_t* nn_total, int64_t* ne_total) {
  int64_t a = 0, b = 0;
  for (int64_t v = 0; v < m->V; ++v) {
    a += (int64_t)m->NN[v].size();
    b += (int64_t)m->NE[v].size();
  }
  *nn_total = a;
  *ne_total = b;
}

void orc_export_rows(const orc_mesh* m, int64_t* nn_off, int32_t* nn, int64_t* ne_off, int32_t* ne) {
  int64_t a = 0, b = 0;
  for (int64_t v = 0; v < m->V; ++v) {
    nn_off[v] = a;
    ne_off[v] = b;
    for (int32_t w : m->NN[v]) nn[a++] = w;
    for (int32_t t : m->NE[v]) ne[b++] = t;
  }
  nn_off[m->V] = a;
  ne_off[m->V] = b;
}

void orc_set_xy(orc_mesh* m, int32_t v, double x, double y) {
  m->x[v] = x;
  m->y[v] = y;
}
void orc_set_metric(orc_mesh* m, int32_t v, double a, double b, double c) {
  m->ma[v] = a;
  m->mb[v] = b;
  m->mc[v] = c;
}
void orc_set_hook(orc_mesh* m, orc_hook hook, void* user) {
  m->hook = hook;
  m->hook_user = user;
}
void orc_set_order_seed(orc_mesh* m, uint64_t s) { m->order_seed = s; }
int32_t orc_set_quality(orc_mesh* m, int32_t kind) {
  if (kind != ORC_QUALITY_MEAN_RATIO && kind != ORC_QUALITY_VASILEVSKII) return -1;
  m->qk = kind;
  return 0;
}
int64_t orc_class_members(const orc_mesh* m, int32_t* out, int64_t cap) {
  int64_t n = (int64_t)m->cur_members.size();
  for (int64_t i = 0; i < n && i < cap; ++i) out[i] = m->cur_members[i];
  return n;
}
int64_t orc_class_whole(const orc_mesh* m, int32_t* out, int64_t cap) {
  int64_t n = (int64_t)m->cur_class.size();
  for (int64_t i = 0; i < n && i < cap; ++i) out[i] = m->cur_class[i];
  return n;
}

int32_t orc_colour(orc_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out) {
  std::vector<int32_t> A;
  for (int64_t v = 0; v < m->V; ++v)
    if (m->valive[v] && (!active || active[v])) A.push_back((int32_t)v);
  std::vector<int32_t> col;
  int32_t n = colour(*m, A, ctx, col);
  if (colour_out)
    for (int64_t v = 0; v < m->V; ++v) colour_out[v] = col[v];
  return n;
}

int32_t orc_coarsen(orc_mesh* mp, int32_t sweep, double L_low2, double q_min, int32_t max_rounds,
                    int64_t* st) {
  Mesh& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  double qmin2 = q_min * q_min;
  std::vector<int32_t> A;
  for (int64_t v = 0; v < m.V; ++v)
    if (m.valive[v] && has_candidate(m, (int32_t)v, L_low2)) A.push_back((int32_t)v);
  int32_t r = 0;
  std::vector<int32_t> col, kept, deferred;
  std::vector<char> next(m.V, 0);
  while (!A.empty() && r < max_rounds) {
    uint32_t ctx = make_ctx(sweep, PH_COARSEN, r);
    int32_t ncol = colour(m, A, ctx, col);
    st[ORC_COLOURED] += (int64_t)A.size();
    st[ORC_COLOURS] += ncol;
    auto cls = classes_of(A, col, ncol);
    for (int32_t c = 0; c < ncol; ++c) {
      revalidate(m, cls[c], col, c, ctx, kept, deferred);
      st[ORC_DEFERRED] += (int64_t)deferred.size();
      st[ORC_EVALUATED] += (int64_t)kept.size();
      for (int32_t v : deferred) next[v] = 1;
      shuffle_members(m, kept, ((uint64_t)r << 16) | (uint64_t)c);
      run_hook(m, PH_COARSEN, r, c, 0, kept, cls[c]);
      for (int32_t v : kept) {
        int32_t u = eval_collapse(m, v, L_low2, qmin2);
        if (u < 0) continue;
        for (int32_t w : m.NN[v]) next[w] = 1;  // includes u
        apply_collapse(m, v, u);
        st[ORC_COMMITTED] += 1;
      }
      run_hook(m, PH_COARSEN, r, c, 1, kept, cls[c]);
    }
    A.clear();
    for (int64_t v = 0; v < m.V; ++v) {
      if (next[v] && m.valive[v] && has_candidate(m, (int32_t)v, L_low2)) A.push_back((int32_t)v);
      next[v] = 0;
    }
    ++r;
  }
  st[ORC_ROUNDS] = r;
  st[ORC_CONVERGED] = A.empty() ? 1 : 0;
  orc_compact(mp);
  return A.empty() ? 0 : 1;
}

// ---- refinement (Sec. 2.4.2) --------------------------------------------------------
// Reading: all long edges (L^2 > L_up^2) split at once each pass, elements cut
// by templates (1, 2 or 3 split edges); each element depends only on its own
// edges, so no colouring is needed. New vertex ids follow the (min id, max id)
// order of the split edges; the first child keeps the parent id and the other
// children take new ids in parent order. A two-split element cuts its quad
// along the metric-shorter diagonal (ties: the diagonal through the first
// vertex of the unsplit edge).
int32_t orc_refine(orc_mesh* mp, double L_up2, int32_t max_passes, int64_t* st) {
  Mesh& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  int32_t p = 0;
  bool done = false;
  for (; p < max_passes; ++p) {
    std::vector<std::pair<int32_t, int32_t>> marked;
    for (int64_t a = 0; a < m.V; ++a) {
      if (!m.valive[a]) continue;
      for (int32_t b : m.NN[a]) {
        if (b <= a) continue;
        st[ORC_EDGES] += 1;
        if (len2(m, (int32_t)a, b) > L_up2) marked.push_back({(int32_t)a, b});
      }
    }
    if (marked.empty()) {
      done = true;
      break;
    }
    std::map<std::pair<int32_t, int32_t>, int32_t> mid;
    int64_t V0 = m.V;
    for (auto& e : marked) {
      int32_t a = e.first, b = e.second;
      int32_t id = (int32_t)m.V++;
      mid[e] = id;
      m.x.push_back((m.x[a] + m.x[b]) * 0.5);
      m.y.push_back((m.y[a] + m.y[b]) * 0.5);
      m.ma.push_back((m.ma[a] + m.ma[b]) * 0.5);
      m.mb.push_back((m.mb[a] + m.mb[b]) * 0.5);
      m.mc.push_back((m.mc[a] + m.mc[b]) * 0.5);
      m.tag.push_back(m.tag[a] & m.tag[b]);
      m.valive.push_back(1);
    }
    st[ORC_NEWV] += m.V - V0;
    st[ORC_COMMITTED] += (int64_t)marked.size();
    auto midpoint = [&](int32_t a, int32_t b) -> int32_t {
      auto it = mid.find({std::min(a, b), std::max(a, b)});
      return it == mid.end() ? -1 : it->second;
    };
    int64_t T0 = m.T;
    for (int64_t t = 0; t < T0; ++t) {
      if (!m.talive[t]) continue;
      Tri e = m.tri[t];
      int32_t mm[3];
      int ns = 0;
      for (int k = 0; k < 3; ++k) {
        mm[k] = midpoint(e[k], e[(k + 1) % 3]);
        ns += mm[k] >= 0;
      }
      if (ns == 0) continue;
      std::vector<Tri> ch;
      if (ns == 1) {
        int k = mm[0] >= 0 ? 0 : (mm[1] >= 0 ? 1 : 2);
        int32_t P = e[k], Q = e[(k + 1) % 3], R = e[(k + 2) % 3], M = mm[k];
        ch.push_back({P, M, R});
        ch.push_back({M, Q, R});
      } else if (ns == 2) {
        int k = mm[0] < 0 ? 0 : (mm[1] < 0 ? 1 : 2);  // the unsplit edge
        int32_t P = e[k], Q = e[(k + 1) % 3], R = e[(k + 2) % 3];
        int32_t M1 = mm[(k + 1) % 3], M2 = mm[(k + 2) % 3];  // on Q-R and R-P
        ch.push_back({M1, R, M2});
        double dP = len2(m, P, M1), dQ = len2(m, Q, M2);
        if (dP <= dQ) {
          ch.push_back({P, Q, M1});
          ch.push_back({P, M1, M2});
        } else {
          ch.push_back({P, Q, M2});
          ch.push_back({Q, M1, M2});
        }
      } else {
        ch.push_back({e[0], mm[0], mm[2]});
        ch.push_back({mm[0], e[1], mm[1]});
        ch.push_back({mm[2], mm[1], e[2]});
        ch.push_back({mm[0], mm[1], mm[2]});
      }
      m.tri[t] = canon(ch[0][0], ch[0][1], ch[0][2]);
      for (size_t i = 1; i < ch.size(); ++i) {
        m.tri.push_back(canon(ch[i][0], ch[i][1], ch[i][2]));
        m.talive.push_back(1);
        m.T++;
      }
    }
    st[ORC_NEWT] += m.T - T0;
    rebuild_rows(m);
  }
  st[ORC_ROUNDS] = p;
  st[ORC_CONVERGED] = done ? 1 : 0;
  return done ? 0 : 1;
}

int32_t orc_swap(orc_mesh* mp, int32_t sweep, int32_t max_rounds, int64_t* st) {
  Mesh& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  std::vector<int32_t> A;
  for (int64_t v = 0; v < m.V; ++v)
    if (m.valive[v]) A.push_back((int32_t)v);
  int32_t r = 0;
  std::vector<int32_t> col, kept, deferred;
  std::vector<char> next(m.V, 0);
  while (!A.empty() && r < max_rounds) {
    uint32_t ctx = make_ctx(sweep, PH_SWAP, r);
    int32_t ncol = colour(m, A, ctx, col);
    st[ORC_COLOURED] += (int64_t)A.size();
    st[ORC_COLOURS] += ncol;
    auto cls = classes_of(A, col, ncol);
    for (int32_t c = 0; c < ncol; ++c) {
      revalidate(m, cls[c], col, c, ctx, kept, deferred);
      st[ORC_DEFERRED] += (int64_t)deferred.size();
      st[ORC_EVALUATED] += (int64_t)kept.size();
      for (int32_t v : deferred) next[v] = 1;
      shuffle_members(m, kept, ((uint64_t)r << 16) | (uint64_t)c);
      run_hook(m, PH_SWAP, r, c, 0, kept, cls[c]);
      for (int32_t v : kept) {
        Flip f;
        if (!eval_flip(m, v, f)) continue;
        if (!apply_flip(m, v, f)) return -2;
        next[v] = next[f.w] = next[f.a] = next[f.b] = 1;
        st[ORC_COMMITTED] += 1;
      }
      run_hook(m, PH_SWAP, r, c, 1, kept, cls[c]);
    }
    A.clear();
    for (int64_t v = 0; v < m.V; ++v) {
      if (next[v] && m.valive[v]) A.push_back((int32_t)v);
      next[v] = 0;
    }
    ++r;
  }
  st[ORC_ROUNDS] = r;
  st[ORC_CONVERGED] = A.empty() ? 1 : 0;
  return A.empty() ? 0 : 1;
}

int32_t orc_smooth(orc_mesh* mp, int32_t sweep, int32_t kind, int32_t sweeps, int64_t* st) {
  Mesh& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  std::vector<int32_t> A;
  for (int64_t v = 0; v < m.V; ++v)
    if (m.valive[v] && m.tag[v] == 0) A.push_back((int32_t)v);
  std::vector<int32_t> col;
  uint32_t ctx = make_ctx(sweep, PH_SMOOTH, 0);
  int32_t ncol = colour(m, A, ctx, col);
  st[ORC_COLOURED] += (int64_t)A.size();
  st[ORC_COLOURS] += ncol;
  auto cls = classes_of(A, col, ncol);
  for (int32_t s = 0; s < sweeps; ++s) {
    for (int32_t c = 0; c < ncol; ++c) {
      std::vector<int32_t> mem = cls[c];
      shuffle_members(m, mem, ((uint64_t)s << 16) | (uint64_t)c);
      run_hook(m, PH_SMOOTH, s, c, 0, mem, cls[c]);
      for (int32_t v : mem) {
        st[ORC_EVALUATED] += 1;
        bool moved = kind == 0 ? smooth_laplace(m, v) : (kind == 1 ? smooth_gradient(m, v) : smooth_minmax(m, v));
        st[ORC_COMMITTED] += moved ? 1 : 0;
      }
      run_hook(m, PH_SMOOTH, s, c, 1, mem, cls[c]);
    }
  }
  st[ORC_ROUNDS] = sweeps;
  st[ORC_CONVERGED] = 1;
  return 0;
}

// stable renumbering: live vertices and elements keep their relative order
void orc_compact(orc_mesh* mp) {
  Mesh& m = *mp;
  std::vector<int32_t> vmap(m.V, -1);
  int32_t nv = 0;
  for (int64_t v = 0; v < m.V; ++v)
    if (m.valive[v]) vmap[v] = nv++;
  Mesh out;
  out.seed = m.seed;
  out.hook = m.hook;
  out.hook_user = m.hook_user;
  out.order_seed = m.order_seed;
  out.ad_iter = m.ad_iter;
  out.ad_phase = m.ad_phase;
  out.ad_changed = m.ad_changed;
  out.qk = m.qk;
  out.V = nv;
  for (int64_t v = 0; v < m.V; ++v) {
    if (!m.valive[v]) continue;
    out.x.push_back(m.x[v]);
    out.y.push_back(m.y[v]);
    out.ma.push_back(m.ma[v]);
    out.mb.push_back(m.mb[v]);
    out.mc.push_back(m.mc[v]);
    out.tag.push_back(m.tag[v]);
    out.valive.push_back(1);
  }
  for (int64_t t = 0; t < m.T; ++t) {
    if (!m.talive[t]) continue;
    const Tri& e = m.tri[t];
    out.tri.push_back({vmap[e[0]], vmap[e[1]], vmap[e[2]]});
    out.talive.push_back(1);
  }
  out.T = (int64_t)out.tri.size();
  rebuild_rows(out);
  static_cast<Mesh&>(m) = std::move(out);
}

void orc_quality(const orc_mesh* m, double* Q, double* qmin, double* dQdx, double* dQdM) {
  double s = 0.0, mn = 0.0;
  bool first = true;
  for (int64_t t = 0; t < m->T; ++t) {
    if (!m->talive[t]) continue;
    double q = qval(*m, geo(*m, m->tri[t]));
    s = s + q;
    if (first || q < mn) mn = q;
    first = false;
  }
  if (Q) *Q = s;
  if (qmin) *qmin = mn;
  if (!dQdx && !dQdM) return;
  for (int64_t v = 0; v < m->V; ++v) {
    double gx = 0.0, gy = 0.0, ga = 0.0, gb = 0.0, gc = 0.0;
    for (int32_t t : m->NE[v]) {
      const Tri& e = m->tri[t];
      Geo g = geo(*m, e);
      double ex, ey, da, db, dc;
      qgrad_x(*m, g, pos_in(e, (int32_t)v), &ex, &ey);
      qgrad_m(*m, g, &da, &db, &dc);
      gx = gx + ex;
      gy = gy + ey;
      ga = ga + da / 3.0;
      gb = gb + db / 3.0;
      gc = gc + dc / 3.0;
    }
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

void orc_element_quality(const orc_mesh* m, double* q) {
  for (int64_t t = 0; t < m->T; ++t) q[t] = m->talive[t] ? qval(*m, geo(*m, m->tri[t])) : 0.0;
}

double orc_patch_quality(const orc_mesh* m, int32_t v) { return patch_q(*m, v, m->x[v], m->y[v]); }

// ---- Algorithm 1 (Sec. 2.3): the mesh optimisation procedure ----------------------------
// Reading: one outer iteration is coarsen, swap, refine, in that order. The
// loop ends after an iteration that changes nothing (no collapse, flip or
// split: the mesh has converged, and every later iteration would change
// nothing either) or after max_iterations iterations; then the mesh is
// smoothed once. Iteration i runs its phases with sweep index i; the final
// smoothing uses sweep index 0 (its context differs from the loop's by the
// phase). The loop state lives in the mesh, so a call that may run only
// max_phases phases stops at a resume point and the next call goes on.
int32_t orc_adapt(orc_mesh* mp, int32_t max_iterations, int32_t max_phases, int32_t smooth_kind,
                  int32_t smooth_sweeps, double L_low2, double L_up2, double q_min, int32_t coarsen_rounds,
                  int32_t swap_rounds, int32_t refine_passes, int64_t* st) {
  Mesh& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  int64_t ph[ORC_NSTATS];
  int32_t run = 0;
  for (;;) {
    if (m.ad_phase == ORC_PHASE_COARSEN && m.ad_iter >= max_iterations) m.ad_phase = ORC_PHASE_SMOOTH;
    if (m.ad_phase == ORC_PHASE_DONE) return 0;
    if (max_phases > 0 && run == max_phases) return 2;
    int32_t phase = m.ad_phase, rc;
    if (phase == ORC_PHASE_COARSEN) rc = orc_coarsen(mp, m.ad_iter, L_low2, q_min, coarsen_rounds, ph);
    else if (phase == ORC_PHASE_SWAP) rc = orc_swap(mp, m.ad_iter, swap_rounds, ph);
    else if (phase == ORC_PHASE_REFINE) rc = orc_refine(mp, L_up2, refine_passes, ph);
    else rc = orc_smooth(mp, 0, smooth_kind, smooth_sweeps, ph);
    if (rc < 0) return rc;
    for (int k = 1; k < ORC_NSTATS; ++k)
      if (k != ORC_CONVERGED) st[k] += ph[k];
    if (phase != ORC_PHASE_SMOOTH && ph[ORC_COMMITTED] > 0) m.ad_changed = 1;
    if (phase == ORC_PHASE_COARSEN) {
      m.ad_phase = ORC_PHASE_SWAP;
    } else if (phase == ORC_PHASE_SWAP) {
      m.ad_phase = ORC_PHASE_REFINE;
    } else if (phase == ORC_PHASE_REFINE) {
      ++m.ad_iter;
      st[ORC_ROUNDS] += 1;
      if (!m.ad_changed) st[ORC_CONVERGED] = 1;
      m.ad_phase = m.ad_changed ? ORC_PHASE_COARSEN : ORC_PHASE_SMOOTH;
      m.ad_changed = 0;
    } else {
      m.ad_phase = ORC_PHASE_DONE;
    }
    ++run;
  }
}

void orc_get_context(const orc_mesh* m, int32_t* iteration, int32_t* phase, int32_t* changed) {
  *iteration = m->ad_iter;
  *phase = m->ad_phase;
  *changed = m->ad_changed;
}
void orc_set_context(orc_mesh* m, int32_t iteration, int32_t phase, int32_t changed) {
  m->ad_iter = iteration;
  m->ad_phase = phase;
  m->ad_changed = changed;
}

}  // extern "C"
