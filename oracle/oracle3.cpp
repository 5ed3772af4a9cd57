// CPU oracle, tetrahedral meshes: plain serial FP64 definition of the 3D
// adaptation path. TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline
// timing); the HIP library never includes, links or calls this file.
//
// Built with g++ -O2 -ffp-contract=off: every floating-point operation below
// is one IEEE-754 binary64 operation rounded to nearest.
//
// Sec. 4 extrudes the method to three dimensions: coarsening, refinement and
// smoothing on tetrahedra, with no swapping. The round structure is the 2D
// one (Sec. 3.2 colouring of the active vertices, classes processed one after
// the other as independent sets, re-validation against the current graph,
// propagation to the touched neighbourhood, Sec. 2.4.5). Readings:
//   - quality (Sec. 2.2; the tetrahedral functional is only cited): the mean
//     ratio q = 12 (3 |K|_M)^(2/3) / S, |K|_M = sqrt(det M) |K| and S the sum
//     of the six squared metric edge lengths, M the mean of the four vertex
//     tensors; 1 for the regular tetrahedron with unit metric edges.
//     Decisions compare q^3 = 432 det(M) D^2 / S^3 (D = 6 |K|, no roots).
//   - collapse (Sec. 2.4.1): as in 2D; u must lie on every boundary face of
//     the unit cube that v lies on; every re-pointed element keeps D > 0 and
//     q^3 >= q_min^3.
//   - refinement (Sec. 2.4.2): every long edge is split at its midpoint in one
//     pass; an element with split edges is bisected along them one at a time
//     in one global edge order (larger L^2 first, ties by (min id, max id)),
//     so two elements sharing a face cut it the same way and the result is
//     conforming without a table of templates.
//   - smoothing (Sec. 2.4.4): the Laplacian in the metric (a 3x3 solve),
//     kept when every element keeps D > 0 and the patch minimum of q^3 does
//     not drop; interior vertices only.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#include "oracle.h"

namespace {

const uint8_t TX0 = 1, TX1 = 2, TY0 = 4, TY1 = 8, TZ0 = 16, TZ1 = 32;
enum { PH_COARSEN = 1, PH_SMOOTH = 3 };

using Tet = std::array<int32_t, 4>;
struct Met3 {
  double a00, a01, a02, a11, a12, a22;
};

struct Mesh3 {
  int64_t V = 0, T = 0;
  std::vector<double> x, y, z;
  std::vector<Met3> met;
  std::vector<uint8_t> tag, valive;
  std::vector<Tet> tet;
  std::vector<uint8_t> talive;
  std::vector<std::vector<int32_t>> NN, NE;
  uint64_t seed = 0;
  orc_hook hook = nullptr;
  void* hook_user = nullptr;
  std::vector<int32_t> cur_members, cur_class;
};

// ---- sorted-set rows ------------------------------------------------------------
void set_insert(std::vector<int32_t>& s, int32_t v) {
  auto it = std::lower_bound(s.begin(), s.end(), v);
  if (it == s.end() || *it != v) s.insert(it, v);
}
void set_erase(std::vector<int32_t>& s, int32_t v) {
  auto it = std::lower_bound(s.begin(), s.end(), v);
  if (it != s.end() && *it == v) s.erase(it);
}

bool has(const Tet& t, int32_t v) { return t[0] == v || t[1] == v || t[2] == v || t[3] == v; }
int pos_of(const Tet& t, int32_t v) { return t[0] == v ? 0 : (t[1] == v ? 1 : (t[2] == v ? 2 : 3)); }

// Orientation-preserving canonical order: the smallest id first (by one of the
// four even permutations that bring a vertex to the front), then the other
// three rotated cyclically so that the smallest of them comes second.
Tet canon(const Tet& t) {
  int k = 0;
  for (int i = 1; i < 4; ++i)
    if (t[i] < t[k]) k = i;
  Tet r;
  if (k == 0) r = t;
  else if (k == 1) r = {t[1], t[0], t[3], t[2]};
  else if (k == 2) r = {t[2], t[3], t[0], t[1]};
  else r = {t[3], t[2], t[1], t[0]};
  int j = 1;
  if (r[2] < r[j]) j = 2;
  if (r[3] < r[j]) j = 3;
  if (j == 2) r = {r[0], r[2], r[3], r[1]};
  else if (j == 3) r = {r[0], r[3], r[1], r[2]};
  return r;
}

void rebuild_rows(Mesh3& m) {
  m.NN.assign(m.V, {});
  m.NE.assign(m.V, {});
  for (int64_t t = 0; t < m.T; ++t) {
    if (!m.talive[t]) continue;
    for (int k = 0; k < 4; ++k) m.NE[m.tet[t][k]].push_back((int32_t)t);
  }
  for (int64_t v = 0; v < m.V; ++v) {
    std::vector<int32_t> nb;
    for (int32_t t : m.NE[v])
      for (int k = 0; k < 4; ++k)
        if (m.tet[t][k] != v) nb.push_back(m.tet[t][k]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    m.NN[v] = nb;
  }
}

// NN(w) from the current NE(w)
void row_from_elements(Mesh3& m, int32_t w) {
  std::vector<int32_t> nb;
  for (int32_t t : m.NE[w])
    for (int k = 0; k < 4; ++k)
      if (m.tet[t][k] != w) nb.push_back(m.tet[t][k]);
  std::sort(nb.begin(), nb.end());
  nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
  m.NN[w] = nb;
}

// ---- metric geometry (Sec. 2.2, in three dimensions) -------------------------------
// Edge tensor = mean of the two end-point tensors; element tensor = mean of
// the four vertex tensors in the element's stored order.
Met3 edge_met(const Met3& p, const Met3& q) {
  return Met3{(p.a00 + q.a00) * 0.5, (p.a01 + q.a01) * 0.5, (p.a02 + q.a02) * 0.5,
              (p.a11 + q.a11) * 0.5, (p.a12 + q.a12) * 0.5, (p.a22 + q.a22) * 0.5};
}

// e^T M e; each term is a product of two components of e, so the value is
// bitwise the same for -e
double qform(const Met3& e, double dx, double dy, double dz) {
  return (((e.a00 * dx) * dx + ((2.0 * e.a01) * dx) * dy) + ((2.0 * e.a02) * dx) * dz) +
         (((e.a11 * dy) * dy + ((2.0 * e.a12) * dy) * dz) + (e.a22 * dz) * dz);
}

double len2(const Mesh3& m, int32_t i, int32_t j) {
  return qform(edge_met(m.met[i], m.met[j]), m.x[j] - m.x[i], m.y[j] - m.y[i], m.z[j] - m.z[i]);
}

double det3(const Met3& g) {
  return (g.a00 * (g.a11 * g.a22 - g.a12 * g.a12) - g.a01 * (g.a01 * g.a22 - g.a12 * g.a02)) +
         g.a02 * (g.a01 * g.a12 - g.a11 * g.a02);
}

struct Geo3 {
  double x[4], y[4], z[4];
  Met3 m;
};

// element t's geometry; vertex ov, if present, placed at p
Geo3 geo(const Mesh3& m, const Tet& t, int32_t ov = -1, double px = 0.0, double py = 0.0, double pz = 0.0) {
  Geo3 g;
  for (int k = 0; k < 4; ++k) {
    int32_t v = t[k];
    bool o = v == ov;
    g.x[k] = o ? px : m.x[v];
    g.y[k] = o ? py : m.y[v];
    g.z[k] = o ? pz : m.z[v];
  }
  const Met3 &a = m.met[t[0]], &b = m.met[t[1]], &c = m.met[t[2]], &d = m.met[t[3]];
  g.m = Met3{(((a.a00 + b.a00) + c.a00) + d.a00) / 4.0, (((a.a01 + b.a01) + c.a01) + d.a01) / 4.0,
             (((a.a02 + b.a02) + c.a02) + d.a02) / 4.0, (((a.a11 + b.a11) + c.a11) + d.a11) / 4.0,
             (((a.a12 + b.a12) + c.a12) + d.a12) / 4.0, (((a.a22 + b.a22) + c.a22) + d.a22) / 4.0};
  return g;
}

// six times the signed Euclidean volume
double vol6(const Geo3& g) {
  double ax = g.x[1] - g.x[0], ay = g.y[1] - g.y[0], az = g.z[1] - g.z[0];
  double bx = g.x[2] - g.x[0], by = g.y[2] - g.y[0], bz = g.z[2] - g.z[0];
  double cx = g.x[3] - g.x[0], cy = g.y[3] - g.y[0], cz = g.z[3] - g.z[0];
  return (ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx)) + az * (bx * cy - by * cx);
}

// sum of the six squared metric edge lengths, edges (01, 02, 03, 12, 13, 23)
double edge_sum(const Geo3& g) {
  static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  double s = 0.0;
  for (int k = 0; k < 6; ++k) {
    int i = E[k][0], j = E[k][1];
    s = s + qform(g.m, g.x[j] - g.x[i], g.y[j] - g.y[i], g.z[j] - g.z[i]);
  }
  return s;
}

// q^3 = 432 det(M) D^2 / S^3: every decision uses this root-free form
double qual3(const Geo3& g) {
  double D = vol6(g), S = edge_sum(g), det = det3(g.m);
  return (((432.0 * det) * D) * D) / ((S * S) * S);
}

// reported quality q = 12 (3 |K|_M)^(2/3) / S, (3 |K|_M)^2 = det D^2 / 4
double qual(const Geo3& g) {
  double D = vol6(g), S = edge_sum(g), det = det3(g.m);
  return (12.0 * std::cbrt(((det * D) * D) * 0.25)) / S;
}

// ---- priorities and colouring (Sec. 3.2), as in two dimensions -----------------------
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
bool key_greater(uint32_t pa, int32_t a, uint32_t pb, int32_t b) { return pa != pb ? pa > pb : a > b; }

// greedy first-fit in descending key order (what Jones-Plassmann computes)
int32_t colour(const Mesh3& m, const std::vector<int32_t>& A, uint32_t ctx, std::vector<int32_t>& col) {
  col.assign(m.V, -1);
  std::vector<std::pair<uint32_t, int32_t>> order;
  for (int32_t v : A) order.push_back({prio(m.seed, ctx, (uint32_t)v), v});
  std::sort(order.begin(), order.end(),
            [](const auto& p, const auto& q) { return key_greater(p.first, p.second, q.first, q.second); });
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

void revalidate(const Mesh3& m, const std::vector<int32_t>& members, const std::vector<int32_t>& col, int32_t c,
                uint32_t ctx, std::vector<int32_t>& kept, std::vector<int32_t>& deferred) {
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

std::vector<std::vector<int32_t>> classes_of(const std::vector<int32_t>& A, const std::vector<int32_t>& col,
                                             int32_t ncol) {
  std::vector<std::vector<int32_t>> cls(ncol);
  for (int32_t v : A) cls[col[v]].push_back(v);
  return cls;
}

void run_hook(Mesh3& m, int phase, int round, int cls, int stage, const std::vector<int32_t>& members,
              const std::vector<int32_t>& whole) {
  if (!m.hook) return;
  m.cur_members = members;
  m.cur_class = whole;
  m.hook(m.hook_user, phase, round, cls, stage);
}

// ---- coarsening (Sec. 2.4.1) --------------------------------------------------------
bool tag_ok(const Mesh3& m, int32_t v, int32_t u) { return (m.tag[v] & ~m.tag[u]) == 0; }

bool has_candidate(const Mesh3& m, int32_t v, double L_low2) {
  for (int32_t u : m.NN[v])
    if (tag_ok(m, v, u) && len2(m, v, u) < L_low2) return true;
  return false;
}

int32_t eval_collapse(const Mesh3& m, int32_t v, double L_low2, double qmin3) {
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
      const Tet& e = m.tet[t];
      if (has(e, u)) continue;  // removed with the edge
      Tet r = e;
      r[pos_of(e, v)] = u;
      Geo3 g = geo(m, canon(r));
      if (!(vol6(g) > 0.0) || !(qual3(g) >= qmin3)) {
        ok = false;
        break;
      }
    }
    if (ok) return u;
  }
  return -1;
}

void apply_collapse(Mesh3& m, int32_t v, int32_t u) {
  std::vector<int32_t> nv = m.NN[v], ne = m.NE[v];
  for (int32_t t : ne) {
    Tet& e = m.tet[t];
    if (has(e, u)) {
      m.talive[t] = 0;
      for (int k = 0; k < 4; ++k)
        if (e[k] != v) set_erase(m.NE[e[k]], t);
    } else {
      e[pos_of(e, v)] = u;
      e = canon(e);
      set_insert(m.NE[u], t);
    }
  }
  m.valive[v] = 0;
  m.NE[v].clear();
  m.NN[v].clear();
  for (int32_t w : nv) row_from_elements(m, w);  // includes u
}

void compact(Mesh3& m) {
  std::vector<int32_t> vmap(m.V, -1);
  int32_t nv = 0;
  for (int64_t v = 0; v < m.V; ++v)
    if (m.valive[v]) vmap[v] = nv++;
  Mesh3 out;
  out.seed = m.seed;
  out.hook = m.hook;
  out.hook_user = m.hook_user;
  out.V = nv;
  for (int64_t v = 0; v < m.V; ++v) {
    if (!m.valive[v]) continue;
    out.x.push_back(m.x[v]);
    out.y.push_back(m.y[v]);
    out.z.push_back(m.z[v]);
    out.met.push_back(m.met[v]);
    out.tag.push_back(m.tag[v]);
    out.valive.push_back(1);
  }
  for (int64_t t = 0; t < m.T; ++t) {
    if (!m.talive[t]) continue;
    const Tet& e = m.tet[t];
    // a monotone renumbering keeps the canonical order
    out.tet.push_back({vmap[e[0]], vmap[e[1]], vmap[e[2]], vmap[e[3]]});
    out.talive.push_back(1);
  }
  out.T = (int64_t)out.tet.size();
  rebuild_rows(out);
  m = std::move(out);
}

// ---- refinement (Sec. 2.4.2) ------------------------------------------------------------
struct Split {
  int32_t a, b, mid;
  double L2;
};
// global order of split edges: larger L^2 first, then (min id, max id)
bool split_before(const Split& p, const Split& q) {
  if (p.L2 != q.L2) return p.L2 > q.L2;
  return p.a != q.a ? p.a < q.a : p.b < q.b;
}

// bisect e along the first edge of `order` that it holds, children depth first
void bisect(const Tet& e, const std::vector<Split>& order, std::vector<Tet>& leaves) {
  for (const Split& s : order) {
    if (!has(e, s.a) || !has(e, s.b)) continue;
    Tet ca = e, cb = e;
    ca[pos_of(e, s.b)] = s.mid;  // keeps a
    cb[pos_of(e, s.a)] = s.mid;  // keeps b
    bisect(ca, order, leaves);
    bisect(cb, order, leaves);
    return;
  }
  leaves.push_back(e);
}

}  // namespace

struct orc3_mesh : Mesh3 {};

extern "C" {

orc3_mesh* orc3_create(int64_t V, int64_t T, const double* xyz, const int32_t* tet, const double* metric,
                       const uint8_t* tags, uint64_t seed) {
  if (V <= 0 || T <= 0 || !xyz || !tet || !metric) return nullptr;
  orc3_mesh* m = new orc3_mesh();
  m->V = V;
  m->T = T;
  m->seed = seed;
  m->x.resize(V);
  m->y.resize(V);
  m->z.resize(V);
  m->met.resize(V);
  m->tag.resize(V);
  m->valive.assign(V, 1);
  for (int64_t v = 0; v < V; ++v) {
    m->x[v] = xyz[3 * v];
    m->y[v] = xyz[3 * v + 1];
    m->z[v] = xyz[3 * v + 2];
    const double* p = metric + 6 * v;
    Met3 g{p[0], p[1], p[2], p[3], p[4], p[5]};
    m->met[v] = g;
    if (!(g.a00 > 0.0) || !(g.a00 * g.a11 - g.a01 * g.a01 > 0.0) || !(det3(g) > 0.0)) {
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
      if (m->z[v] == 0.0) t |= TZ0;
      if (m->z[v] == 1.0) t |= TZ1;
      m->tag[v] = t;
    }
  }
  m->tet.resize(T);
  m->talive.assign(T, 1);
  for (int64_t t = 0; t < T; ++t) {
    Tet e{tet[4 * t], tet[4 * t + 1], tet[4 * t + 2], tet[4 * t + 3]};
    for (int k = 0; k < 4; ++k)
      if (e[k] < 0 || e[k] >= V) {
        delete m;
        return nullptr;
      }
    if (e[0] == e[1] || e[0] == e[2] || e[0] == e[3] || e[1] == e[2] || e[1] == e[3] || e[2] == e[3]) {
      delete m;
      return nullptr;
    }
    m->tet[t] = canon(e);
    if (!(vol6(geo(*m, m->tet[t])) > 0.0)) {
      delete m;
      return nullptr;
    }
  }
  rebuild_rows(*m);
  return m;
}

void orc3_destroy(orc3_mesh* m) { delete m; }

void orc3_sizes(const orc3_mesh* m, int64_t* V, int64_t* T) {
  if (V) *V = m->V;
  if (T) *T = m->T;
}

void orc3_export(const orc3_mesh* m, double* xyz, int32_t* tet, double* metric, uint8_t* tags, uint8_t* valive,
                 uint8_t* talive) {
  for (int64_t v = 0; v < m->V; ++v) {
    if (xyz) {
      xyz[3 * v] = m->x[v];
      xyz[3 * v + 1] = m->y[v];
      xyz[3 * v + 2] = m->z[v];
    }
    if (metric) {
      const Met3& g = m->met[v];
      double* p = metric + 6 * v;
      p[0] = g.a00;
      p[1] = g.a01;
      p[2] = g.a02;
      p[3] = g.a11;
      p[4] = g.a12;
      p[5] = g.a22;
    }
    if (tags) tags[v] = m->tag[v];
    if (valive) valive[v] = m->valive[v];
  }
  for (int64_t t = 0; t < m->T; ++t) {
    if (tet)
      for (int k = 0; k < 4; ++k) tet[4 * t + k] = m->tet[t][k];
    if (talive) talive[t] = m->talive[t];
  }
}

void orc3_row_totals(const orc3_mesh* m, int64_t* nn_total, int64_t* ne_total) {
  int64_t a = 0, b = 0;
  for (int64_t v = 0; v < m->V; ++v) {
    a += (int64_t)m->NN[v].size();
    b += (int64_t)m->NE[v].size();
  }
  *nn_total = a;
  *ne_total = b;
}

void orc3_export_rows(const orc3_mesh* m, int64_t* nn_off, int32_t* nn, int64_t* ne_off, int32_t* ne) {
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

void orc3_set_xyz(orc3_mesh* m, int32_t v, double x, double y, double z) {
  m->x[v] = x;
  m->y[v] = y;
  m->z[v] = z;
}

void orc3_set_hook(orc3_mesh* m, orc_hook hook, void* user) {
  m->hook = hook;
  m->hook_user = user;
}

int64_t orc3_class_members(const orc3_mesh* m, int32_t* out, int64_t cap) {
  int64_t n = (int64_t)m->cur_members.size();
  for (int64_t i = 0; i < n && i < cap; ++i) out[i] = m->cur_members[i];
  return n;
}

int64_t orc3_class_whole(const orc3_mesh* m, int32_t* out, int64_t cap) {
  int64_t n = (int64_t)m->cur_class.size();
  for (int64_t i = 0; i < n && i < cap; ++i) out[i] = m->cur_class[i];
  return n;
}

int32_t orc3_colour(orc3_mesh* m, const uint8_t* active, uint32_t ctx, int32_t* colour_out) {
  std::vector<int32_t> A, col;
  for (int64_t v = 0; v < m->V; ++v)
    if (m->valive[v] && (!active || active[v])) A.push_back((int32_t)v);
  int32_t n = colour(*m, A, ctx, col);
  if (colour_out)
    for (int64_t v = 0; v < m->V; ++v) colour_out[v] = col[v];
  return n;
}

int32_t orc3_coarsen(orc3_mesh* mp, int32_t sweep, double L_low2, double q_min, int32_t max_rounds, int64_t* st) {
  Mesh3& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  double qmin3 = (q_min * q_min) * q_min;
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
      run_hook(m, PH_COARSEN, r, c, 0, kept, cls[c]);
      for (int32_t v : kept) {
        int32_t u = eval_collapse(m, v, L_low2, qmin3);
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
  compact(m);
  return A.empty() ? 0 : 1;
}

int32_t orc3_refine(orc3_mesh* mp, double L_up2, int32_t max_passes, int64_t* st) {
  Mesh3& m = *mp;
  std::fill(st, st + ORC_NSTATS, 0);
  int32_t p = 0;
  bool done = false;
  for (; p < max_passes; ++p) {
    // split edges in (min id, max id) order; new vertex ids in that order
    std::vector<Split> splits;
    for (int64_t a = 0; a < m.V; ++a) {
      if (!m.valive[a]) continue;
      for (int32_t b : m.NN[a]) {
        if (b <= a) continue;
        st[ORC_EDGES] += 1;
        double L2 = len2(m, (int32_t)a, b);
        if (L2 > L_up2) splits.push_back(Split{(int32_t)a, b, -1, L2});
      }
    }
    if (splits.empty()) {
      done = true;
      break;
    }
    int64_t V0 = m.V;
    for (Split& s : splits) {
      int32_t a = s.a, b = s.b;
      s.mid = (int32_t)m.V++;
      m.x.push_back((m.x[a] + m.x[b]) * 0.5);
      m.y.push_back((m.y[a] + m.y[b]) * 0.5);
      m.z.push_back((m.z[a] + m.z[b]) * 0.5);
      m.met.push_back(edge_met(m.met[a], m.met[b]));
      m.tag.push_back(m.tag[a] & m.tag[b]);
      m.valive.push_back(1);
    }
    st[ORC_NEWV] += m.V - V0;
    st[ORC_COMMITTED] += (int64_t)splits.size();
    std::map<std::pair<int32_t, int32_t>, Split> by_edge;
    for (const Split& s : splits) by_edge[{s.a, s.b}] = s;
    int64_t T0 = m.T;
    std::vector<Split> own;
    std::vector<Tet> leaves;
    for (int64_t t = 0; t < T0; ++t) {
      if (!m.talive[t]) continue;
      const Tet e = m.tet[t];
      own.clear();
      for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j) {
          auto it = by_edge.find({std::min(e[i], e[j]), std::max(e[i], e[j])});
          if (it != by_edge.end()) own.push_back(it->second);
        }
      if (own.empty()) continue;
      std::sort(own.begin(), own.end(), split_before);
      leaves.clear();
      bisect(e, own, leaves);
      m.tet[t] = canon(leaves[0]);
      for (size_t i = 1; i < leaves.size(); ++i) {
        m.tet.push_back(canon(leaves[i]));
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

}  // extern "C"

namespace {

// patch minimum of q^3 with v at p; valid = every element keeps D > 0
double patch_min_q3(const Mesh3& m, int32_t v, double px, double py, double pz, bool& valid) {
  valid = true;
  double mn = 0.0;
  bool first = true;
  for (int32_t t : m.NE[v]) {
    Geo3 g = geo(m, m.tet[t], v, px, py, pz);
    if (!(vol6(g) > 0.0)) valid = false;
    double q = qual3(g);
    if (first || q < mn) mn = q;
    first = false;
  }
  return mn;
}

// Laplacian in the metric: p = x_v + G^-1 r, G = sum of the edge tensors,
// r = sum of M_vj (x_j - x_v) over NN(v) in ascending order, G^-1 by its
// adjugate over its determinant
bool smooth_laplace(Mesh3& m, int32_t v) {
  double xv = m.x[v], yv = m.y[v], zv = m.z[v];
  Met3 G{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double rx = 0.0, ry = 0.0, rz = 0.0;
  for (int32_t j : m.NN[v]) {
    Met3 e = edge_met(m.met[v], m.met[j]);
    double dx = m.x[j] - xv, dy = m.y[j] - yv, dz = m.z[j] - zv;
    G.a00 = G.a00 + e.a00;
    G.a01 = G.a01 + e.a01;
    G.a02 = G.a02 + e.a02;
    G.a11 = G.a11 + e.a11;
    G.a12 = G.a12 + e.a12;
    G.a22 = G.a22 + e.a22;
    rx = rx + ((e.a00 * dx + e.a01 * dy) + e.a02 * dz);
    ry = ry + ((e.a01 * dx + e.a11 * dy) + e.a12 * dz);
    rz = rz + ((e.a02 * dx + e.a12 * dy) + e.a22 * dz);
  }
  double det = det3(G);
  double c00 = G.a11 * G.a22 - G.a12 * G.a12, c01 = G.a02 * G.a12 - G.a01 * G.a22,
         c02 = G.a01 * G.a12 - G.a02 * G.a11, c11 = G.a00 * G.a22 - G.a02 * G.a02,
         c12 = G.a01 * G.a02 - G.a00 * G.a12, c22 = G.a00 * G.a11 - G.a01 * G.a01;
  double px = xv + ((c00 * rx + c01 * ry) + c02 * rz) / det;
  double py = yv + ((c01 * rx + c11 * ry) + c12 * rz) / det;
  double pz = zv + ((c02 * rx + c12 * ry) + c22 * rz) / det;
  bool vo, vn;
  double oldmin = patch_min_q3(m, v, xv, yv, zv, vo);
  double newmin = patch_min_q3(m, v, px, py, pz, vn);
  if (!(vn && newmin >= oldmin)) return false;
  m.x[v] = px;
  m.y[v] = py;
  m.z[v] = pz;
  return true;
}

}  // namespace

extern "C" {

int32_t orc3_smooth(orc3_mesh* mp, int32_t sweep, int32_t sweeps, int64_t* st) {
  Mesh3& m = *mp;
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
      run_hook(m, PH_SMOOTH, s, c, 0, cls[c], cls[c]);
      for (int32_t v : cls[c]) {
        st[ORC_EVALUATED] += 1;
        st[ORC_COMMITTED] += smooth_laplace(m, v) ? 1 : 0;
      }
      run_hook(m, PH_SMOOTH, s, c, 1, cls[c], cls[c]);
    }
  }
  st[ORC_ROUNDS] = sweeps;
  st[ORC_CONVERGED] = 1;
  return 0;
}

void orc3_quality(const orc3_mesh* m, double* Q, double* qmin) {
  double s = 0.0, mn = 0.0;
  bool first = true;
  for (int64_t t = 0; t < m->T; ++t) {
    if (!m->talive[t]) continue;
    double q = qual(geo(*m, m->tet[t]));
    s = s + q;
    if (first || q < mn) mn = q;
    first = false;
  }
  if (Q) *Q = s;
  if (qmin) *qmin = mn;
}

void orc3_element_quality(const orc3_mesh* m, double* q) {
  for (int64_t t = 0; t < m->T; ++t) q[t] = m->talive[t] ? qual(geo(*m, m->tet[t])) : 0.0;
}

}  // extern "C"
