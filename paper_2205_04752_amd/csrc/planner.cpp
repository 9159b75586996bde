// Host planner: input validation, triangle geometry, binary cluster tree,
// admissibility and block partition (Sec. 2.1), quadrature rules.
//
// Compiled with -ffp-contract=off: the centroids, boxes and admissibility
// tests below are evaluated operation by operation in IEEE binary64, so the
// partition depends on the mesh only (no contraction-dependent ties).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hmat_internal.hpp"

namespace hm {

hmat_status validate_params(double E, double nu, double eta, int32_t leaf, double eps,
                            std::string& err) {
  if (!(E > 0.0) || !std::isfinite(E)) { err = "E must be finite and > 0"; return HMAT_EINVAL; }
  if (!(nu > 0.0 && nu < 0.5)) { err = "nu must lie in (0, 1/2)"; return HMAT_EINVAL; }
  if (!(eta > 0.0) || !std::isfinite(eta)) { err = "eta must be finite and > 0"; return HMAT_EINVAL; }
  if (leaf < 1) { err = "leaf must be >= 1"; return HMAT_EINVAL; }
  if (!(eps > 0.0 && eps < 1.0)) { err = "eps must lie in (0, 1)"; return HMAT_EINVAL; }
  return HMAT_OK;
}

static void tri_points(const hmat_mesh* m, int32_t i, const double* P[3]) {
  for (int v = 0; v < 3; v++) P[v] = m->vertices + 3 * (int64_t)m->triangles[3 * (int64_t)i + v];
}

static double tri_area(const double* P[3]) {
  double u[3], w[3];
  for (int d = 0; d < 3; d++) {
    u[d] = P[1][d] - P[0][d];
    w[d] = P[2][d] - P[0][d];
  }
  double nx = u[1] * w[2] - u[2] * w[1];
  double ny = u[2] * w[0] - u[0] * w[2];
  double nz = u[0] * w[1] - u[1] * w[0];
  return 0.5 * std::sqrt(nx * nx + ny * ny + nz * nz);
}

hmat_status validate_mesh(const hmat_mesh* m, std::string& err) {
  if (!m) { err = "mesh is NULL"; return HMAT_EINVAL; }
  if (m->n_triangles < 1 || m->n_vertices < 3) { err = "mesh needs >= 1 triangle and >= 3 vertices"; return HMAT_EINVAL; }
  if (!m->vertices || !m->triangles) { err = "mesh arrays are NULL"; return HMAT_EINVAL; }
  if ((int64_t)m->n_triangles * 3 > (int64_t)INT32_MAX / 2) { err = "mesh too large"; return HMAT_EINVAL; }
  for (int64_t k = 0; k < 3 * (int64_t)m->n_vertices; k++)
    if (!std::isfinite(m->vertices[k])) { err = "non-finite vertex coordinate"; return HMAT_EINVAL; }
  for (int64_t k = 0; k < 3 * (int64_t)m->n_triangles; k++) {
    int32_t v = m->triangles[k];
    if (v < 0 || v >= m->n_vertices) {
      err = "triangle " + std::to_string(k / 3) + " has vertex index out of range";
      return HMAT_EINVAL;
    }
  }
  for (int32_t i = 0; i < m->n_triangles; i++) {
    const double* P[3];
    tri_points(m, i, P);
    if (!(tri_area(P) > 0.0)) {
      err = "triangle " + std::to_string(i) + " has zero area";
      return HMAT_EINVAL;
    }
  }
  return HMAT_OK;
}

// ---------------------------------------------------------------------------
// Cluster tree: bisection of the centroid box at the midpoint of its longest
// extent (lowest axis index on ties); son 0 takes coordinates <= mid, the
// relative order of triangles is kept; at most `leaf` triangles or a zero
// extent make a leaf. Built iteratively over an explicit work stack.

namespace {

void leaf_box(const hmat_mesh* m, const int32_t* idx, int32_t len, double lo[3], double hi[3]) {
  for (int d = 0; d < 3; d++) {
    lo[d] = INFINITY;
    hi[d] = -INFINITY;
  }
  for (int32_t k = 0; k < len; k++) {
    const double* P[3];
    tri_points(m, idx[k], P);
    for (int v = 0; v < 3; v++)
      for (int d = 0; d < 3; d++) {
        lo[d] = std::min(lo[d], P[v][d]);
        hi[d] = std::max(hi[d], P[v][d]);
      }
  }
}

double diam(const Cluster& c) {
  double dx = c.hi[0] - c.lo[0];
  double dy = c.hi[1] - c.lo[1];
  double dz = c.hi[2] - c.lo[2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

double dist(const Cluster& a, const Cluster& b) {
  double g[3];
  for (int d = 0; d < 3; d++) g[d] = std::max(0.0, std::max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d]));
  return std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

}  // namespace

// Indices of `key` in decreasing key order, equal keys in increasing index
// order: least-significant-digit radix sort, 16 bits per pass, as many
// passes as the largest key needs (a comparison sort of the ~10^5 product
// items took several ms of every build).
std::vector<int32_t> order_desc_stable(const std::vector<uint64_t>& key) {
  const size_t n = key.size();
  std::vector<int32_t> idx(n), tmp(n);
  for (size_t t = 0; t < n; t++) idx[t] = (int32_t)t;
  uint64_t kmax = 0;
  for (uint64_t k : key) kmax = std::max(kmax, k);
  std::vector<size_t> cnt(65537);
  for (int sh = 0; sh < 64 && (sh == 0 || (kmax >> sh) != 0); sh += 16) {
    std::fill(cnt.begin(), cnt.end(), 0);
    // digit d goes to bucket 65535 - d: larger digits first
    for (size_t t = 0; t < n; t++) cnt[65535 - ((key[idx[t]] >> sh) & 0xFFFF) + 1]++;
    for (size_t b = 0; b < 65536; b++) cnt[b + 1] += cnt[b];
    for (size_t t = 0; t < n; t++) tmp[cnt[65535 - ((key[idx[t]] >> sh) & 0xFFFF)]++] = idx[t];
    idx.swap(tmp);
  }
  return idx;
}

void make_plan(const hmat_mesh* m, double eta, int32_t leaf, Plan& plan) {
  const int32_t nt = m->n_triangles;
  plan.nt = nt;
  std::vector<double> cen(3 * (size_t)nt);
  for (int32_t i = 0; i < nt; i++) {
    const double* P[3];
    tri_points(m, i, P);
    for (int d = 0; d < 3; d++) cen[3 * (size_t)i + d] = ((P[0][d] + P[1][d]) + P[2][d]) / 3.0;
  }
  plan.order.resize(nt);
  for (int32_t i = 0; i < nt; i++) plan.order[i] = i;
  plan.cl.clear();
  plan.cl.reserve(2 * (size_t)nt / std::max(1, leaf) + 8);
  plan.cl.push_back(Cluster{0, nt, -1, -1, 0, {0, 0, 0}, {0, 0, 0}});
  std::vector<int32_t> stack{0};
  while (!stack.empty()) {
    int32_t id = stack.back();
    stack.pop_back();
    Cluster c = plan.cl[id];
    if (c.len <= leaf) continue;
    int32_t* idx = plan.order.data() + c.off;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t k = 0; k < c.len; k++)
      for (int d = 0; d < 3; d++) {
        double x = cen[3 * (size_t)idx[k] + d];
        lo[d] = std::min(lo[d], x);
        hi[d] = std::max(hi[d], x);
      }
    int ax = 0;
    for (int d = 1; d < 3; d++)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    if (!(hi[ax] - lo[ax] > 0.0)) continue;
    const double mid = 0.5 * (lo[ax] + hi[ax]);
    auto it = std::stable_partition(idx, idx + c.len,
                                    [&](int32_t t) { return cen[3 * (size_t)t + ax] <= mid; });
    int32_t n0 = (int32_t)(it - idx);
    if (n0 == 0 || n0 == c.len) continue;
    int32_t s0 = (int32_t)plan.cl.size();
    plan.cl.push_back(Cluster{c.off, n0, -1, -1, c.level + 1, {0, 0, 0}, {0, 0, 0}});
    plan.cl.push_back(Cluster{c.off + n0, c.len - n0, -1, -1, c.level + 1, {0, 0, 0}, {0, 0, 0}});
    plan.cl[id].son0 = s0;
    plan.cl[id].son1 = s0 + 1;
    stack.push_back(s0 + 1);
    stack.push_back(s0);
  }
  // Support boxes X_t (vertices of the cluster's triangles): leaves directly,
  // inner clusters as the union of their sons' boxes (children have larger ids).
  plan.depth = 0;
  for (int32_t id = (int32_t)plan.cl.size() - 1; id >= 0; id--) {
    Cluster& c = plan.cl[id];
    plan.depth = std::max(plan.depth, c.level);
    if (c.son0 < 0) {
      leaf_box(m, plan.order.data() + c.off, c.len, c.lo, c.hi);
    } else {
      const Cluster& a = plan.cl[c.son0];
      const Cluster& b = plan.cl[c.son1];
      for (int d = 0; d < 3; d++) {
        c.lo[d] = std::min(a.lo[d], b.lo[d]);
        c.hi[d] = std::max(a.hi[d], b.hi[d]);
      }
    }
  }
  // Block partition: leaves of the block-cluster tree (both sons split together).
  plan.blk.clear();
  std::vector<std::pair<int32_t, int32_t>> todo{{0, 0}};
  while (!todo.empty()) {
    auto [t, s] = todo.back();
    todo.pop_back();
    const Cluster& T = plan.cl[t];
    const Cluster& S = plan.cl[s];
    const double d = dist(T, S);
    if (d > 0.0 && std::min(diam(T), diam(S)) <= eta * d) {
      plan.blk.push_back(BlockRec{t, s, 1});
    } else if (T.son0 < 0 || S.son0 < 0) {
      plan.blk.push_back(BlockRec{t, s, 0});
    } else {
      todo.push_back({T.son0, S.son0});
      todo.push_back({T.son0, S.son1});
      todo.push_back({T.son1, S.son0});
      todo.push_back({T.son1, S.son1});
    }
  }
  // canonical order: by row offset, then column offset (the pairs are unique)
  {
    std::vector<uint64_t> key(plan.blk.size());
    for (size_t q = 0; q < plan.blk.size(); q++)
      key[q] = ~(((uint64_t)(uint32_t)plan.cl[plan.blk[q].t].off << 32) | (uint32_t)plan.cl[plan.blk[q].s].off);
    const std::vector<int32_t> ord = order_desc_stable(key);  // descending complement = ascending
    std::vector<BlockRec> sorted(plan.blk.size());
    for (size_t q = 0; q < plan.blk.size(); q++) sorted[q] = plan.blk[ord[q]];
    plan.blk.swap(sorted);
  }
  std::vector<int32_t> nr(plan.cl.size(), 0), nc(plan.cl.size(), 0);
  for (const BlockRec& b : plan.blk) {
    nr[b.t]++;
    nc[b.s]++;
  }
  plan.csp = 0;
  for (size_t i = 0; i < plan.cl.size(); i++) plan.csp = std::max(plan.csp, std::max(nr[i], nc[i]));
}

// ---------------------------------------------------------------------------
// Quadrature rules.

// Radon's degree-5 seven-point rule (Stroud T2:5-1): centroid with weight 9/40;
// for s = +1 and s = -1, b = (6 + s sqrt15)/21, a = 1 - 2b, weight
// (155 + s sqrt15)/1200, at (a,b,b), (b,a,b), (b,b,a).
void radon7(double bary[7][3], double w[7]) {
  const double r = std::sqrt(15.0);
  bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
  w[0] = 9.0 / 40.0;
  int k = 1;
  for (double s : {1.0, -1.0}) {
    const double b = (6.0 + s * r) / 21.0;
    const double a = 1.0 - 2.0 * b;
    for (int v = 0; v < 3; v++, k++) {
      for (int c = 0; c < 3; c++) bary[k][c] = (c == v) ? a : b;
      w[k] = (155.0 + s * r) / 1200.0;
    }
  }
}

// Legendre P_n and P_n' at x by the three-term recurrence.
static void legendre(int n, double x, double& p, double& dp) {
  double pm = 1.0, pc = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; k++) {
    const double pn = ((2 * k - 1) * x * pc - (k - 1) * pm) / k;
    pm = pc;
    pc = pn;
  }
  p = pc;
  dp = n * (pm - x * pc) / (1.0 - x * x);
}

// Gauss-Legendre rule mapped to [0,1]: roots of P_n bracketed by sign changes
// of P_n on a uniform grid of [-1,1] (spacing far below the root spacing),
// refined by bisection and one Newton step; weights 2/((1-x^2) P_n'(x)^2),
// halved for the unit interval. Nodes ascending.
void gauss_legendre_unit(int n, double* x, double* w) {
  const int grid = 64 * n;
  int found = 0;
  double a = -1.0;
  double pa = (n % 2 == 0) ? 1.0 : -1.0;  // P_n(-1) = (-1)^n
  for (int g = 1; g <= grid && found < n; g++) {
    const double b = -1.0 + 2.0 * g / grid;
    double pb = 1.0, dpb;  // P_n(1) = 1
    if (g < grid) legendre(n, b, pb, dpb);
    double root;
    if (pb == 0.0) {
      root = b;
    } else if ((pa < 0.0) != (pb < 0.0) && pa != 0.0) {
      double lo = a, hi = b, flo = pa;
      for (int it = 0; it < 200; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm, dfm;
        legendre(n, mid, fm, dfm);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      root = 0.5 * (lo + hi);
      double p, dp;
      legendre(n, root, p, dp);
      root -= p / dp;
    } else {
      a = b;
      pa = pb;
      continue;
    }
    double p, dp;
    legendre(n, root, p, dp);
    x[found] = 0.5 * (root + 1.0);
    w[found] = 0.5 * (2.0 / ((1.0 - root * root) * dp * dp));
    found++;
    a = b;
    pa = pb;
  }
}

// Geometry in cluster order: centroids, quadrature nodes y_k = sum_v bary[k][v] P_v
// with weights w_k |tau|, vertices, and the Gauss-Legendre rule for the self term.
void make_geometry(const hmat_mesh* m, const Plan& plan, HostGeometry& g) {
  const int32_t nt = plan.nt;
  double bary[7][3], wr[7];
  radon7(bary, wr);
  g.cen.assign(3 * (size_t)nt, 0.0);
  g.q.assign(4 * 7 * (size_t)nt, 0.0);
  g.vtx.assign(9 * (size_t)nt, 0.0);
  for (int32_t p = 0; p < nt; p++) {
    const double* P[3];
    tri_points(m, plan.order[p], P);
    const double area = tri_area(P);
    for (int d = 0; d < 3; d++) g.cen[(size_t)d * nt + p] = ((P[0][d] + P[1][d]) + P[2][d]) / 3.0;
    for (int k = 0; k < 7; k++) {
      for (int d = 0; d < 3; d++)
        g.q[((size_t)d * 7 + k) * nt + p] =
            (bary[k][0] * P[0][d] + bary[k][1] * P[1][d]) + bary[k][2] * P[2][d];
      g.q[((size_t)3 * 7 + k) * nt + p] = wr[k] * area;
    }
    for (int v = 0; v < 3; v++)
      for (int d = 0; d < 3; d++) g.vtx[((size_t)v * 3 + d) * nt + p] = P[v][d];
  }
  g.gl.assign(32, 0.0);
  gauss_legendre_unit(16, g.gl.data(), g.gl.data() + 16);
}

}  // namespace hm
