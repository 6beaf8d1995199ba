// Host-side setup of libseird: mesh checks, node graph, incidence records,
// lumped mass (Section 2.2); subdomains, overlap, local ordering, tile
// envelopes, extraction maps (Section 3, Eq. RAS); nested P1 coarse space and
// Galerkin maps (Section 3.1).
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <queue>

#include "internal.h"

namespace seird {

void build_mesh(int64_t n, const double *xy, int64_t nt, const int32_t *tri,
                MeshHost &m) {
  if (n <= 0 || nt <= 0 || !xy || !tri) fail(SEIRD_ERR_ARG, "empty mesh");
  if (n > INT32_MAX / 8) fail(SEIRD_ERR_ARG, "too many nodes");
  m.n = n;
  m.nt = nt;
  m.xy.assign(xy, xy + 2 * n);
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(xy[i])) fail(SEIRD_ERR_MESH, "nonfinite node coordinate");
  std::vector<double> K(nt * 6);  // Kaa, Kbb, Kcc, Kab, Kac, Kbc
  std::vector<double> areas(nt);
  m.mass.assign(n, 0.0);
  std::vector<int32_t> deg(n, 0);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n)
      fail(SEIRD_ERR_MESH, "triangle " + std::to_string(t) + " has an out-of-range vertex");
    if (a == b || b == c || a == c)
      fail(SEIRD_ERR_MESH, "triangle " + std::to_string(t) + " repeats a vertex");
    const double x0 = xy[2 * a], y0 = xy[2 * a + 1];
    const double x1 = xy[2 * b], y1 = xy[2 * b + 1];
    const double x2 = xy[2 * c], y2 = xy[2 * c + 1];
    const double det = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    const double scale = std::fabs((x1 - x0) * (y2 - y0)) + std::fabs((x2 - x0) * (y1 - y0));
    if (!(std::fabs(det) > 1e-14 * scale) || !std::isfinite(det))
      fail(SEIRD_ERR_MESH, "triangle " + std::to_string(t) + " has zero area");
    const double area = 0.5 * std::fabs(det);
    areas[t] = area;
    // grad phi_k = (y_{k+1} - y_{k+2}, x_{k+2} - x_{k+1}) / det
    const double gx[3] = {(y1 - y2) / det, (y2 - y0) / det, (y0 - y1) / det};
    const double gy[3] = {(x2 - x1) / det, (x0 - x2) / det, (x1 - x0) / det};
    auto k = [&](int p, int q) { return area * (gx[p] * gx[q] + gy[p] * gy[q]); };
    double *Kt = &K[6 * t];
    Kt[0] = k(0, 0); Kt[1] = k(1, 1); Kt[2] = k(2, 2);
    Kt[3] = k(0, 1); Kt[4] = k(0, 2); Kt[5] = k(1, 2);
    m.mass[a] += area / 3.0;
    m.mass[b] += area / 3.0;
    m.mass[c] += area / 3.0;
    deg[a] += 2; deg[b] += 2; deg[c] += 2;
  }
  // node graph: per-node neighbour lists, sorted unique
  std::vector<int64_t> cp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) cp[i + 1] = cp[i] + deg[i];
  std::vector<int32_t> cand(cp[n]);
  std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    for (int k = 0; k < 3; ++k) {
      cand[fill[v[k]]++] = v[(k + 1) % 3];
      cand[fill[v[k]]++] = v[(k + 2) % 3];
    }
  }
  m.rowptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    auto b = cand.begin() + cp[i], e = cand.begin() + cp[i + 1];
    std::sort(b, e);
    m.rowptr[i + 1] = m.rowptr[i] + (std::unique(b, e) - b);
  }
  m.col.resize(m.rowptr[n]);
  for (int64_t i = 0; i < n; ++i) {
    std::copy(cand.begin() + cp[i], cand.begin() + cp[i] + (m.rowptr[i + 1] - m.rowptr[i]),
              m.col.begin() + m.rowptr[i]);
  }
  for (int64_t i = 0; i < n; ++i)
    if (m.rowptr[i + 1] == m.rowptr[i]) fail(SEIRD_ERR_MESH, "node " + std::to_string(i) + " belongs to no triangle");
  auto slot_of = [&](int32_t i, int32_t j) -> int32_t {
    auto b = m.col.begin() + m.rowptr[i], e = m.col.begin() + m.rowptr[i + 1];
    auto it = std::lower_bound(b, e, j);
    return static_cast<int32_t>(it - m.col.begin());
  };
  m.tslot.resize(m.col.size());
  for (int64_t i = 0; i < n; ++i)
    for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) m.tslot[s] = slot_of(m.col[s], (int32_t)i);
  // consistent mass: the element matrix |T|/12 (1 + delta_kl), the
  // off-diagonal part summed into the slots of the node graph
  m.cmass_d.assign(n, 0.0);
  m.cmass_o.assign(m.col.size(), 0.0);
  // boundary edges: an edge (a, b) seen in one triangle only
  std::vector<std::array<int64_t, 3>> edges;  // (min, max, triangle)
  edges.reserve(3 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    for (int k = 0; k < 3; ++k) {
      const int32_t a = v[k], b = v[(k + 1) % 3];
      m.cmass_d[a] += areas[t] / 6.0;
      m.cmass_o[slot_of(a, b)] += areas[t] / 12.0;
      m.cmass_o[slot_of(b, a)] += areas[t] / 12.0;
      edges.push_back({std::min(a, b), std::max(a, b), t});
    }
  }
  std::sort(edges.begin(), edges.end());
  std::vector<std::array<int64_t, 3>> bnd;  // boundary edges (a, b, third vertex)
  for (size_t k = 0; k < edges.size();) {
    size_t e = k + 1;
    while (e < edges.size() && edges[e][0] == edges[k][0] && edges[e][1] == edges[k][1]) ++e;
    if (e - k == 1) {
      const int64_t t = edges[k][2];
      int32_t third = tri[3 * t];
      for (int q = 0; q < 3; ++q)
        if (tri[3 * t + q] != edges[k][0] && tri[3 * t + q] != edges[k][1]) third = tri[3 * t + q];
      bnd.push_back({edges[k][0], edges[k][1], third});
    }
    k = e;
  }
  m.bnd_ptr.assign(n + 1, 0);
  for (const auto &b : bnd) {
    m.bnd_ptr[b[0] + 1]++;
    m.bnd_ptr[b[1] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) m.bnd_ptr[i + 1] += m.bnd_ptr[i];
  m.bnd_j.assign(m.bnd_ptr[n], 0);
  m.bnd_nl.assign(2 * m.bnd_ptr[n], 0.0);
  {
    std::vector<int64_t> f(m.bnd_ptr.begin(), m.bnd_ptr.end() - 1);
    for (const auto &b : bnd) {
      const double dx = xy[2 * b[1]] - xy[2 * b[0]], dy = xy[2 * b[1] + 1] - xy[2 * b[0] + 1];
      double nx = dy, ny = -dx;  // |(nx, ny)| = edge length
      const double ox = xy[2 * b[0]] - xy[2 * b[2]], oy = xy[2 * b[0] + 1] - xy[2 * b[2] + 1];
      if (ox * nx + oy * ny < 0) {  // point away from the third vertex
        nx = -nx;
        ny = -ny;
      }
      for (int side = 0; side < 2; ++side) {
        const int64_t i = b[side], r = f[i]++;
        m.bnd_j[r] = (int32_t)b[1 - side];
        m.bnd_nl[2 * r] = nx;
        m.bnd_nl[2 * r + 1] = ny;
      }
    }
  }
  // incidence records grouped by node
  m.inc_ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) m.inc_ptr[i + 1] = m.inc_ptr[i] + deg[i] / 2;
  const int64_t ninc = m.inc_ptr[n];
  m.inc_j.resize(ninc); m.inc_l.resize(ninc); m.inc_sj.resize(ninc); m.inc_sl.resize(ninc);
  m.inc_K.resize(3 * ninc);
  std::vector<int64_t> pos(m.inc_ptr.begin(), m.inc_ptr.end() - 1);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    const double *Kt = &K[6 * t];
    // full symmetric 3x3 from the 6 unique entries
    const double Kf[3][3] = {{Kt[0], Kt[3], Kt[4]}, {Kt[3], Kt[1], Kt[5]}, {Kt[4], Kt[5], Kt[2]}};
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      const int32_t i = v[k];
      const int64_t r = pos[i]++;
      m.inc_j[r] = v[k1];
      m.inc_l[r] = v[k2];
      m.inc_sj[r] = slot_of(i, v[k1]);
      m.inc_sl[r] = slot_of(i, v[k2]);
      m.inc_K[3 * r + 0] = Kf[k][k];
      m.inc_K[3 * r + 1] = Kf[k][k1];
      m.inc_K[3 * r + 2] = Kf[k][k2];
    }
  }
  // slot -> row and the incidence records that reach it (an edge lies in
  // one or two triangles of a conforming mesh)
  const int64_t ns = (int64_t)m.col.size();
  if (2 * ninc >= (int64_t)INT32_MAX) fail(SEIRD_ERR_MESH, "mesh too large for 32-bit incidence indices");
  m.slot_row.assign(ns, 0);
  m.slot_ek.assign(2 * ns, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) m.slot_row[s] = (int32_t)i;
    for (int64_t k = m.inc_ptr[i]; k < m.inc_ptr[i + 1]; ++k)
      for (int w = 0; w < 2; ++w) {
        const int32_t s = w == 0 ? m.inc_sj[k] : m.inc_sl[k];
        int32_t *e = &m.slot_ek[2 * (int64_t)s];
        if (e[0] < 0)
          e[0] = (int32_t)(2 * k + w);
        else if (e[1] < 0)
          e[1] = (int32_t)(2 * k + w);
        else
          fail(SEIRD_ERR_MESH, "an edge is shared by more than two triangles");
      }
  }
  m.kd.assign(n, 0.0);
  m.ko.assign(ns, 0.0);
  m.kw.assign(ns, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = m.inc_ptr[i]; k < m.inc_ptr[i + 1]; ++k) {
      m.kd[i] += m.inc_K[3 * k];
      m.ko[m.inc_sj[k]] += m.inc_K[3 * k + 1];
      m.ko[m.inc_sl[k]] += m.inc_K[3 * k + 2];
      m.kw[m.inc_sj[k]] += m.inc_K[3 * k];
      m.kw[m.inc_sl[k]] += m.inc_K[3 * k];
    }
}

// Reverse Cuthill-McKee ordering of an induced subgraph given as a local
// CSR (adjacency excluding self).  Returns perm (position -> local node).
static std::vector<int32_t> rcm(const std::vector<int32_t> &ptr, const std::vector<int32_t> &adj) {
  const int32_t nn = (int32_t)ptr.size() - 1;
  std::vector<int32_t> perm;
  perm.reserve(nn);
  std::vector<char> seen(nn, 0);
  std::vector<int32_t> level(nn, -1);
  auto degree = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };
  auto bfs_far = [&](int32_t s, std::vector<int32_t> &comp) {
    // returns the last node of a BFS from s (a node of maximal level,
    // smallest degree among those); fills comp with the component
    comp.clear();
    std::queue<int32_t> q;
    q.push(s);
    level[s] = 0;
    comp.push_back(s);
    while (!q.empty()) {
      int32_t v = q.front();
      q.pop();
      for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
        int32_t w = adj[k];
        if (level[w] < 0) {
          level[w] = level[v] + 1;
          q.push(w);
          comp.push_back(w);
        }
      }
    }
    int32_t best = s;
    for (int32_t v : comp)
      if (level[v] > level[best] || (level[v] == level[best] && degree(v) < degree(best))) best = v;
    int32_t ecc = level[best];
    for (int32_t v : comp) level[v] = -1;
    return std::make_pair(best, ecc);
  };
  std::vector<int32_t> comp;
  for (int32_t s0 = 0; s0 < nn; ++s0) {
    if (seen[s0]) continue;
    // pseudo-peripheral start node (George-Liu style)
    int32_t s = s0;
    auto r = bfs_far(s, comp);
    int32_t ecc = -1;
    for (int it = 0; it < 4 && r.second > ecc; ++it) {
      ecc = r.second;
      s = r.first;
      r = bfs_far(s, comp);
    }
    // Cuthill-McKee from s
    std::vector<int32_t> cm;
    cm.push_back(s);
    seen[s] = 1;
    std::vector<int32_t> nb;
    for (size_t h = 0; h < cm.size(); ++h) {
      int32_t v = cm[h];
      nb.clear();
      for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k)
        if (!seen[adj[k]]) {
          nb.push_back(adj[k]);
          seen[adj[k]] = 1;
        }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return degree(a) != degree(b) ? degree(a) < degree(b) : a < b;
      });
      cm.insert(cm.end(), nb.begin(), nb.end());
    }
    std::reverse(cm.begin(), cm.end());
    perm.insert(perm.end(), cm.begin(), cm.end());
  }
  return perm;
}

// Strip ordering: nodes sorted along the principal axis of their point
// cloud (ties by the other coordinate, then by index).  On a compact 2D
// patch its bandwidth is about the node count across the short side.
static std::vector<int32_t> strip_order(const std::vector<double> &pts) {
  const int32_t nn = (int32_t)(pts.size() / 2);
  double mx = 0, my = 0;
  for (int32_t k = 0; k < nn; ++k) { mx += pts[2 * k]; my += pts[2 * k + 1]; }
  mx /= std::max(nn, 1); my /= std::max(nn, 1);
  double sxx = 0, sxy = 0, syy = 0;
  for (int32_t k = 0; k < nn; ++k) {
    const double dx = pts[2 * k] - mx, dy = pts[2 * k + 1] - my;
    sxx += dx * dx; sxy += dx * dy; syy += dy * dy;
  }
  // principal direction of the 2x2 covariance
  const double th = 0.5 * std::atan2(2 * sxy, sxx - syy);
  const double ux = std::cos(th), uy = std::sin(th);
  std::vector<double> key(nn), key2(nn);
  for (int32_t k = 0; k < nn; ++k) {
    key[k] = ux * pts[2 * k] + uy * pts[2 * k + 1];
    key2[k] = -uy * pts[2 * k] + ux * pts[2 * k + 1];
  }
  std::vector<int32_t> perm(nn);
  std::iota(perm.begin(), perm.end(), 0);
  std::sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    if (key[a] != key[b]) return key[a] < key[b];
    if (key2[a] != key2[b]) return key2[a] < key2[b];
    return a < b;
  });
  return perm;
}

static int32_t bandwidth_of(const std::vector<int32_t> &perm, const std::vector<int32_t> &lp,
                            const std::vector<int32_t> &la) {
  const int32_t nn = (int32_t)perm.size();
  std::vector<int32_t> where(nn);
  for (int32_t k = 0; k < nn; ++k) where[perm[k]] = k;
  int32_t bw = 0;
  for (int32_t k = 0; k < nn; ++k)
    for (int32_t q = lp[k]; q < lp[k + 1]; ++q) bw = std::max(bw, std::abs(where[k] - where[la[q]]));
  return bw;
}

// the smaller-bandwidth one of reverse Cuthill-McKee and the strip ordering
static std::vector<int32_t> band_order(const std::vector<int32_t> &lp, const std::vector<int32_t> &la,
                                       const std::vector<double> &pts) {
  std::vector<int32_t> a = rcm(lp, la);
  std::vector<int32_t> b = strip_order(pts);
  return bandwidth_of(b, lp, la) < bandwidth_of(a, lp, la) ? b : a;
}

static SubInfo tile_geometry(int32_t nn, int32_t bw, int tile, int bs = NC) {
  SubInfo si{};
  si.n_loc = bs * nn;
  const int32_t kl = bs * bw + bs - 1;
  si.nt = (si.n_loc + tile - 1) / tile;
  si.bl = std::min<int32_t>((kl + tile - 1) / tile, si.nt - 1);
  si.bu = si.bl;
  si.env_off = -1;
  return si;
}

// Tile envelope of a subdomain matrix in the local order (node position k
// holds unknowns bs k .. bs k + bs - 1, full bs x bs node blocks; bs = 5 for
// the coupled system, 1 for one compartment): lo[K] = first tile
// column of tile row K, made nondecreasing (suffix minimum) so that the
// envelope is closed under elimination; row[K] = tile offset of row K,
// whose tiles are the columns lo[K] .. hi[K] with hi[K] = max{J : lo[J] <=
// K}.  Sets si.bl = si.bu to the largest extent.
static void tile_envelope(const std::vector<int32_t> &lp, const std::vector<int32_t> &la,
                          const std::vector<int32_t> &perm, const std::vector<int32_t> &where, int tile,
                          SubInfo &si, std::vector<int32_t> &lo, std::vector<int32_t> &row, int bs) {
  const int32_t nn = (int32_t)perm.size(), nt = si.nt;
  lo.assign(nt, 0);
  for (int32_t K = 0; K < nt; ++K) lo[K] = K;
  for (int32_t k = 0; k < nn; ++k) {
    int32_t left = k;
    for (int32_t q = lp[perm[k]]; q < lp[perm[k] + 1]; ++q) left = std::min(left, where[la[q]]);
    const int32_t K = (bs * k) / tile, K2 = (bs * k + bs - 1) / tile;  // tile rows of the node's unknowns
    const int32_t J = (bs * left) / tile;
    lo[K] = std::min(lo[K], J);
    lo[K2] = std::min(lo[K2], J);
  }
  for (int32_t K = nt - 2; K >= 0; --K) lo[K] = std::min(lo[K], lo[K + 1]);
  row.assign(nt + 1, 0);
  int32_t bl = 0, bu = 0, J = 0;
  for (int32_t K = 0; K < nt; ++K) {
    while (J + 1 < nt && lo[J + 1] <= K) ++J;
    const int32_t hi = std::max(J, K);
    row[K + 1] = row[K] + (hi - lo[K] + 1);
    bl = std::max(bl, K - lo[K]);
    bu = std::max(bu, hi - K);
  }
  si.bl = bl;
  si.bu = bu;
}

void build_precond(const MeshHost &m, const seird_schwarz_opts &o, const int32_t *part,
                   PrecondHost &ph, int bs) {
  const int64_t n = m.n;
  if (bs != NC && bs != 1) fail(SEIRD_ERR_ARG, "internal: block size must be 1 or 5");
  if (bs != NC && o.n_ref > 0) fail(SEIRD_ERR_ARG, "the compartment-wise preconditioner is one-level");
  ph.bs = bs;
  if (o.n_sub <= 0 || o.overlap < 0 || !part) fail(SEIRD_ERR_ARG, "bad Schwarz options");
  if (o.tile != 16 && o.tile != 32) fail(SEIRD_ERR_ARG, "tile must be 16 or 32");
  if (o.factor_prec < 0 || o.factor_prec > 2) fail(SEIRD_ERR_ARG, "factor_prec must be 0, 1 or 2");
  ph.n_sub = o.n_sub;
  ph.overlap = o.overlap;
  ph.tile = o.tile;
  ph.prec = o.factor_prec;
  std::vector<std::vector<int32_t>> owned(o.n_sub);
  for (int64_t i = 0; i < n; ++i) {
    if (part[i] < 0 || part[i] >= o.n_sub) fail(SEIRD_ERR_ARG, "partition entry out of range");
    owned[part[i]].push_back((int32_t)i);
  }
  for (int s = 0; s < o.n_sub; ++s)
    if (owned[s].empty()) fail(SEIRD_ERR_ARG, "subdomain " + std::to_string(s) + " owns no node");
  std::vector<int32_t> stamp(n, -1), lpos(n, -1);
  const int t = o.tile;
  int64_t base = 0;
  ph.trow_ptr.assign(1, 0);
  for (int s = 0; s < o.n_sub; ++s) {
    // overlap growth: `overlap` layers of graph neighbours
    std::vector<int32_t> nodes = owned[s];
    for (int32_t v : nodes) stamp[v] = s;
    size_t front_b = 0;
    for (int layer = 0; layer < o.overlap; ++layer) {
      size_t front_e = nodes.size();
      for (size_t h = front_b; h < front_e; ++h) {
        int32_t v = nodes[h];
        for (int64_t k = m.rowptr[v]; k < m.rowptr[v + 1]; ++k) {
          int32_t w = m.col[k];
          if (stamp[w] != s) {
            stamp[w] = s;
            nodes.push_back(w);
          }
        }
      }
      front_b = front_e;
    }
    std::sort(nodes.begin(), nodes.end());
    const int32_t nn = (int32_t)nodes.size();
    for (int32_t k = 0; k < nn; ++k) lpos[nodes[k]] = k;
    // induced subgraph CSR
    std::vector<int32_t> lp(nn + 1, 0), la;
    for (int32_t k = 0; k < nn; ++k) {
      int32_t v = nodes[k];
      for (int64_t q = m.rowptr[v]; q < m.rowptr[v + 1]; ++q)
        if (stamp[m.col[q]] == s) la.push_back(lpos[m.col[q]]);
      lp[k + 1] = (int32_t)la.size();
    }
    std::vector<double> pts(2 * (size_t)nn);
    for (int32_t k = 0; k < nn; ++k) {
      pts[2 * k] = m.xy[2 * (size_t)nodes[k]];
      pts[2 * k + 1] = m.xy[2 * (size_t)nodes[k] + 1];
    }
    std::vector<int32_t> perm = band_order(lp, la, pts);
    std::vector<int32_t> where(nn);
    for (int32_t k = 0; k < nn; ++k) where[perm[k]] = k;
    int32_t bw = 0;
    for (int32_t k = 0; k < nn; ++k)
      for (int32_t q = lp[k]; q < lp[k + 1]; ++q) bw = std::max(bw, std::abs(where[k] - where[la[q]]));
    SubInfo si = tile_geometry(nn, bw, t, bs);
    std::vector<int32_t> elo, erow;
    tile_envelope(lp, la, perm, where, t, si, elo, erow, bs);
    si.base = base;
    si.l2g_off = (int32_t)ph.l2g.size();
    si.env_off = (int32_t)ph.env_row.size();
    ph.env_row.insert(ph.env_row.end(), erow.begin(), erow.end());
    ph.env_lo.insert(ph.env_lo.end(), elo.begin(), elo.end());
    ph.env_lo.push_back(0);  // same length as the row offsets
    base += (int64_t)erow[si.nt] * t * t;
    ph.max_nodes = std::max(ph.max_nodes, nn);
    ph.max_bw = std::max(ph.max_bw, bw);
    ph.mean_bw += (double)bw / o.n_sub;
    ph.max_nloc = std::max(ph.max_nloc, si.n_loc);
    // local unknown map and ownership, in the local (RCM) order
    for (int32_t k = 0; k < nn; ++k) {
      int32_t g = nodes[perm[k]];
      for (int c = 0; c < bs; ++c) {
        ph.l2g.push_back(bs * g + c);
        ph.owned.push_back(part[g] == s ? 1 : 0);
      }
    }
    // extraction entries (row block p, column block q), node by node; each
    // block must lie inside the stored tiles of its rows
    for (int32_t k = 0; k < nn; ++k) {
      int32_t g = nodes[perm[k]];
      ph.ent_ptr.push_back((int32_t)ph.extract.size());
      ph.extract.push_back({s, k, k, -g - 1});
      for (int64_t q = m.rowptr[g]; q < m.rowptr[g + 1]; ++q) {
        int32_t h = m.col[q];
        if (stamp[h] == s) ph.extract.push_back({s, k, where[lpos[h]], (int32_t)q});
      }
      for (size_t e = ph.ent_ptr.back(); e < ph.extract.size(); ++e) {
        const int32_t J0 = bs * ph.extract[e].q / t, J1 = (bs * ph.extract[e].q + bs - 1) / t;
        for (int32_t K = bs * k / t; K <= (bs * k + bs - 1) / t; ++K)
          if (J0 < elo[K] || J1 >= elo[K] + (erow[K + 1] - erow[K]))
            fail(SEIRD_ERR_ARG, "internal: local matrix entry outside the stored tiles");
      }
      if (ph.extract.size() >= (size_t)INT32_MAX) fail(SEIRD_ERR_ARG, "too many local matrix blocks");
      ph.max_node_blocks = std::max(ph.max_node_blocks, (int32_t)(ph.extract.size() - ph.ent_ptr.back()));
    }
    {
      // step K: panels of nu tiles right of the diagonal and nu below it
      // (the envelope is symmetric), then nu x nu Schur products
      const double T3 = (double)t * t * t;
      for (int32_t K = 0; K < si.nt; ++K) {
        const double nu = (double)(elo[K] + (erow[K + 1] - erow[K]) - 1 - K);
        ph.lu_mfma_flops += 2.0 * T3 * (2.0 * nu + nu * nu);
        ph.lu_useful_flops += T3 * (2.0 * nu + 2.0 * nu * nu) + 4.0 / 3.0 * T3;
      }
    }
    ph.trow_ptr.push_back(ph.trow_ptr.back() + si.nt);
    ph.trow_sub.insert(ph.trow_sub.end(), si.nt, s);
    ph.subs.push_back(si);
  }
  ph.factor_entries = base;
  ph.ent_ptr.push_back((int32_t)ph.extract.size());
  // largest subdomains first (longest-processing-time order)
  ph.order.resize(o.n_sub);
  std::iota(ph.order.begin(), ph.order.end(), 0);
  std::stable_sort(ph.order.begin(), ph.order.end(), [&](int a, int b) {
    // work ~ stored tiles times the band width
    const SubInfo &x = ph.subs[a], &y = ph.subs[b];
    const int64_t tx = ph.env_row[x.env_off + x.nt], ty = ph.env_row[y.env_off + y.nt];
    return tx * (x.bu + 1) > ty * (y.bu + 1);
  });

  // ------------------------------------------------------------------
  // two-grid coarse space (nested P1 interpolation, Galerkin product)
  // ------------------------------------------------------------------
  if (o.n_ref <= 0) return;
  if (!o.level_n || !o.parents) fail(SEIRD_ERR_ARG, "two-level needs level_n and parents");
  if (o.level_n[o.n_ref] != n) fail(SEIRD_ERR_ARG, "finest refinement level must match the mesh");
  ph.two_level = true;
  const int64_t nc = o.level_n[0];
  if (nc <= 0) fail(SEIRD_ERR_ARG, "empty coarse level");
  ph.nc = nc;
  // Z rows as sparse vectors, level by level
  std::vector<int64_t> zp(nc + 1);
  std::vector<int32_t> zc(nc);
  std::vector<double> zv(nc, 1.0);
  for (int64_t i = 0; i <= nc; ++i) zp[i] = i;
  for (int64_t i = 0; i < nc; ++i) zc[i] = (int32_t)i;
  const int32_t *par = o.parents;
  for (int r = 1; r <= o.n_ref; ++r) {
    const int64_t nl = o.level_n[r], nprev = o.level_n[r - 1];
    std::vector<int64_t> np(nl + 1, 0);
    std::vector<int32_t> nc_;
    std::vector<double> nv;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t a = 0; a < nl; ++a) {
      int32_t p = par[2 * a], q = par[2 * a + 1];
      if (p < 0 || q < 0 || p >= nprev || q >= nprev) fail(SEIRD_ERR_ARG, "refinement record out of range");
      row.clear();
      for (int64_t k = zp[p]; k < zp[p + 1]; ++k) row.push_back({zc[k], 0.5 * zv[k]});
      for (int64_t k = zp[q]; k < zp[q + 1]; ++k) row.push_back({zc[k], 0.5 * zv[k]});
      std::sort(row.begin(), row.end());
      for (size_t k = 0; k < row.size(); ++k) {
        if (!nc_.empty() && (int64_t)nc_.size() > np[a] && nc_.back() == row[k].first)
          nv.back() += row[k].second;
        else {
          nc_.push_back(row[k].first);
          nv.push_back(row[k].second);
        }
      }
      np[a + 1] = (int64_t)nc_.size();
    }
    par += 2 * nl;
    zp.swap(np);
    zc.swap(nc_);
    zv.swap(nv);
  }
  ph.z_ptr = zp;
  ph.z_col = zc;
  ph.z_val = zv;
  // Z^T
  ph.zt_ptr.assign(nc + 1, 0);
  for (int32_t c : zc) ph.zt_ptr[c + 1]++;
  for (int64_t i = 0; i < nc; ++i) ph.zt_ptr[i + 1] += ph.zt_ptr[i];
  ph.zt_col.resize(zc.size());
  ph.zt_val.resize(zc.size());
  {
    std::vector<int64_t> f(ph.zt_ptr.begin(), ph.zt_ptr.end() - 1);
    for (int64_t a = 0; a < n; ++a)
      for (int64_t k = zp[a]; k < zp[a + 1]; ++k) {
        ph.zt_col[f[zc[k]]] = (int32_t)a;
        ph.zt_val[f[zc[k]]++] = zv[k];
      }
  }
  // Galerkin contributions per coarse row I: for fine a in supp(I) and fine
  // b in {a} U adj(a), every J in Z row b gets w = Z_aI Z_bJ times block (a,b)
  std::vector<int64_t> cptr(nc + 1, 0);
  std::vector<int32_t> cadj;  // coarse graph (including self)
  struct Contrib { int32_t J; int32_t ref; double w; };
  std::vector<std::vector<Contrib>> rows(nc);
  std::vector<Contrib> tmp;
  for (int64_t I = 0; I < nc; ++I) {
    tmp.clear();
    for (int64_t k = ph.zt_ptr[I]; k < ph.zt_ptr[I + 1]; ++k) {
      const int32_t a = ph.zt_col[k];
      const double wa = ph.zt_val[k];
      for (int64_t kb = zp[a]; kb < zp[a + 1]; ++kb) tmp.push_back({zc[kb], -a - 1, wa * zv[kb]});
      for (int64_t q = m.rowptr[a]; q < m.rowptr[a + 1]; ++q) {
        const int32_t b = m.col[q];
        for (int64_t kb = zp[b]; kb < zp[b + 1]; ++kb) tmp.push_back({zc[kb], (int32_t)q, wa * zv[kb]});
      }
    }
    std::stable_sort(tmp.begin(), tmp.end(), [](const Contrib &x, const Contrib &y) { return x.J < y.J; });
    rows[I] = tmp;
    for (size_t k = 0; k < tmp.size(); ++k)
      if (k == 0 || tmp[k].J != tmp[k - 1].J) cadj.push_back(tmp[k].J);
    cptr[I + 1] = (int64_t)cadj.size();
  }
  // coarse RCM ordering over the coarse graph without self loops
  std::vector<int32_t> lp(nc + 1, 0), la;
  for (int64_t I = 0; I < nc; ++I) {
    for (int64_t k = cptr[I]; k < cptr[I + 1]; ++k)
      if (cadj[k] != I) la.push_back(cadj[k]);
    lp[I + 1] = (int32_t)la.size();
  }
  // coarse node positions: Z-weighted mean of the fine nodes they support
  std::vector<double> cpts(2 * (size_t)nc, 0.0);
  for (int64_t I = 0; I < nc; ++I) {
    double wsum = 0, x = 0, y = 0;
    for (int64_t k = ph.zt_ptr[I]; k < ph.zt_ptr[I + 1]; ++k) {
      const double w = ph.zt_val[k];
      x += w * m.xy[2 * (size_t)ph.zt_col[k]];
      y += w * m.xy[2 * (size_t)ph.zt_col[k] + 1];
      wsum += w;
    }
    cpts[2 * I] = x / wsum;
    cpts[2 * I + 1] = y / wsum;
  }
  std::vector<int32_t> perm = band_order(lp, la, cpts);
  ph.c_perm.assign(nc, 0);
  for (int64_t k = 0; k < nc; ++k) ph.c_perm[perm[k]] = (int32_t)k;
  int32_t bw = 0;
  for (int64_t I = 0; I < nc; ++I)
    for (int64_t k = cptr[I]; k < cptr[I + 1]; ++k)
      bw = std::max(bw, std::abs(ph.c_perm[I] - ph.c_perm[cadj[k]]));
  ph.coarse = tile_geometry((int32_t)nc, bw, t);
  ph.coarse_bw = bw;
  ph.coarse.base = 0;
  ph.coarse.l2g_off = -1;
  ph.coarse_entries = (int64_t)ph.coarse.nt * (ph.coarse.bl + ph.coarse.bu + 1) * t * t;
  ph.gal_ptr.push_back(0);
  for (int64_t I = 0; I < nc; ++I) {
    const auto &rw = rows[I];
    for (size_t k = 0; k < rw.size(); ++k) {
      if (k == 0 || rw[k].J != rw[k - 1].J) {
        if (k > 0) ph.gal_ptr.push_back((int64_t)ph.gal_ref.size());
        ph.gal_p.push_back(ph.c_perm[I]);
        ph.gal_q.push_back(ph.c_perm[rw[k].J]);
      }
      ph.gal_ref.push_back(rw[k].ref);
      ph.gal_w.push_back(rw[k].w);
    }
    if (!rw.empty()) ph.gal_ptr.push_back((int64_t)ph.gal_ref.size());
    std::vector<Contrib>().swap(rows[I]);
  }
  // coarse graph over positions (sorted neighbour lists), node points and
  // owners: the owner of coarse node I is the subdomain of the fine node
  // with the largest weight in column I of Z (the node itself when nested)
  {
    std::vector<std::vector<int32_t>> nb(nc);
    for (int64_t I = 0; I < nc; ++I)
      for (int64_t k = cptr[I]; k < cptr[I + 1]; ++k)
        if (cadj[k] != I) nb[ph.c_perm[I]].push_back(ph.c_perm[cadj[k]]);
    ph.cg_rowptr.assign(nc + 1, 0);
    ph.cg_xy.assign(2 * (size_t)nc, 0.0);
    ph.cg_owner.assign(nc, 0);
    for (int64_t p = 0; p < nc; ++p) {
      std::sort(nb[p].begin(), nb[p].end());
      ph.cg_col.insert(ph.cg_col.end(), nb[p].begin(), nb[p].end());
      ph.cg_rowptr[p + 1] = (int64_t)ph.cg_col.size();
    }
    for (int64_t I = 0; I < nc; ++I) {
      const int32_t p = ph.c_perm[I];
      ph.cg_xy[2 * (size_t)p] = cpts[2 * I];
      ph.cg_xy[2 * (size_t)p + 1] = cpts[2 * I + 1];
      double wbest = -1.0;
      int32_t abest = -1;
      for (int64_t k = ph.zt_ptr[I]; k < ph.zt_ptr[I + 1]; ++k)
        if (ph.zt_val[k] > wbest) {
          wbest = ph.zt_val[k];
          abest = ph.zt_col[k];
        }
      if (abest < 0) fail(SEIRD_ERR_ARG, "coarse node with an empty interpolation column");
      ph.cg_owner[p] = part[abest];
    }
    ph.gal_dst.resize(ph.gal_p.size());
    for (size_t k = 0; k < ph.gal_p.size(); ++k) {
      const int32_t p = ph.gal_p[k], q = ph.gal_q[k];
      if (p == q) {
        ph.gal_dst[k] = -p - 1;
        continue;
      }
      const auto b = ph.cg_col.begin() + ph.cg_rowptr[p], e = ph.cg_col.begin() + ph.cg_rowptr[p + 1];
      const auto it = std::lower_bound(b, e, q);
      if (it == e || *it != q) fail(SEIRD_ERR_ARG, "internal: Galerkin block outside the coarse graph");
      ph.gal_dst[k] = (int32_t)(it - ph.cg_col.begin());
    }
  }
}

}  // namespace seird
