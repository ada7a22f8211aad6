// Host combinatorics of the dual-primal split (integer work, bit-exact).
//
// Sec. 3: the insulating region is gauged by a spanning tree of the control
// mesh grown over the wirebasket first, then the subdomain faces, then the
// subdomain interiors; tree edges inside the insulator are eliminated,
// interface tree edges become primal, all other kept edges are remainder
// unknowns.  For many patches and floating conductors the rule is applied to
// the contracted insulator graph H (root = outer boundary plus every
// conductor component touching it, one super-vertex per floating conductor
// component, every other node plain), so the eliminated set is exactly a
// spanning tree of H and never closes a loop through a conductor.
// Primal = per-interface-face trees of conductor/insulator faces plus every
// non-Dirichlet wirebasket edge outside the gauge tree.  Dual = the remaining
// face-interior edges of interior faces (one multiplier each, ordered by edge
// id, +1 on the lower patch id).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <numeric>
#include <sstream>

#include "tcf_internal.h"

namespace tcf {

std::string validate_desc(const tcf_problem_desc& d) {
  std::ostringstream err;
  for (int a = 0; a < 3; ++a) {
    if (d.np[a] < 1) { err << "np[" << a << "] < 1"; return err.str(); }
    if (!d.breaks[a] || !d.nel[a] || !d.deg[a]) { err << "null row array in direction " << a; return err.str(); }
    for (int r = 0; r < d.np[a]; ++r) {
      if (!(d.breaks[a][r + 1] > d.breaks[a][r])) { err << "breaks[" << a << "] not increasing"; return err.str(); }
      if (d.nel[a][r] < 1) { err << "nel[" << a << "][" << r << "] < 1"; return err.str(); }
      if (d.deg[a][r] < 1 || d.deg[a][r] > 8) { err << "deg[" << a << "][" << r << "] outside 1..8"; return err.str(); }
    }
  }
  int64_t np = (int64_t)d.np[0] * d.np[1] * d.np[2];
  if (!d.sigma || !d.nu || !d.src_mask) return "null sigma/nu/src_mask";
  for (int64_t s = 0; s < np; ++s) {
    if (!(d.sigma[s] >= 0) || !std::isfinite(d.sigma[s])) { err << "sigma[" << s << "] < 0"; return err.str(); }
    if (!(d.nu[s] > 0) || !std::isfinite(d.nu[s])) { err << "nu[" << s << "] <= 0"; return err.str(); }
  }
  if (d.n_rhs < 1) return "n_rhs < 1";
  if (!(d.dt > 0)) return "dt <= 0";
  if (d.n_steps < 0) return "n_steps < 0";
  if (d.n_steps > 0 && !d.amp) return "null amp";
  bool any_src = false;
  for (int64_t s = 0; s < np; ++s) any_src |= d.src_mask[s] != 0;
  if (any_src && !d.phi && !d.jvol) return "source mask set but neither phi nor jvol given";
  return "";
}

Grid build_grid(const tcf_problem_desc& d) {
  Grid g;
  for (int a = 0; a < 3; ++a) {
    g.P[a] = d.np[a];
    int64_t o = 0;
    for (int r = 0; r < d.np[a]; ++r) {
      int m = d.nel[a][r] + d.deg[a][r];
      g.m[a].push_back(m);
      g.off[a].push_back(o);
      o += m - 1;
    }
    g.N[a] = o + 1;
    g.on_plane[a].assign(g.N[a], 0);
    for (int r = 0; r < d.np[a]; ++r) g.on_plane[a][g.off[a][r]] = 1;
    g.on_plane[a][g.N[a] - 1] = 1;
  }
  g.Ex = (g.N[0] - 1) * g.N[1] * g.N[2];
  g.Ey = g.N[0] * (g.N[1] - 1) * g.N[2];
  g.Ez = g.N[0] * g.N[1] * (g.N[2] - 1);
  return g;
}

namespace {

struct Box { int64_t lo[3], hi[3]; };  // inclusive node ranges

Box patch_box(const Grid& g, int i, int j, int k) {
  Box b;
  int ijk[3] = {i, j, k};
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = g.off[a][ijk[a]];
    b.hi[a] = b.lo[a] + g.m[a][ijk[a]] - 1;
  }
  return b;
}

// Calls f(edge_id) for every edge whose both nodes lie in the box.
template <class F>
void for_box_edges(const Grid& g, const Box& b, F&& f) {
  for (int d = 0; d < 3; ++d) {
    int64_t hi[3] = {b.hi[0], b.hi[1], b.hi[2]};
    hi[d] -= 1;
    for (int64_t K = b.lo[2]; K <= hi[2]; ++K)
      for (int64_t J = b.lo[1]; J <= hi[1]; ++J)
        for (int64_t I = b.lo[0]; I <= hi[0]; ++I) f(g.edge_id(d, I, J, K));
  }
}

struct UnionFind {
  std::vector<int> p;
  explicit UnionFind(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int find(int a) { while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; } return a; }
  void unite(int a, int b) { a = find(a); b = find(b); if (a != b) p[std::max(a, b)] = std::min(a, b); }
};

// BFS over an adjacency list whose per-vertex lists are sorted by edge id.
void bfs(const std::vector<int64_t>& start, const std::vector<int64_t>& nbr_edge,
         const std::vector<int64_t>& nbr_vert, std::vector<uint8_t>& visited,
         const std::vector<int64_t>& seeds, std::vector<int64_t>& tree) {
  std::vector<int64_t> queue(seeds.begin(), seeds.end());
  size_t head = 0;
  while (head < queue.size()) {
    int64_t v = queue[head++];
    for (int64_t k = start[v]; k < start[v + 1]; ++k) {
      int64_t u = nbr_vert[k];
      if (!visited[u]) {
        visited[u] = 1;
        tree.push_back(nbr_edge[k]);
        queue.push_back(u);
      }
    }
  }
}

// Adjacency in CSR form from an edge list given in increasing edge id, so
// each vertex's list is sorted by edge id.
void build_adjacency(int64_t nV, const std::vector<int64_t>& eid, const std::vector<int64_t>& va,
                     const std::vector<int64_t>& vb, std::vector<int64_t>& start,
                     std::vector<int64_t>& nbr_edge, std::vector<int64_t>& nbr_vert) {
  start.assign(nV + 1, 0);
  for (size_t k = 0; k < eid.size(); ++k) { start[va[k] + 1]++; start[vb[k] + 1]++; }
  for (int64_t v = 0; v < nV; ++v) start[v + 1] += start[v];
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  nbr_edge.assign(start[nV], 0);
  nbr_vert.assign(start[nV], 0);
  for (size_t k = 0; k < eid.size(); ++k) {
    int64_t a = va[k], b = vb[k];
    nbr_edge[fill[a]] = eid[k]; nbr_vert[fill[a]++] = b;
    nbr_edge[fill[b]] = eid[k]; nbr_vert[fill[b]++] = a;
  }
}

}  // namespace

std::string compute_topology(const tcf_problem_desc& d, const Grid& g, Topology& t,
                             std::vector<PatchPlan>& plans) {
  const int P0 = g.P[0], P1 = g.P[1], P2 = g.P[2];
  const int np = P0 * P1 * P2;
  const int64_t nE = g.n_edges(), nN = g.n_nodes();

  // ---- per-edge flags: Dirichlet, class, conductor closure -------------
  std::vector<uint8_t> dir(nE, 0), cls(nE, 0), cond(nE, 0);
  for (int64_t e = 0; e < nE; ++e) {
    int dd; int64_t I, J, K;
    g.edge_decode(e, dd, I, J, K);
    bool b0 = g.node_boundary(I, J, K);
    bool b1 = g.node_boundary(I + (dd == 0), J + (dd == 1), K + (dd == 2));
    dir[e] = b0 && b1;
    int hits = 0;
    if (dd != 0) hits += g.on_plane[0][I];
    if (dd != 1) hits += g.on_plane[1][J];
    if (dd != 2) hits += g.on_plane[2][K];
    cls[e] = hits == 2 ? kWirebasket : (hits == 1 ? kFace : kInterior);
  }
  auto pid = [&](int i, int j, int k) { return i + P0 * (j + P1 * k); };
  for (int k = 0; k < P2; ++k)
    for (int j = 0; j < P1; ++j)
      for (int i = 0; i < P0; ++i)
        if (d.sigma[pid(i, j, k)] > 0)
          for_box_edges(g, patch_box(g, i, j, k), [&](int64_t e) { cond[e] = 1; });

  // ---- vertices of the contracted insulator graph H --------------------
  UnionFind uf(np);
  for (int s = 0; s < np; ++s) {
    if (!(d.sigma[s] > 0)) continue;
    int i = s % P0, j = (s / P0) % P1, k = s / (P0 * P1);
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          int a = i + di, b = j + dj, c = k + dk;
          if (a < 0 || b < 0 || c < 0 || a >= P0 || b >= P1 || c >= P2) continue;
          int s2 = pid(a, b, c);
          if (d.sigma[s2] > 0) uf.unite(s, s2);
        }
  }
  std::vector<int64_t> node_vertex(nN, -1);
  for (int64_t K = 0; K < g.N[2]; ++K)
    for (int64_t J = 0; J < g.N[1]; ++J)
      for (int64_t I = 0; I < g.N[0]; ++I)
        if (g.node_boundary(I, J, K)) node_vertex[g.node_id(I, J, K)] = 0;
  // components: root patch -> (touches boundary, smallest member node id)
  std::vector<int> comp_roots;
  std::vector<uint8_t> touches(np, 0);
  std::vector<int64_t> minnode(np, INT64_MAX);
  for (int s = 0; s < np; ++s) {
    if (!(d.sigma[s] > 0)) continue;
    int r = uf.find(s);
    int i = s % P0, j = (s / P0) % P1, k = s / (P0 * P1);
    if (i == 0 || j == 0 || k == 0 || i == P0 - 1 || j == P1 - 1 || k == P2 - 1) touches[r] = 1;
    Box b = patch_box(g, i, j, k);
    minnode[r] = std::min(minnode[r], g.node_id(b.lo[0], b.lo[1], b.lo[2]));
    if (r == s) comp_roots.push_back(s);
  }
  std::vector<int> floating;
  for (int r : comp_roots)
    if (!touches[r]) floating.push_back(r);
  std::sort(floating.begin(), floating.end(), [&](int a, int b) { return minnode[a] < minnode[b]; });
  std::vector<int64_t> comp_vertex(np, -1);
  for (int r : comp_roots) comp_vertex[r] = 0;
  for (size_t f = 0; f < floating.size(); ++f) comp_vertex[floating[f]] = 1 + (int64_t)f;
  for (int s = 0; s < np; ++s) {
    if (!(d.sigma[s] > 0)) continue;
    int64_t v = comp_vertex[uf.find(s)];
    int i = s % P0, j = (s / P0) % P1, k = s / (P0 * P1);
    Box b = patch_box(g, i, j, k);
    for (int64_t K = b.lo[2]; K <= b.hi[2]; ++K)
      for (int64_t J = b.lo[1]; J <= b.hi[1]; ++J)
        for (int64_t I = b.lo[0]; I <= b.hi[0]; ++I) {
          int64_t n = g.node_id(I, J, K);
          if (v == 0) {
            node_vertex[n] = 0;
          } else {
            if (node_vertex[n] == 0) return "floating conductor component overlaps the root";
            node_vertex[n] = v;
          }
        }
  }
  int64_t nV = 1 + (int64_t)floating.size();
  int64_t n_plain = 0;
  for (int64_t n = 0; n < nN; ++n)
    if (node_vertex[n] < 0) { node_vertex[n] = nV++; ++n_plain; }

  // ---- phased BFS: wirebasket, faces, interiors ------------------------
  std::vector<uint8_t> visited(nV, 0);
  visited[0] = 1;
  std::vector<int64_t> tree;
  for (int phase = 0; phase < 3; ++phase) {
    std::vector<int64_t> eid, va, vb;
    for (int64_t e = 0; e < nE; ++e) {
      if (dir[e] || cond[e] || cls[e] != phase) continue;
      int64_t tl, hd;
      g.edge_nodes(e, tl, hd);
      int64_t a = node_vertex[tl], b = node_vertex[hd];
      if (a == b) continue;
      eid.push_back(e); va.push_back(a); vb.push_back(b);
    }
    std::vector<int64_t> start, ne, nv;
    build_adjacency(nV, eid, va, vb, start, ne, nv);
    std::vector<int64_t> seeds;
    if (phase == 0) seeds.push_back(0);
    else for (int64_t v = 0; v < nV; ++v) if (visited[v]) seeds.push_back(v);
    bfs(start, ne, nv, visited, seeds, tree);
  }
  for (int64_t v = 0; v < nV; ++v)
    if (!visited[v]) return "gauge tree does not span the insulator graph";
  std::sort(tree.begin(), tree.end());
  if ((int64_t)tree.size() != nV - 1) return "gauge tree size mismatch";
  std::vector<uint8_t> in_tree(nE, 0);
  for (int64_t e : tree) in_tree[e] = 1;

  // ---- interface (conductor/insulator) face trees ----------------------
  std::vector<int64_t> gamma;
  for (int s = 0; s < np; ++s) {
    int ijk[3] = {s % P0, (s / P0) % P1, s / (P0 * P1)};
    for (int dd = 0; dd < 3; ++dd) {
      if (ijk[dd] + 1 >= g.P[dd]) continue;
      int n2[3] = {ijk[0], ijk[1], ijk[2]};
      n2[dd] += 1;
      int t2 = pid(n2[0], n2[1], n2[2]);
      if ((d.sigma[s] > 0) == (d.sigma[t2] > 0)) continue;
      Box b = patch_box(g, ijk[0], ijk[1], ijk[2]);
      int64_t plane = b.hi[dd];
      int u = (dd + 1) % 3, v = (dd + 2) % 3;
      Box f = b;
      f.lo[dd] = f.hi[dd] = plane;
      // local face node index: (cu, cv) over the face rectangle
      int64_t nu_ = f.hi[u] - f.lo[u] + 1, nv_ = f.hi[v] - f.lo[v] + 1;
      auto fnode = [&](int64_t I, int64_t J, int64_t K) -> int64_t {
        int64_t c[3] = {I, J, K};
        int64_t cu = c[u] - f.lo[u], cv = c[v] - f.lo[v];
        if (cu == 0 || cv == 0 || cu == nu_ - 1 || cv == nv_ - 1) return 0;  // merged boundary
        return 1 + (cu - 1) + (nu_ - 2) * (cv - 1);
      };
      int64_t nfv = 1 + std::max<int64_t>(0, (nu_ - 2)) * std::max<int64_t>(0, (nv_ - 2));
      std::vector<int64_t> eid, va, vb;
      // face-interior edges of this face, collected then sorted by id
      for (int dirn : {u, v}) {
        int64_t hi[3] = {f.hi[0], f.hi[1], f.hi[2]};
        hi[dirn] -= 1;
        for (int64_t K = f.lo[2]; K <= hi[2]; ++K)
          for (int64_t J = f.lo[1]; J <= hi[1]; ++J)
            for (int64_t I = f.lo[0]; I <= hi[0]; ++I) {
              int64_t e = g.edge_id(dirn, I, J, K);
              if (cls[e] != kFace) continue;
              eid.push_back(e);
            }
      }
      std::sort(eid.begin(), eid.end());
      for (int64_t e : eid) {
        int dd2; int64_t I, J, K;
        g.edge_decode(e, dd2, I, J, K);
        va.push_back(fnode(I, J, K));
        vb.push_back(fnode(I + (dd2 == 0), J + (dd2 == 1), K + (dd2 == 2)));
      }
      std::vector<int64_t> e2, a2, b2;
      for (size_t k = 0; k < eid.size(); ++k)
        if (va[k] != vb[k]) { e2.push_back(eid[k]); a2.push_back(va[k]); b2.push_back(vb[k]); }
      std::vector<int64_t> start, ne, nv;
      build_adjacency(nfv, e2, a2, b2, start, ne, nv);
      std::vector<uint8_t> vis(nfv, 0);
      vis[0] = 1;
      bfs(start, ne, nv, vis, {0}, gamma);
    }
  }
  std::sort(gamma.begin(), gamma.end());

  // ---- classes ----------------------------------------------------------
  std::vector<uint8_t> primal(nE, 0), dual(nE, 0), interior(nE, 0);
  for (int64_t e : gamma) primal[e] = 1;
  t = Topology();
  for (int64_t e = 0; e < nE; ++e) {
    if (cls[e] == kWirebasket && !dir[e] && !in_tree[e]) primal[e] = 1;
    if (cls[e] == kInterior && !in_tree[e]) interior[e] = 1;
  }
  for (int64_t e = 0; e < nE; ++e)
    if (cls[e] == kFace && !dir[e] && !in_tree[e] && !primal[e]) dual[e] = 1;
  std::vector<int64_t> rank(nE, -1), row(nE, -1);
  for (int64_t e = 0; e < nE; ++e) {
    if (dir[e]) t.dirichlet.push_back(e);
    if (primal[e]) { rank[e] = (int64_t)t.primal.size(); t.primal.push_back(e); }
    if (dual[e]) { row[e] = (int64_t)t.dual.size(); t.dual.push_back(e); }
    if (interior[e]) t.interior.push_back(e);
  }
  t.tree_I = tree;
  t.tree_gamma = gamma;
  t.n_vertices_H = nV;
  t.n_plain = n_plain;
  t.n_floating = (int64_t)floating.size();
  t.n_kept = nE - (int64_t)t.dirichlet.size() - (int64_t)tree.size();

  // ---- per-patch plans and the multiplier table ------------------------
  std::vector<int64_t> owner_lo(nE, -1), owner_hi(nE, -1);
  plans.assign(np, PatchPlan());
  for (int s = 0; s < np; ++s) {
    PatchPlan& pp = plans[s];
    pp.ijk[0] = s % P0; pp.ijk[1] = (s / P0) % P1; pp.ijk[2] = s / (P0 * P1);
    for (int a = 0; a < 3; ++a) {
      int r = pp.ijk[a];
      pp.m[a] = g.m[a][r];
      pp.nel[a] = d.nel[a][r];
      pp.deg[a] = d.deg[a][r];
      pp.lo[a] = d.breaks[a][r];
      pp.hi[a] = d.breaks[a][r + 1];
      pp.node0[a] = g.off[a][r];
    }
    pp.sigma = d.sigma[s];
    pp.nu = d.nu[s];
    pp.src = d.src_mask[s] != 0;
    const int mx = pp.m[0], my = pp.m[1], mz = pp.m[2];
    const int nX = (mx - 1) * my * mz, nY = mx * (my - 1) * mz, nZ = mx * my * (mz - 1);
    pp.n_loc = nX + nY + nZ;
    std::vector<std::pair<int64_t, int32_t>> ci, cb, cp;  // (gid, local)
    int32_t loc = 0;
    for (int dd = 0; dd < 3; ++dd) {
      int dims[3] = {mx, my, mz};
      dims[dd] -= 1;
      for (int c = 0; c < dims[2]; ++c)
        for (int b = 0; b < dims[1]; ++b)
          for (int a = 0; a < dims[0]; ++a, ++loc) {
            int64_t e = g.edge_id(dd, pp.node0[0] + a, pp.node0[1] + b, pp.node0[2] + c);
            if (interior[e]) ci.push_back({e, loc});
            else if (dual[e]) cb.push_back({e, loc});
            else if (primal[e]) cp.push_back({e, loc});
          }
    }
    std::sort(ci.begin(), ci.end());
    std::sort(cb.begin(), cb.end());
    std::sort(cp.begin(), cp.end());
    pp.n_i = (int)ci.size(); pp.n_b = (int)cb.size(); pp.n_p = (int)cp.size();
    pp.loc2r.assign(pp.n_loc, -1);
    for (auto* v : {&ci, &cb, &cp})
      for (auto& x : *v) {
        pp.loc2r[x.second] = (int32_t)pp.r_loc.size();
        pp.r_loc.push_back(x.second);
        pp.r_gid.push_back(x.first);
      }
    for (auto& x : cb) {
      int64_t e = x.first;
      if (owner_lo[e] < 0) owner_lo[e] = s;
      else if (owner_hi[e] < 0) owner_hi[e] = s;
      else return "dual edge shared by more than two patches";
      pp.b_row.push_back((int32_t)row[e]);
    }
    for (auto& x : cp) pp.p_rank.push_back((int32_t)rank[x.first]);
  }
  t.mult.resize(t.dual.size() * 3);
  for (size_t r = 0; r < t.dual.size(); ++r) {
    int64_t e = t.dual[r];
    if (owner_hi[e] < 0) return "dual edge with a single owner";
    t.mult[3 * r] = e;
    t.mult[3 * r + 1] = owner_lo[e];  // patches visited in increasing id
    t.mult[3 * r + 2] = owner_hi[e];
  }
  for (int s = 0; s < np; ++s) {
    PatchPlan& pp = plans[s];
    for (int k = 0; k < pp.n_b; ++k) {
      int64_t e = pp.r_gid[pp.n_i + k];
      pp.b_sgn.push_back(owner_lo[e] == s ? 1 : -1);
    }
  }
  return "";
}

// Loop rows of the reduced primal split (the outlook of Sec. 5 asks for a
// split without the interface trees in the primal set).  There the insulator
// eliminates the tree edges of every conductor/insulator face, the conductor
// keeps them as remainder unknowns, and the multiplier of each cotree edge e
// of the face ties the insulator's a_I(e) to the conductor's circulation
// a_C(e) + psi(head e) - psi(tail e).  psi is a nodal function on the face:
// zero on the face boundary, and on the face's tree edges
// a_C(t) + psi(head t) - psi(tail t) = 0, so psi at a face node is a signed
// sum of a_C along its tree path.  Returns the conductor-side terms as
// (multiplier row, edge id, +1 / -1) triples, by row, then by edge id.
std::vector<int64_t> loop_rows(const Grid& g, const Topology& t,
                               const std::vector<PatchPlan>& plans, std::vector<NodePsi>* face_psi) {
  const int64_t nE = g.n_edges();
  std::vector<uint8_t> in_tg(nE, 0);
  for (int64_t e : t.tree_gamma) in_tg[e] = 1;
  std::vector<int64_t> row(nE, -1);
  for (size_t r = 0; r < t.dual.size(); ++r) row[t.dual[r]] = (int64_t)r;
  const int P0 = g.P[0], P1 = g.P[1];
  const int np = P0 * P1 * g.P[2];
  std::vector<std::array<int64_t, 3>> out;
  for (int s = 0; s < np; ++s) {
    const int* ijk = plans[s].ijk;
    for (int dd = 0; dd < 3; ++dd) {
      if (ijk[dd] + 1 >= g.P[dd]) continue;
      int n2[3] = {ijk[0], ijk[1], ijk[2]};
      n2[dd] += 1;
      const int t2 = n2[0] + P0 * (n2[1] + P1 * n2[2]);
      if ((plans[s].sigma > 0) == (plans[t2].sigma > 0)) continue;
      Box f = patch_box(g, ijk[0], ijk[1], ijk[2]);
      f.lo[dd] = f.hi[dd];
      const int u = (dd + 1) % 3, v = (dd + 2) % 3;
      const int64_t nu_ = f.hi[u] - f.lo[u] + 1, nv_ = f.hi[v] - f.lo[v] + 1;
      // face vertex: 0 = the whole face boundary, else one interior node
      auto fnode = [&](int64_t I, int64_t J, int64_t K) -> int64_t {
        const int64_t c[3] = {I, J, K};
        const int64_t cu = c[u] - f.lo[u], cv = c[v] - f.lo[v];
        if (cu == 0 || cv == 0 || cu == nu_ - 1 || cv == nv_ - 1) return 0;
        return 1 + (cu - 1) + (nu_ - 2) * (cv - 1);
      };
      const int64_t nfv =
          1 + std::max<int64_t>(0, nu_ - 2) * std::max<int64_t>(0, nv_ - 2);
      std::vector<int64_t> tree, cotree;
      for (int dirn : {u, v}) {
        int64_t hi[3] = {f.hi[0], f.hi[1], f.hi[2]};
        hi[dirn] -= 1;
        for (int64_t K = f.lo[2]; K <= hi[2]; ++K)
          for (int64_t J = f.lo[1]; J <= hi[1]; ++J)
            for (int64_t I = f.lo[0]; I <= hi[0]; ++I) {
              const int64_t e = g.edge_id(dirn, I, J, K);
              if (in_tg[e]) tree.push_back(e);
              else if (row[e] >= 0) cotree.push_back(e);
            }
      }
      std::sort(tree.begin(), tree.end());
      std::sort(cotree.begin(), cotree.end());
      auto ends = [&](int64_t e, int64_t& a, int64_t& b) {
        int d2; int64_t I, J, K;
        g.edge_decode(e, d2, I, J, K);
        a = fnode(I, J, K);
        b = fnode(I + (d2 == 0), J + (d2 == 1), K + (d2 == 2));
      };
      std::vector<int64_t> va(tree.size()), vb(tree.size()), start, ne, nv;
      for (size_t k = 0; k < tree.size(); ++k) ends(tree[k], va[k], vb[k]);
      build_adjacency(nfv, tree, va, vb, start, ne, nv);
      // psi per face vertex as signed tree edges, grown from the boundary
      std::vector<std::vector<std::pair<int64_t, int>>> psi(nfv);
      std::vector<uint8_t> vis(nfv, 0);
      vis[0] = 1;
      std::vector<int64_t> queue{0};
      for (size_t qh = 0; qh < queue.size(); ++qh) {
        const int64_t x = queue[qh];
        for (int64_t k = start[x]; k < start[x + 1]; ++k) {
          const int64_t y = nv[k], e = ne[k];
          if (vis[y]) continue;
          vis[y] = 1;
          int64_t a, b;
          ends(e, a, b);
          psi[y] = psi[x];
          psi[y].push_back({e, a == x ? -1 : 1});  // psi(head) = psi(tail) - a(e)
          queue.push_back(y);
          if (face_psi) {
            int64_t tl, hd;
            g.edge_nodes(e, tl, hd);
            face_psi->push_back({a == x ? hd : tl, psi[y]});
          }
        }
      }
      for (int64_t e : cotree) {
        int64_t a, b;
        ends(e, a, b);
        std::map<int64_t, int> terms;
        terms[e] += 1;
        for (const auto& tc : psi[b]) terms[tc.first] += tc.second;
        for (const auto& tc : psi[a]) terms[tc.first] -= tc.second;
        for (const auto& tc : terms)
          if (tc.second != 0) out.push_back({row[e], tc.first, (int64_t)tc.second});
      }
    }
  }
  std::sort(out.begin(), out.end());
  std::vector<int64_t> flat;
  flat.reserve(out.size() * 3);
  for (const auto& o : out) flat.insert(flat.end(), o.begin(), o.end());
  return flat;
}

// psi of the loop split as a function of a_C on the face-tree edges, at every
// node where it can be nonzero.  On the interior nodes of each conductor /
// insulator face it is the signed tree-path sum that loop_rows builds.  Into
// the insulator it is continued as a constant along the gauge tree T_I (so
// G psi vanishes on T_I and the gauge is kept), away from grounded nodes:
// those on the domain boundary or in the closed box of a conductor patch.
// A subtree of T_I hangs from one face node, since T_I is a tree of the graph
// in which every conductor closure is one vertex.  The load correction of a
// face-tree edge t is then -sum_n (G^T f_I)(n) c(n, t) over these terms.
// Returns (node id, edge id, +1 / -1) triples, by node, then by edge id.
std::vector<int64_t> loop_psi(const Grid& g, const Topology& t,
                              const std::vector<PatchPlan>& plans, std::string& err) {
  std::vector<NodePsi> fp;
  loop_rows(g, t, plans, &fp);
  const int64_t nN = g.n_nodes();
  std::vector<uint8_t> grounded(nN, 0);
  for (int64_t K = 0; K < g.N[2]; ++K)
    for (int64_t J = 0; J < g.N[1]; ++J)
      for (int64_t I = 0; I < g.N[0]; ++I)
        if (g.node_boundary(I, J, K)) grounded[g.node_id(I, J, K)] = 1;
  for (const PatchPlan& pp : plans) {
    if (!(pp.sigma > 0)) continue;
    const Box b = patch_box(g, pp.ijk[0], pp.ijk[1], pp.ijk[2]);
    for (int64_t K = b.lo[2]; K <= b.hi[2]; ++K)
      for (int64_t J = b.lo[1]; J <= b.hi[1]; ++J)
        for (int64_t I = b.lo[0]; I <= b.hi[0]; ++I) grounded[g.node_id(I, J, K)] = 1;
  }
  // T_I as node adjacency (CSR)
  std::vector<int64_t> start(nN + 1, 0), nbr(2 * t.tree_I.size());
  for (int64_t e : t.tree_I) {
    int64_t a, b;
    g.edge_nodes(e, a, b);
    ++start[a + 1];
    ++start[b + 1];
  }
  for (int64_t n = 0; n < nN; ++n) start[n + 1] += start[n];
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t e : t.tree_I) {
      int64_t a, b;
      g.edge_nodes(e, a, b);
      nbr[fill[a]++] = b;
      nbr[fill[b]++] = a;
    }
  }
  // src[n]: index into fp of the face node whose psi n carries, or -1
  std::vector<int64_t> src(nN, -1), queue;
  for (size_t k = 0; k < fp.size(); ++k) {
    src[fp[k].first] = (int64_t)k;
    queue.push_back(fp[k].first);
  }
  for (size_t qh = 0; qh < queue.size(); ++qh) {
    const int64_t x = queue[qh];
    for (int64_t k = start[x]; k < start[x + 1]; ++k) {
      const int64_t y = nbr[k];
      if (grounded[y]) continue;
      if (src[y] >= 0) {
        if (src[y] != src[x]) {
          err = "loop split: a gauge subtree is reached from two interface nodes";
          return {};
        }
        continue;
      }
      src[y] = src[x];
      queue.push_back(y);
    }
  }
  std::vector<int64_t> flat;
  for (int64_t n = 0; n < nN; ++n) {
    if (src[n] < 0) continue;
    std::map<int64_t, int> terms;
    for (const auto& tc : fp[src[n]].second) terms[tc.first] += tc.second;
    for (const auto& tc : terms)
      if (tc.second != 0) flat.insert(flat.end(), {n, tc.first, (int64_t)tc.second});
  }
  return flat;
}

// Per-patch plan of the loop split, in the layout the device setup would take.
// The interface trees leave the primal set: a conductor keeps its face-tree
// edges as remainder, appended to its b block (by edge id); an insulator
// eliminates them.  The i block is unchanged.  Coarse ranks are renumbered
// over the primal edges left.  Each own b edge carries its multiplier row:
// on a loop row the insulator's entry is -1 and the conductor's entries are
// the row's loop terms (own edge and face-tree path); on any other row the
// entry is today's +1 on the lower patch id, -1 on the other.
// Returns 5-wide records, per patch in order:
//   (s, 0, b index, edge id, 0)       b block, in order
//   (s, 1, p index, edge id, rank)    p block, in order, coarse rank
//   (s, 2, row, b index, +1 / -1)     entries of B_s, by row, then b index
std::vector<int64_t> loop_plan(const Grid& g, const Topology& t,
                               const std::vector<PatchPlan>& plans) {
  const int64_t nE = g.n_edges();
  std::vector<uint8_t> in_tg(nE, 0);
  for (int64_t e : t.tree_gamma) in_tg[e] = 1;
  std::vector<int64_t> rank(nE, -1);
  int64_t nP = 0;
  for (int64_t e : t.primal)
    if (!in_tg[e]) rank[e] = nP++;
  const std::vector<int64_t> lr = loop_rows(g, t, plans);
  std::map<int64_t, std::vector<std::pair<int64_t, int>>> terms;
  for (size_t k = 0; k + 2 < lr.size(); k += 3) terms[lr[k]].push_back({lr[k + 1], (int)lr[k + 2]});
  std::vector<int64_t> out;
  for (size_t s = 0; s < plans.size(); ++s) {
    const PatchPlan& pp = plans[s];
    const bool cond = pp.sigma > 0;
    std::vector<int64_t> b_gid(pp.r_gid.begin() + pp.n_i, pp.r_gid.begin() + pp.n_i + pp.n_b);
    std::vector<int64_t> p_gid;
    for (int j = 0; j < pp.n_p; ++j) {
      const int64_t e = pp.r_gid[pp.n_i + pp.n_b + j];
      if (!in_tg[e]) p_gid.push_back(e);
      else if (cond) b_gid.push_back(e);
    }
    std::map<int64_t, int64_t> bpos;
    for (size_t k = 0; k < b_gid.size(); ++k) {
      bpos[b_gid[k]] = (int64_t)k;
      out.insert(out.end(), {(int64_t)s, 0, (int64_t)k, b_gid[k], 0});
    }
    for (size_t k = 0; k < p_gid.size(); ++k)
      out.insert(out.end(), {(int64_t)s, 1, (int64_t)k, p_gid[k], rank[p_gid[k]]});
    std::vector<std::array<int64_t, 3>> ent;
    for (int k = 0; k < pp.n_b; ++k) {
      const int64_t r = pp.b_row[k];
      auto it = terms.find(r);
      if (it == terms.end()) {
        ent.push_back({r, k, pp.b_sgn[k]});
      } else if (!cond) {
        ent.push_back({r, k, -1});
      } else {
        for (const auto& tc : it->second) ent.push_back({r, bpos.at(tc.first), tc.second});
      }
    }
    std::sort(ent.begin(), ent.end());
    for (const auto& x : ent) out.insert(out.end(), {(int64_t)s, 2, x[0], x[1], x[2]});
  }
  return out;
}

}  // namespace tcf
