// Host plan of the coarse (primal) factorisation: a nested dissection of the
// coarse unknowns over the patch grid, and the block structure of its
// Cholesky factor.
//
// The coarse matrix S_Pi = sum_s N_s^T S_pp^(s) N_s (Sec. 3: the second Schur
// complement of the three-field system) couples two primal unknowns exactly
// when some patch holds both.  Group the primal unknowns into entities by
// the set of patches that hold them (the unknowns of one interface face, of
// one patch edge line, ...).  Cut the patch grid by a plane between two
// patch rows: an entity whose patches all lie on one side couples only to
// entities that touch that side, so the entities that straddle the plane
// separate the two halves of the coarse graph.  Recursing on both halves
// gives a nested dissection whose elimination tree has one node per
// separator (and one per leaf region); eliminating in postorder confines
// fill-in to the ancestors of each node.
//
// Per node J the factor has a dense diagonal block over J's own unknowns
// and a dense block over its structure S_J: the ancestor unknowns coupled to
// J, directly or through eliminated descendants.  The last node (the top
// separator) has no structure; its whole Schur complement is inverted
// densely.  A plan with a single node is the plain dense inverse of S_Pi.
#include <algorithm>
#include <map>
#include <numeric>
#include <set>

#include "tcf_internal.h"

namespace tcf {

namespace {

struct NdBuild {
  const int* P;
  std::vector<std::array<int, 6>> box;  // per entity: min/max patch coords
  std::vector<int> units;               // per entity: unknown count
  std::vector<std::vector<int>> ent_nodes;  // per node: its entities
  std::vector<std::vector<int>> children;
  int leaf_max = 0;

  int total(const std::vector<int>& ents) const {
    int t = 0;
    for (int e : ents) t += units[e];
    return t;
  }
  // Orders the region [lo, hi) (patch coordinates) and returns the roots of
  // the sub-forest it produced, in postorder.
  std::vector<int> split(const int lo[3], const int hi[3], std::vector<int> ents, bool top,
                         int dense_max) {
    std::vector<int> roots;
    if (ents.empty()) return roots;
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    const int ext = hi[ax] - lo[ax];
    const int tot = total(ents);
    const bool stop = ext <= 1 || (top ? tot <= dense_max : tot <= leaf_max);
    if (stop) {
      ent_nodes.push_back(ents);
      children.emplace_back();
      roots.push_back((int)ent_nodes.size() - 1);
      return roots;
    }
    const int mid = lo[ax] + ext / 2;
    std::vector<int> L, R, S;
    for (int e : ents) {
      if (box[e][3 + ax] < mid) L.push_back(e);
      else if (box[e][ax] >= mid) R.push_back(e);
      else S.push_back(e);
    }
    int hl[3] = {hi[0], hi[1], hi[2]}, lr[3] = {lo[0], lo[1], lo[2]};
    hl[ax] = mid;
    lr[ax] = mid;
    std::vector<int> cl = split(lo, hl, std::move(L), false, dense_max);
    std::vector<int> cr = split(lr, hi, std::move(R), false, dense_max);
    cl.insert(cl.end(), cr.begin(), cr.end());
    if (S.empty()) return cl;  // the halves do not couple: a forest
    ent_nodes.push_back(S);
    children.push_back(cl);
    roots.push_back((int)ent_nodes.size() - 1);
    return roots;
  }
};

}  // namespace

CoarsePlan plan_coarse(const std::vector<PatchPlan>& plans, const int P[3], int n_primal,
                       int dense_max, int leaf_max) {
  CoarsePlan cp;
  cp.nd.assign(n_primal, -1);
  if (n_primal == 0) return cp;
  // patches holding each coarse unknown (patch ids ascending)
  std::vector<std::vector<int>> owners(n_primal);
  for (size_t s = 0; s < plans.size(); ++s)
    for (int g : plans[s].p_rank) owners[g].push_back((int)s);
  std::map<std::vector<int>, int> ent_of;
  std::vector<int> ent(n_primal);
  std::vector<std::vector<int>> ent_units, ent_patches;
  for (int g = 0; g < n_primal; ++g) {
    auto it = ent_of.find(owners[g]);
    if (it == ent_of.end()) {
      it = ent_of.emplace(owners[g], (int)ent_units.size()).first;
      ent_units.emplace_back();
      ent_patches.push_back(owners[g]);
    }
    ent[g] = it->second;
    ent_units[it->second].push_back(g);
  }
  const int ne = (int)ent_units.size();
  NdBuild b;
  b.P = P;
  b.leaf_max = leaf_max;
  b.box.resize(ne);
  b.units.resize(ne);
  for (int e = 0; e < ne; ++e) {
    std::array<int, 6> bx = {1 << 30, 1 << 30, 1 << 30, -1, -1, -1};
    for (int s : ent_patches[e]) {
      const int c[3] = {s % P[0], (s / P[0]) % P[1], s / (P[0] * P[1])};
      for (int a = 0; a < 3; ++a) {
        bx[a] = std::min(bx[a], c[a]);
        bx[3 + a] = std::max(bx[3 + a], c[a]);
      }
    }
    b.box[e] = bx;
    b.units[e] = (int)ent_units[e].size();
  }
  std::vector<int> all(ne);
  std::iota(all.begin(), all.end(), 0);
  const int lo[3] = {0, 0, 0}, hi[3] = {P[0], P[1], P[2]};
  b.split(lo, hi, all, true, dense_max);
  const int nn = (int)b.ent_nodes.size();
  cp.nodes.resize(nn);
  std::vector<int> node_of_ent(ne, -1);
  // ND numbering: nodes in postorder (creation order), entities within a
  // node by their first unknown, unknowns within an entity ascending
  int next = 0;
  for (int i = 0; i < nn; ++i) {
    auto& es = b.ent_nodes[i];
    std::sort(es.begin(), es.end(),
              [&](int x, int y) { return ent_units[x][0] < ent_units[y][0]; });
    CoarseNode& nd = cp.nodes[i];
    nd.j0 = next;
    for (int e : es) {
      node_of_ent[e] = i;
      for (int g : ent_units[e]) cp.nd[g] = next++;
    }
    nd.nj = next - nd.j0;
    for (int c : b.children[i]) cp.nodes[c].parent = i;
  }
  // entities of each patch, for the direct couplings
  std::vector<std::vector<int>> ents_of_patch(plans.size());
  for (int e = 0; e < ne; ++e)
    for (int s : ent_patches[e]) ents_of_patch[s].push_back(e);
  // structure by entity: direct couplings to ancestors, then what the
  // children's structures pass up (everything but this node's own)
  std::vector<std::set<int>> sent(nn);
  for (int i = 0; i < nn; ++i) {
    CoarseNode& nd = cp.nodes[i];
    std::vector<char> anc(nn, 0);
    for (int a = nd.parent; a >= 0; a = cp.nodes[a].parent) anc[a] = 1;
    std::set<int>& S = sent[i];
    for (int e : b.ent_nodes[i])
      for (int s : ent_patches[e])
        for (int f : ents_of_patch[s])
          if (anc[node_of_ent[f]]) S.insert(f);
    for (int c : b.children[i]) {
      nd.height = std::max(nd.height, cp.nodes[c].height + 1);
      for (int f : sent[c])
        if (node_of_ent[f] != i) S.insert(f);
    }
    std::vector<int> se(S.begin(), S.end());
    std::sort(se.begin(), se.end(),
              [&](int x, int y) { return cp.nd[ent_units[x][0]] < cp.nd[ent_units[y][0]]; });
    for (int f : se) {
      const int g0 = cp.nd[ent_units[f][0]];
      for (int u = 0; u < (int)ent_units[f].size(); ++u) nd.S.push_back(g0 + u);
    }
  }
  return cp;
}

}  // namespace tcf
