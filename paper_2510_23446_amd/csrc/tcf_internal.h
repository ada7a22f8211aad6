// Internal host-side structures of libtcf (not part of the C-ABI).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tcf.h"

namespace tcf {

enum EdgeClass : uint8_t { kWirebasket = 0, kFace = 1, kInterior = 2 };

// Global control grid of a multi-patch box: rows of m = nel + deg nodes,
// neighbouring rows share their boundary node plane.
struct Grid {
  int P[3] = {0, 0, 0};
  std::vector<int> m[3];        // nodes per row
  std::vector<int64_t> off[3];  // first global node of each row
  int64_t N[3] = {0, 0, 0};     // global nodes per direction
  std::vector<uint8_t> on_plane[3];  // per global node index: on a break plane
  int64_t Ex = 0, Ey = 0, Ez = 0;

  int64_t n_edges() const { return Ex + Ey + Ez; }
  int64_t n_nodes() const { return N[0] * N[1] * N[2]; }
  int64_t node_id(int64_t I, int64_t J, int64_t K) const { return I + N[0] * (J + N[1] * K); }
  int64_t edge_id(int d, int64_t I, int64_t J, int64_t K) const {
    if (d == 0) return I + (N[0] - 1) * (J + N[1] * K);
    if (d == 1) return Ex + I + N[0] * (J + (N[1] - 1) * K);
    return Ex + Ey + I + N[0] * (J + N[1] * K);
  }
  void edge_decode(int64_t e, int& d, int64_t& I, int64_t& J, int64_t& K) const {
    int64_t nx, ny;
    if (e < Ex) { d = 0; nx = N[0] - 1; ny = N[1]; }
    else if (e < Ex + Ey) { d = 1; e -= Ex; nx = N[0]; ny = N[1] - 1; }
    else { d = 2; e -= Ex + Ey; nx = N[0]; ny = N[1]; }
    I = e % nx;
    J = (e / nx) % ny;
    K = e / (nx * ny);
  }
  void edge_nodes(int64_t e, int64_t& tail, int64_t& head) const {
    int d; int64_t I, J, K;
    edge_decode(e, d, I, J, K);
    tail = node_id(I, J, K);
    head = node_id(I + (d == 0), J + (d == 1), K + (d == 2));
  }
  bool node_boundary(int64_t I, int64_t J, int64_t K) const {
    return I == 0 || J == 0 || K == 0 || I == N[0] - 1 || J == N[1] - 1 || K == N[2] - 1;
  }
};

// One patch: its box in the grid, its spline rows, and the [i | b | p]
// ordering of its kept ("remainder" + primal) unknowns.
struct PatchPlan {
  int ijk[3];
  int m[3], nel[3], deg[3];
  double lo[3], hi[3];
  double sigma, nu;
  bool src;
  int64_t node0[3];
  int n_loc = 0;                 // all local edges
  int n_i = 0, n_b = 0, n_p = 0; // kept classes
  int n_r() const { return n_i + n_b + n_p; }
  std::vector<int32_t> r_loc;    // [n_r] local edge index, order [i|b|p], each by edge id
  std::vector<int64_t> r_gid;    // [n_r] global edge id
  std::vector<int32_t> loc2r;    // [n_loc] kept index or -1 (eliminated)
  std::vector<int32_t> b_row;    // [n_b] multiplier row
  std::vector<int8_t> b_sgn;     // [n_b] +1 / -1
  std::vector<int32_t> p_rank;   // [n_p] coarse index
};

struct Topology {
  std::vector<int64_t> dirichlet, tree_I, tree_gamma, primal, dual, interior;
  std::vector<int64_t> mult;     // [n_lambda*3]: edge, s+, s-
  int64_t n_vertices_H = 0, n_plain = 0, n_floating = 0, n_kept = 0;
};

Grid build_grid(const tcf_problem_desc& d);
// Returns empty string on success, else an error message.
std::string validate_desc(const tcf_problem_desc& d);
std::string compute_topology(const tcf_problem_desc& d, const Grid& g, Topology& t,
                             std::vector<PatchPlan>& plans);
// psi of one face node of the loop split: node id, signed face-tree edges
using NodePsi = std::pair<int64_t, std::vector<std::pair<int64_t, int>>>;
// Conductor-side terms (row, edge, +-1) of the loop rows of the reduced
// primal split; see the definition.  With face_psi, also appends psi of
// every face-interior node that the face trees reach.
std::vector<int64_t> loop_rows(const Grid& g, const Topology& t,
                               const std::vector<PatchPlan>& plans,
                               std::vector<NodePsi>* face_psi = nullptr);
// psi coefficients (node, edge, +-1) of the loop split on the face nodes and
// along the gauge tree into the insulator; err is set if T_I is inconsistent.
std::vector<int64_t> loop_psi(const Grid& g, const Topology& t,
                              const std::vector<PatchPlan>& plans, std::string& err);

// Per-patch plan of the loop split as 5-wide records (patch, kind, ...):
// kind 0 b block, kind 1 p block with coarse ranks, kind 2 entries of B_s.
std::vector<int64_t> loop_plan(const Grid& g, const Topology& t,
                               const std::vector<PatchPlan>& plans);

// Nested-dissection plan of the coarse Cholesky factor (tcf_coarse.cpp).
struct CoarseNode {
  int j0 = 0, nj = 0;       // its own unknowns: ND indices [j0, j0 + nj)
  int parent = -1;          // -1: a root of the elimination forest
  int height = 0;           // 0 for a leaf, else 1 + the highest child
  std::vector<int> S;       // structure: ascending ND indices of the ancestor
                            // unknowns its factor columns reach
};
struct CoarsePlan {
  std::vector<int> nd;             // coarse unknown (primal rank) -> ND index
  std::vector<CoarseNode> nodes;   // postorder (children before parents)
};
// Regions of more than dense_max (top) / leaf_max (below) unknowns are cut
// at the middle patch plane of their longest extent, down to single patch
// rows.  dense_max >= n_primal gives one node: the dense inverse.
CoarsePlan plan_coarse(const std::vector<PatchPlan>& plans, const int P[3], int n_primal,
                       int dense_max, int leaf_max);

}  // namespace tcf
