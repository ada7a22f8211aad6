/*
 * Host-only driver of the topology code (gauge tree, primal/dual split,
 * multiplier table) and of the loop-split host plan (loop rows, psi, per-patch
 * plan), built with AddressSanitizer and UBSan by the test that runs it.  Four
 * layouts: conductors below, an uneven checkerboard, a floating conductor and a
 * flat 4x4x2 checkerboard; each prints its sizes.
 */
#include <cstdio>
#include <vector>
#include "../paper_2510_23446_amd/csrc/tcf_internal.h"
using namespace tcf;

static int run(const char* name, int P0, int P1, int P2, std::vector<double> sigma,
               std::vector<int32_t> nel, std::vector<int32_t> deg) {
  std::vector<double> br[3];
  int P[3] = {P0, P1, P2};
  tcf_problem_desc d = {};
  static std::vector<int32_t> nels[3], degs[3];
  for (int a = 0; a < 3; ++a) {
    for (int i = 0; i <= P[a]; ++i) br[a].push_back(double(i) / P[a]);
    nels[a].assign(P[a], 0); degs[a].assign(P[a], 0);
    for (int i = 0; i < P[a]; ++i) { nels[a][i] = nel[(i + a) % nel.size()]; degs[a][i] = deg[(i + a) % deg.size()]; }
    d.np[a] = P[a]; d.breaks[a] = br[a].data(); d.nel[a] = nels[a].data(); d.deg[a] = degs[a].data();
  }
  std::vector<double> nu(sigma.size(), 1.0);
  std::vector<uint8_t> src(sigma.size(), 0);
  std::vector<double> amp(4, 1.0);
  d.sigma = sigma.data(); d.nu = nu.data(); d.src_mask = src.data(); d.n_rhs = 1;
  d.amp = amp.data(); d.dt = 1e-3; d.n_steps = 4;
  std::string e = validate_desc(d);
  if (!e.empty()) { printf("%s: validate %s\n", name, e.c_str()); return 1; }
  Grid g = build_grid(d);
  Topology t; std::vector<PatchPlan> plans;
  e = compute_topology(d, g, t, plans);
  if (!e.empty()) { printf("%s: topology %s\n", name, e.c_str()); return 1; }
  auto lr = loop_rows(g, t, plans);
  std::string err;
  auto lp = loop_psi(g, t, plans, err);
  auto pl = loop_plan(g, t, plans);
  printf("%s: edges %lld plan records %zu loop terms %zu psi terms %zu err '%s'\n", name,
         (long long)g.n_edges(), pl.size() / 5, lr.size() / 3, lp.size() / 3, err.c_str());
  return err.empty() ? 0 : 1;
}

int main() {
  int rc = 0;
  rc |= run("cond_bottom", 2, 2, 2, {1, 1, 1, 1, 0, 0, 0, 0}, {4}, {2});
  std::vector<double> cb(27), fl(27, 0.0);
  for (int s = 0; s < 27; ++s) cb[s] = ((s % 3 + (s / 3) % 3 + s / 9) % 2) ? 1.0 : 0.0;
  fl[13] = 1.0;  // floating conductor in the middle
  rc |= run("checker_uneven", 3, 3, 3, cb, {3, 2, 4}, {2, 3, 1});
  rc |= run("floating", 3, 3, 3, fl, {3, 2}, {2, 3});
  std::vector<double> cb2(4 * 4 * 2);
  for (int s = 0; s < 32; ++s) cb2[s] = ((s % 4 + (s / 4) % 4 + s / 16) % 2) ? 1.0 : 0.0;
  rc |= run("checker_4x4x2", 4, 4, 2, cb2, {2, 3}, {2});
  return rc;
}
