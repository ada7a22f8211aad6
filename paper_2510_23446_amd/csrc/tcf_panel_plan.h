// Host-side planning of the row-panel jobs (no device code): tile sizes,
// split lengths and the order jobs are dispatched in.  Plain functions, so
// that host tests can build them with a host compiler.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "tcf_jobs.h"

namespace tcf {

// Elements one stored panel tile of nc columns takes: columns padded to the
// quantum of the matrix-core operand order, 4 x (16 bytes / element size).
static int64_t panel_tile_elems(int nc, int elem_bytes) {
  const int q = 4 * (16 / elem_bytes);
  return 64 * (int64_t)((nc + q - 1) / q * q);
}

// A panel longer than the split length becomes several jobs of about equal
// length (more workgroups in flight); their partial rows add atomically.
static std::vector<PanelJob> split_jobs(const std::vector<PanelJob>& whole, int chunk,
                                        const std::vector<PanelTile>& tl, int eb) {
  std::vector<PanelJob> v;
  for (const PanelJob& j : whole) {
    const int parts = (j.nt + chunk - 1) / chunk;
    int64_t off = j.m_off;
    for (int q = 0, t = j.t0; q < parts; ++q) {
      const int n = j.nt / parts + (q < j.nt % parts ? 1 : 0);
      PanelJob c = j;
      c.m_off = off;
      c.t0 = t;
      c.nt = n;
      if (parts > 1) c.flags |= 1;
      for (int k = 0; k < n; ++k) off += panel_tile_elems(tl[t + k].nc, eb);
      t += n;
      v.push_back(c);
    }
  }
  return v;
}

// Dispatch order of one coarse-sweep launch's jobs (block b takes entry b;
// the hardware deals consecutive blocks to the 8 XCDs in turn): runs of
// kXcdRun consecutive jobs (panels of one node, which take the same inputs)
// go to one XCD, whose L2 then serves their inputs, and the runs are dealt
// to the XCDs in turn, so that the blocks in flight still stream one window
// of the buffer.  Measured against the plain order on one GPU: the coarse
// solve 4% faster, the per-patch operators (F apply, coarse correction)
// 7-10% slower, so those keep the plain order.
constexpr int kXcdRun = 16;
static std::vector<PanelJob> xcd_order(const std::vector<PanelJob>& v) {
  const int n = (int)v.size();
  std::vector<std::vector<int>> q(8);
  for (int r = 0; r * kXcdRun < n; ++r)
    for (int k = r * kXcdRun; k < std::min(n, (r + 1) * kXcdRun); ++k) q[r % 8].push_back(k);
  std::vector<PanelJob> out;
  out.reserve(n);
  for (size_t k = 0; (int)out.size() < n; ++k)
    for (int x = 0; x < 8; ++x)
      if (k < q[x].size()) out.push_back(v[q[x][k]]);
  return out;
}

}  // namespace tcf
