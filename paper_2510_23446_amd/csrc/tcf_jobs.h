// Job descriptors of the row-panel and tile-packing kernels (plain structs,
// shared by the device code and the host planning).
#pragma once

#include <cstdint>

namespace tcf {

// A row panel of an operator for the matrix-core path: nr <= 64 output rows
// and a run of nt tiles (tiles[t0 ..]) along the columns, each tile nc <= 64
// stored columns of 64 rows (zero past nr), stored back to back from m_off.
// y[yr_off + r] (or y[ymap[yr_off + r]]) += sum over the panel's tiles of
// A x; the quadratic form x_r^T (A x) uses the inputs at xr_off.
// flags: bit 0 outputs shared with other panels (atomic adds), bit 1 output
// rows through ymap, bit 2 quadratic form.
struct PanelJob {
  int64_t m_off;
  int t0, nt;
  int yr_off, nr;
  int xr_off, flags;
};
struct PanelTile {
  int xc_off, nc;
};

// Copy the nr x nc block at (row0, col0) of a column-major source into a tile
// of 64-row columns (rows beyond the block are zero).  trans = 0: nc stored
// columns, tile(r, c) = block(r, c); trans = 1: nr stored columns,
// tile(c, r) = block(r, c).
struct PackJob {
  int64_t src_off;
  int64_t dst_off;
  int ld, row0, col0, nr, nc;
  int trans;
};

}  // namespace tcf
