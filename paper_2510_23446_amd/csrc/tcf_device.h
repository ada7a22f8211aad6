// Device-side data structures shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define TCF_MAXP 8
#define TCF_NB 32  // factorisation panel width; all block sizes are padded to it
#define TCF_QSLOTS 1024  // slots of a tile-accumulated quadratic form (atomic spread)

#include "tcf_jobs.h"

namespace tcf {

// One patch as seen by the kernels.
struct DevPatch {
  int m[3], nel[3], deg[3];
  double lo[3], hi[3];
  double sigma, nu;
  int n_i, n_b, n_p, n_r, n_loc;
  int ni_pad, nb_pad, np_pad, nr_pad;  // padded to TCF_NB
  int src, cond;
  int64_t A_off;   // dense [i|b|p] matrix, nr_pad x nr_pad column-major
  int64_t G_off;   // [Sbb^-1 | Phi_b], ld = nb_pad, n_b + n_p columns
  int64_t S_off;   // Sbb, ld = nb_pad, n_b columns
  int64_t Q_off;   // Q^T = [L_ii^-T | E_bi^T | E_pi^T], ld = ni_pad, n_r columns
  int r_off, i_off, b_off, p_off, bp_off, loc_off;
  int tab_off[3];  // 1-D Galerkin tables per direction
  int ptab_off[3]; // basis values at load quadrature points per direction
  int nq_load[3];  // load quadrature points per direction (nel * (deg + 3))
};

// A block of columns [c_begin, c_end) of one dense SPD matrix to factor.
// One patch of a batched source load: field values at F + f_off, result
// scaled by scale (1, or sigma for the initial-value load)
struct LoadJob {
  int64_t f_off;
  int s, pad;
  double scale;
};

struct FactorJob {
  int64_t off;  // matrix offset (elements)
  int ld;       // leading dimension == padded order
  int n;        // padded order (multiple of TCF_NB)
  int c_begin, c_end;
  int tag;      // patch id reported on a non-positive pivot (-1 coarse)
};

// Triangular solve with the lower block L (order n, multiple of TCF_NB) at
// (l_row0, l_row0) of a matrix with leading dimension ldl, against ncols
// right-hand sides stored with leading dimension ldb.  The first tri
// right-hand sides are the identity columns (the solution is then
// triangular there and its zero rows are skipped).
struct TrsmJob {
  int64_t l_off;
  int ldl, l_row0, n;
  int64_t b_off;
  int ldb, ncols;
  int tri;
  int pad;
};

// Column-dot matrix-vector job: out[j] = sum_{r < nrows} M[r + j*ld] x[r].
struct DotJob {
  int64_t m_off;
  int ld, nrows, ncols;
  int x_off;    // offset into gather tables / input vector
  int out_off;
};

// Row-stripe matrix-vector job: out[r] = base[r] + alpha * sum_j M[r + (c0+j)*ld] y[j].
struct AxpyJob {
  int64_t m_off;
  int ld, nrows, ncols, c0;
  int y_off;    // offset into the gather index table of y
  int out_off;
};

// One tile of an operator stored tile by tile: nc columns of 64 rows each
// (column-major, zero beyond row nr).  N part: y[yr_off + r] += sum_c A[r,c]
// x[xc_off + c]; T part: y[yc_off + c] += sum_r A[r,c] x[xr_off + r].
// flags bit 0 = N, bit 1 = T, bit 2 = T output at y[ymap[yc_off + c]],
// bit 3 = N output at y[ymap[yr_off + r]].
struct TileJob {
  int64_t m_off;
  int xr_off, xc_off;
  int yr_off, yc_off;
  int nr, nc;
  int flags;
  int pad;
};

// One node of the coarse factor's elimination tree as the kernels see it.
// Its front is dense, column-major, order nf = nj_pad + ns_pad: the node's
// own nj unknowns (padded to TCF_NB with an identity diagonal), then its
// structure S (ns ND indices, ascending, at slist + s_off).
struct CoarseNodeDev {
  int64_t f_off;     // front offset in the front buffer
  int64_t l_off;     // [L_JJ^-1 | -L_JJ^-T L_SJ^T] offset in the operator buffer
  int j0, nj, nj_pad, ns, nf, s_off;
  int parent, pad;
};

struct PcgScalars {
  double dd;         // ||d||^2
  double rz[2];      // r.z of the current / next iteration (parity)
  double rr;         // last ||r||^2
  int done;
  int iters;
  int pad[2];
};

}  // namespace tcf
