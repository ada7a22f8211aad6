// HIP kernels of libtcf for gfx950 (CDNA4, 64-wide wavefronts).
//
// Setup: 1-D Galerkin tables by Gauss quadrature, dense patch matrices in
// [interior | dual | primal] order, batched partial Cholesky (right-looking,
// 32-wide panels), multi-RHS triangular solves that produce the explicit
// Schur operators.  Per step: matrix-free conductor mass, condensation,
// column-dot and row-stripe matrix-vector products for the dual-primal
// operator, the signed jump, and PCG recurrences with device-side scalars.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cfloat>
#include <algorithm>
#include <climits>
#include <type_traits>

#include "tcf_device.h"
#include "tcf_kernels.h"

// 4-wide FP64 accumulator of v_mfma_f64_16x16x4
typedef double tcf_v4d __attribute__((ext_vector_type(4)));
typedef float tcf_v4f __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 matrix-core product per element type, FP32 accumulating
// in FP32 and FP64 in FP64.  Both take A[l % 16][l / 16] and
// B[l / 16][l % 16] from lane l; they differ in where the 16 x 16 result
// lands (checked by probes on the device): element e of lane l is
// C[row(l / 16, e)][l % 16] with row = l/16 + 4 e for FP64 and
// 4 (l/16) + e for FP32.
template <class T>
struct Mfma16;
template <>
struct Mfma16<double> {
  typedef tcf_v4d acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int e) { return lk + 4 * e; }
};
template <>
struct Mfma16<float> {
  typedef tcf_v4f acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int e) { return 4 * lk + e; }
};

namespace tcf {

// 16-byte vector of stored matrix entries (2 doubles or 4 floats)
template <class T>
struct TileVec;
template <>
struct TileVec<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <>
struct TileVec<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};

// ===========================================================================
// 1-D splines on one patch row (open uniform knots)
// ===========================================================================
struct Row1D {
  double lo, hi;
  int nel, p;
};

__device__ inline double knot(const Row1D& r, int i) {
  if (i <= r.p) return r.lo;
  int t = i - r.p;
  if (t >= r.nel) return r.hi;
  return (r.hi - r.lo) / r.nel * t + r.lo;
}

// Degree-q B-splines active on element t (span k = p + t of the degree-p
// knot vector): out[j] = N_{k-q+j, q}(x), j = 0..q.  Cox-de Boor recursion,
// updated in place from the highest index down.
__device__ inline void bspline_span(const Row1D& r, int t, double x, int q, double* out) {
  const int k = r.p + t;
  out[0] = 1.0;
  for (int d = 1; d <= q; ++d) {
    for (int j = d; j >= 0; --j) {
      const int i = k - d + j;
      const double lo_v = (j >= 1) ? out[j - 1] : 0.0;
      const double hi_v = (j <= d - 1) ? out[j] : 0.0;
      double v = 0.0;
      const double ui = knot(r, i), uid = knot(r, i + d);
      if (uid - ui > 0.0) v += (x - ui) / (uid - ui) * lo_v;
      const double ui1 = knot(r, i + 1), uid1 = knot(r, i + d + 1);
      if (uid1 - ui1 > 0.0) v += (uid1 - x) / (uid1 - ui1) * hi_v;
      out[j] = v;
    }
  }
}

// On element t at x: N[j] = N_{t+j}, dN[j] = N'_{t+j} (j = 0..p) and the
// edge functions D[j] = D_{t+j} = p/(U_{t+j+p+1} - U_{t+j+1}) N^{p-1}_{t+j+1}
// (j = 0..p-1).  The derivative uses N'_i = D_{i-1} - D_i.
__device__ inline void eval_element(const Row1D& r, int t, double x, double* N, double* D,
                                    double* dN) {
  const int p = r.p;
  double Nl[TCF_MAXP + 1];
  bspline_span(r, t, x, p - 1, Nl);
  for (int j = 0; j < p; ++j) {
    const int e = t + j;
    D[j] = p / (knot(r, e + p + 1) - knot(r, e + 1)) * Nl[j];
  }
  bspline_span(r, t, x, p, N);
  for (int j = 0; j <= p; ++j) dN[j] = (j >= 1 ? D[j - 1] : 0.0) - (j <= p - 1 ? D[j] : 0.0);
}

__device__ inline int gauss_off(int nq) { return nq * (nq - 1) / 2; }

// Tables per (patch, direction): Nn = int N_i N_j, NdNd = int N'_i N'_j,
// Dd = int D_i D_j, DNd = int D_i N'_j, by Gauss-Legendre with p+1 points per
// element (exact).  One block per (patch, direction).
__global__ void k_tables1d(const DevPatch* P, const double* gx, const double* gw, double* tabs) {
  const int s = blockIdx.x / 3, d = blockIdx.x % 3;
  const DevPatch& pp = P[s];
  const Row1D r{pp.lo[d], pp.hi[d], pp.nel[d], pp.deg[d]};
  const int m = pp.m[d], p = r.p, nq = p + 1;
  const double* g = gx + gauss_off(nq);
  const double* w = gw + gauss_off(nq);
  double* base = tabs + pp.tab_off[d];
  const int n0 = m * m, n1 = 2 * m * m, n2 = n1 + (m - 1) * (m - 1), total = n2 + (m - 1) * m;
  const double h = (r.hi - r.lo) / r.nel;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int type, i, j;
    if (idx < n0) { type = 0; i = idx / m; j = idx % m; }
    else if (idx < n1) { type = 1; i = (idx - n0) / m; j = (idx - n0) % m; }
    else if (idx < n2) { type = 2; i = (idx - n1) / (m - 1); j = (idx - n1) % (m - 1); }
    else { type = 3; i = (idx - n2) / m; j = (idx - n2) % m; }
    int tmin = max(0, max(i, j) - p), tmax = min(r.nel - 1, min(i, j));
    double acc = 0.0;
    for (int t = tmin; t <= tmax; ++t) {
      const bool ai_N = (i >= t && i <= t + p), aj_N = (j >= t && j <= t + p);
      const bool ai_D = (i >= t && i <= t + p - 1), aj_D = (j >= t && j <= t + p - 1);
      bool act;
      switch (type) {
        case 0: case 1: act = ai_N && aj_N; break;
        case 2: act = ai_D && aj_D; break;
        default: act = ai_D && aj_N; break;
      }
      if (!act) continue;
      const double lo_t = h * t + r.lo;
      for (int q = 0; q < nq; ++q) {
        const double x = lo_t + 0.5 * h * (g[q] + 1.0);
        const double wq = 0.5 * h * w[q];
        double N[TCF_MAXP + 1], D[TCF_MAXP], dN[TCF_MAXP + 1];
        eval_element(r, t, x, N, D, dN);
        double vi, vj;
        switch (type) {
          case 0: vi = N[i - t]; vj = N[j - t]; break;
          case 1: vi = dN[i - t]; vj = dN[j - t]; break;
          case 2: vi = D[i - t]; vj = D[j - t]; break;
          default: vi = D[i - t]; vj = dN[j - t]; break;
        }
        acc += wq * vi * vj;
      }
    }
    base[idx] = acc;
  }
}

// Basis values at the load quadrature points (p+3 per element): per point
// [x, w, N_0..N_{m-1}, N'_0..N'_{m-1}, D_0..D_{m-2}] (zeros off support).
__global__ void k_point_tables(const DevPatch* P, const double* gx, const double* gw,
                               double* ptab) {
  const int s = blockIdx.x / 3, d = blockIdx.x % 3;
  const DevPatch& pp = P[s];
  const Row1D r{pp.lo[d], pp.hi[d], pp.nel[d], pp.deg[d]};
  const int m = pp.m[d], p = r.p, nq = p + 3;
  const double* g = gx + gauss_off(nq);
  const double* w = gw + gauss_off(nq);
  const int stride = 3 * m + 1;
  const double h = (r.hi - r.lo) / r.nel;
  double* base = ptab + pp.ptab_off[d];
  const int npts = r.nel * nq;
  for (int ip = threadIdx.x; ip < npts; ip += blockDim.x) {
    const int t = ip / nq, q = ip % nq;
    const double x = (h * t + r.lo) + 0.5 * h * (g[q] + 1.0);
    double N[TCF_MAXP + 1], D[TCF_MAXP], dN[TCF_MAXP + 1];
    eval_element(r, t, x, N, D, dN);
    double* o = base + (int64_t)ip * stride;
    o[0] = x;
    o[1] = 0.5 * h * w[q];
    for (int i = 0; i < m; ++i) { o[2 + i] = 0.0; o[2 + m + i] = 0.0; }
    for (int i = 0; i < m - 1; ++i) o[2 + 2 * m + i] = 0.0;
    for (int j = 0; j <= p; ++j) { o[2 + t + j] = N[j]; o[2 + m + t + j] = dN[j]; }
    for (int j = 0; j < p; ++j) o[2 + 2 * m + t + j] = D[j];
  }
}

// ===========================================================================
// Patch matrix entries: W = sigma M + dt nu K on the edge basis
// x-edge (a,b,c) = D_a(x) N_b(y) N_c(z) e_x (cyclic for y, z)
// ===========================================================================
struct Tab1 {
  const double* Nn;
  const double* NdNd;
  const double* Dd;
  const double* DNd;
  int m;
  __device__ double nn(int i, int j) const { return Nn[i * m + j]; }
  __device__ double dndn(int i, int j) const { return NdNd[i * m + j]; }
  __device__ double dd(int i, int j) const { return Dd[i * (m - 1) + j]; }
  __device__ double dnd(int i, int j) const { return DNd[i * m + j]; }  // int D_i N'_j
};

__device__ inline Tab1 make_tab(const DevPatch& pp, const double* tabs, int d) {
  const int m = pp.m[d];
  const double* b = tabs + pp.tab_off[d];
  return Tab1{b, b + m * m, b + 2 * m * m, b + 2 * m * m + (m - 1) * (m - 1), m};
}

struct EdgeCode {
  int dir, a, b, c;
};

__device__ inline EdgeCode decode_local(const DevPatch& pp, int loc) {
  const int mx = pp.m[0], my = pp.m[1], mz = pp.m[2];
  const int nX = (mx - 1) * my * mz, nY = mx * (my - 1) * mz;
  EdgeCode e;
  if (loc < nX) {
    e.dir = 0; e.a = loc % (mx - 1); e.b = (loc / (mx - 1)) % my; e.c = loc / ((mx - 1) * my);
  } else if (loc < nX + nY) {
    const int l = loc - nX;
    e.dir = 1; e.a = l % mx; e.b = (l / mx) % (my - 1); e.c = l / (mx * (my - 1));
  } else {
    const int l = loc - nX - nY;
    e.dir = 2; e.a = l % mx; e.b = (l / mx) % my; e.c = l / (mx * my);
  }
  return e;
}

__device__ inline int encode_local(const DevPatch& pp, int dir, int a, int b, int c) {
  const int mx = pp.m[0], my = pp.m[1], mz = pp.m[2];
  const int nX = (mx - 1) * my * mz, nY = mx * (my - 1) * mz;
  if (dir == 0) return a + (mx - 1) * (b + my * c);
  if (dir == 1) return nX + a + mx * (b + (my - 1) * c);
  return nX + nY + a + mx * (b + my * c);
}

// Returns (M, K) entry pair for row edge u and column edge v (unscaled).
__device__ inline void mk_entry(const Tab1& X, const Tab1& Y, const Tab1& Z, const EdgeCode& u,
                                const EdgeCode& v, double& M, double& K) {
  M = 0.0;
  K = 0.0;
  const int a = u.a, b = u.b, c = u.c, a2 = v.a, b2 = v.b, c2 = v.c;
  if (u.dir == v.dir) {
    if (u.dir == 0) {
      const double dx = X.dd(a, a2);
      M = dx * Y.nn(b, b2) * Z.nn(c, c2);
      K = dx * (Y.nn(b, b2) * Z.dndn(c, c2) + Y.dndn(b, b2) * Z.nn(c, c2));
    } else if (u.dir == 1) {
      const double dy = Y.dd(b, b2);
      M = X.nn(a, a2) * dy * Z.nn(c, c2);
      K = dy * (X.nn(a, a2) * Z.dndn(c, c2) + X.dndn(a, a2) * Z.nn(c, c2));
    } else {
      const double dz = Z.dd(c, c2);
      M = X.nn(a, a2) * Y.nn(b, b2) * dz;
      K = dz * (X.nn(a, a2) * Y.dndn(b, b2) + X.dndn(a, a2) * Y.nn(b, b2));
    }
    return;
  }
  const int pr = u.dir * 3 + v.dir;
  switch (pr) {
    case 1:  // x row, y col: -int D_a N'_a2 . int N'_b D_b2 . int N_c N_c2
      K = -X.dnd(a, a2) * Y.dnd(b2, b) * Z.nn(c, c2); break;
    case 3:  // y row, x col
      K = -X.dnd(a2, a) * Y.dnd(b, b2) * Z.nn(c2, c); break;
    case 2:  // x row, z col: -int D_a N'_a2 . int N_b N_b2 . int N'_c D_c2
      K = -X.dnd(a, a2) * Y.nn(b, b2) * Z.dnd(c2, c); break;
    case 6:  // z row, x col
      K = -X.dnd(a2, a) * Y.nn(b2, b) * Z.dnd(c, c2); break;
    case 5:  // y row, z col: -int N_a N_a2 . int D_b N'_b2 . int N'_c D_c2
      K = -X.nn(a, a2) * Y.dnd(b, b2) * Z.dnd(c2, c); break;
    default:  // 7: z row, y col
      K = -X.nn(a2, a) * Y.dnd(b2, b) * Z.dnd(c, c2); break;
  }
}

// padded position -> kept index (-1 for padding)
__device__ inline int pad_to_r(const DevPatch& pp, int pos) {
  if (pos < pp.ni_pad) return pos < pp.n_i ? pos : -1;
  pos -= pp.ni_pad;
  if (pos < pp.nb_pad) return pos < pp.n_b ? pp.n_i + pos : -1;
  pos -= pp.nb_pad;
  return pos < pp.n_p ? pp.n_i + pp.n_b + pos : -1;
}

__device__ inline int find_job(const int* prefix, int njobs, int b) {
  int lo = 0, hi = njobs;  // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Dense assembly: one block per padded column of every patch.
template <class T>
__global__ void k_assemble(const DevPatch* P, const int* col_prefix, int np, const int* r_loc,
                           const double* tabs, double dt, T* A) {
  const int s = find_job(col_prefix, np, blockIdx.x);
  const DevPatch& pp = P[s];
  const int col = blockIdx.x - col_prefix[s];
  const int rc = pad_to_r(pp, col);
  const Tab1 X = make_tab(pp, tabs, 0), Y = make_tab(pp, tabs, 1), Z = make_tab(pp, tabs, 2);
  EdgeCode v{};
  if (rc >= 0) v = decode_local(pp, r_loc[pp.r_off + rc]);
  T* out = A + pp.A_off + (int64_t)col * pp.nr_pad;
  const double nudt = pp.nu * dt;
  for (int row = threadIdx.x; row < pp.nr_pad; row += blockDim.x) {
    const int rr = pad_to_r(pp, row);
    double val;
    if (rr < 0 || rc < 0) {
      val = (row == col) ? 1.0 : 0.0;
    } else {
      const EdgeCode u = decode_local(pp, r_loc[pp.r_off + rr]);
      double M, K;
      mk_entry(X, Y, Z, u, v, M, K);
      val = pp.sigma * M + nudt * K;
    }
    out[row] = (T)val;
  }
}

// Matrix-free y = W x (full) or y = sigma M x (mass only) on the kept
// unknowns of each listed patch, FP64.  x, y are kept-ordered vectors.
template <int C>
__global__ void k_wapply(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                         const int* r_loc, const int* loc2r, const double* tabs, double dt,
                         int mass_only, int nrhs, const double* x, double* y, int64_t ldv) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= row_prefix[nlist]) return;
  const int li = find_job(row_prefix, nlist, gi);
  const int s = plist[li];
  const DevPatch& pp = P[s];
  const int j = gi - row_prefix[li];
  // columns rhs0 .. rhs0 + C - 1 (those below nrhs): each matrix entry is
  // formed once and applied to all of them
  const int rhs0 = blockIdx.y * C;
  const int nc = min(C, nrhs - rhs0);
  const Tab1 X = make_tab(pp, tabs, 0), Y = make_tab(pp, tabs, 1), Z = make_tab(pp, tabs, 2);
  const EdgeCode u = decode_local(pp, r_loc[pp.r_off + j]);
  const double* xs = x + (int64_t)rhs0 * ldv + pp.r_off;
  const int* l2r = loc2r + pp.loc_off;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  const int px = pp.deg[0], py = pp.deg[1], pz = pp.deg[2];
  for (int dir = 0; dir < 3; ++dir) {
    if (mass_only && dir != u.dir) continue;
    const int na = pp.m[0] - (dir == 0), nb = pp.m[1] - (dir == 1), nc3 = pp.m[2] - (dir == 2);
    const int a0 = max(0, u.a - px), a1 = min(na - 1, u.a + px);
    const int b0 = max(0, u.b - py), b1 = min(nb - 1, u.b + py);
    const int c0 = max(0, u.c - pz), c1 = min(nc3 - 1, u.c + pz);
    for (int c = c0; c <= c1; ++c)
      for (int b = b0; b <= b1; ++b)
        for (int a = a0; a <= a1; ++a) {
          const int r2 = l2r[encode_local(pp, dir, a, b, c)];
          if (r2 < 0) continue;
          double M, K;
          mk_entry(X, Y, Z, u, EdgeCode{dir, a, b, c}, M, K);
          const double wv = mass_only ? pp.sigma * M : pp.sigma * M + pp.nu * dt * K;
#pragma unroll
          for (int q = 0; q < C; ++q)
            if (q < nc) acc[q] += wv * xs[(int64_t)q * ldv + r2];
        }
  }
#pragma unroll
  for (int q = 0; q < C; ++q)
    if (q < nc) y[(int64_t)(rhs0 + q) * ldv + pp.r_off + j] = acc[q];
}

// Curl-form load of one patch: jhat_e = int phi (curl w_e)_z, with
// (curl w)_z = -D_a N'_b N_c (x-edges), N'_a D_b N_c (y-edges), 0 (z-edges).
// phi holds the callback values on the patch's tensor grid of load points,
// one block of nx*ny*nz per excitation.
// Curl-form load of local kept edge j of a patch: the integral of
// phi (curl w_j)_z over the patch on the load points, phi given there
// (x fastest).  (curl w)_z is -D_a N'_b N_c for x-edges, N'_a D_b N_c for
// y-edges and 0 for z-edges.
__device__ double load_curl_edge(const DevPatch& pp, const EdgeCode& u, const double* ptab,
                                 const double* ph) {
  double val = 0.0;
  if (u.dir != 2) {
    const int mx = pp.m[0], my = pp.m[1], mz = pp.m[2];
    const int sx = 3 * mx + 1, sy = 3 * my + 1, sz = 3 * mz + 1;
    const double* TX = ptab + pp.ptab_off[0];
    const double* TY = ptab + pp.ptab_off[1];
    const double* TZ = ptab + pp.ptab_off[2];
    const int NX = pp.nq_load[0], NY = pp.nq_load[1];
    const int qx = pp.deg[0] + 3, qy = pp.deg[1] + 3, qz = pp.deg[2] + 3;
    const int px = pp.deg[0], py = pp.deg[1], pz = pp.deg[2];
    (void)mz;
    // element ranges where each factor is active
    int tx0, tx1, ty0, ty1;
    if (u.dir == 0) {  // D_a(x): t in [a-p+1, a];  N'_b(y): t in [b-p, b]
      tx0 = u.a - px + 1; tx1 = u.a; ty0 = u.b - py; ty1 = u.b;
    } else {           // N'_a(x): t in [a-p, a];    D_b(y): t in [b-p+1, b]
      tx0 = u.a - px; tx1 = u.a; ty0 = u.b - py + 1; ty1 = u.b;
    }
    tx0 = max(tx0, 0); tx1 = min(tx1, pp.nel[0] - 1);
    ty0 = max(ty0, 0); ty1 = min(ty1, pp.nel[1] - 1);
    const int tz0 = max(u.c - pz, 0), tz1 = min(u.c, pp.nel[2] - 1);
    for (int iz = tz0 * qz; iz < (tz1 + 1) * qz; ++iz) {
      const double* oz = TZ + (int64_t)iz * sz;
      const double fz = oz[1] * oz[2 + u.c];  // w N_c(z)
      if (fz == 0.0) continue;
      for (int iy = ty0 * qy; iy < (ty1 + 1) * qy; ++iy) {
        const double* oy = TY + (int64_t)iy * sy;
        const double fy = oy[1] * (u.dir == 0 ? oy[2 + my + u.b] : oy[2 + 2 * my + u.b]);
        if (fy == 0.0) continue;
        const double fyz = fy * fz;
        const double* prow = ph + (int64_t)NX * (iy + (int64_t)NY * iz);
        double sx_acc = 0.0;
        for (int ix = tx0 * qx; ix < (tx1 + 1) * qx; ++ix) {
          const double* ox = TX + (int64_t)ix * sx;
          const double fx = ox[1] * (u.dir == 0 ? ox[2 + 2 * mx + u.a] : ox[2 + mx + u.a]);
          sx_acc += fx * prow[ix];
        }
        val += sx_acc * fyz;
      }
    }
    if (u.dir == 0) val = -val;
  }
  return val;
}

// Volume-form load of local kept edge j of a patch (Sec. 2.2: the integral
// of F . w_j): sum over the load points of w F_dir(x) w_j,dir(x), where an
// edge of direction dir is D in that direction and N in the other two.  F
// holds the field at the load points, component fastest:
// F[c + 3 (ix + NX (iy + NY iz))].
__device__ double load_vec_edge(const DevPatch& pp, const EdgeCode& u, const double* ptab,
                                const double* F) {
  const int id[3] = {u.a, u.b, u.c};
  const double* T[3];
  int stride[3], col[3], nq[3], t0[3], t1[3];
  for (int a = 0; a < 3; ++a) {
    const int m = pp.m[a], p = pp.deg[a];
    const bool isD = a == u.dir;
    T[a] = ptab + pp.ptab_off[a];
    stride[a] = 3 * m + 1;
    nq[a] = p + 3;
    col[a] = isD ? 2 + 2 * m + id[a] : 2 + id[a];  // D_i or N_i column of the table
    // elements where the factor is nonzero: D_i on [i-p+1, i], N_i on [i-p, i]
    t0[a] = max(isD ? id[a] - p + 1 : id[a] - p, 0);
    t1[a] = min(id[a], pp.nel[a] - 1);
  }
  const int NX = pp.nq_load[0], NY = pp.nq_load[1];
  const double* f = F + u.dir;
  double val = 0.0;
  for (int iz = t0[2] * nq[2]; iz < (t1[2] + 1) * nq[2]; ++iz) {
    const double* oz = T[2] + (int64_t)iz * stride[2];
    const double fz = oz[1] * oz[col[2]];
    if (fz == 0.0) continue;
    for (int iy = t0[1] * nq[1]; iy < (t1[1] + 1) * nq[1]; ++iy) {
      const double* oy = T[1] + (int64_t)iy * stride[1];
      const double fy = oy[1] * oy[col[1]];
      if (fy == 0.0) continue;
      const double* frow = f + 3 * (int64_t)NX * (iy + (int64_t)NY * iz);
      double acc = 0.0;
      for (int ix = t0[0] * nq[0]; ix < (t1[0] + 1) * nq[0]; ++ix) {
        const double* ox = T[0] + (int64_t)ix * stride[0];
        acc += ox[1] * ox[col[0]] * frow[3 * ix];
      }
      val += acc * fy * fz;
    }
  }
  return val;
}

// Source loads of a batch of patches in one launch: job x covers patch
// jobs[x].s with its field values at F + jobs[x].f_off (per excitation k,
// F_k follows at k times the patch's point count, times 3 for vector
// fields); out[k][r_off + j] += jobs[x].scale * load of kept edge j.
// vec = 0: curl form (phi), 1: volume form (vector field).
__global__ void k_load_batch(const DevPatch* P, const LoadJob* jobs, const int* prefix,
                             int njobs, const int* r_loc, const double* ptab, const double* F,
                             int vec, double* out, int64_t ldv) {
  const int jx = find_job(prefix, njobs, blockIdx.x);
  const LoadJob jb = jobs[jx];
  const DevPatch& pp = P[jb.s];
  const int j = (blockIdx.x - prefix[jx]) * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (j >= pp.n_r) return;
  const EdgeCode u = decode_local(pp, r_loc[pp.r_off + j]);
  const int64_t npts = (int64_t)pp.nq_load[0] * pp.nq_load[1] * pp.nq_load[2];
  const double* f = F + jb.f_off + (int64_t)k * (vec ? 3 : 1) * npts;
  const double v = vec ? load_vec_edge(pp, u, ptab, f) : load_curl_edge(pp, u, ptab, f);
  out[(int64_t)k * ldv + pp.r_off + j] += jb.scale * v;
}

// ===========================================================================
// Batched partial Cholesky (lower, column-major, right-looking, 32 panels)
// ===========================================================================
template <class T>
__global__ void k_potrf_panel(const FactorJob* jobs, int k, T* A, int* fail) {
  const FactorJob jb = jobs[blockIdx.x];
  const int col0 = jb.c_begin + TCF_NB * k;
  if (col0 >= jb.c_end) return;
  __shared__ T L[TCF_NB][TCF_NB + 1];
  T* a = A + jb.off;
  const int64_t ld = jb.ld;
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += blockDim.x) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    L[r][c] = (r >= c) ? a[(col0 + r) + (int64_t)(col0 + c) * ld] : T(0);
  }
  __syncthreads();
  for (int j = 0; j < TCF_NB; ++j) {
    if (threadIdx.x == 0) {
      T d = L[j][j];
      if (!(d > T(0))) {
        atomicExch(fail, jb.tag + 2);
        d = T(1);
      }
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    if (threadIdx.x > j && threadIdx.x < TCF_NB) L[threadIdx.x][j] /= L[j][j];
    __syncthreads();
    for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += blockDim.x) {
      const int i = idx % TCF_NB, l = idx / TCF_NB;
      if (l > j && i >= l) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += blockDim.x) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    if (r >= c) a[(col0 + r) + (int64_t)(col0 + c) * ld] = L[r][c];
  }
}

// Rows below the panel: L_ik = A_ik L_kk^-T.  64 rows per block, one per lane.
template <class T>
__global__ void k_trsm_panel(const FactorJob* jobs, const int* prefix, int njobs, int k, T* A) {
  const int j = find_job(prefix, njobs, blockIdx.x);
  const FactorJob jb = jobs[j];
  const int chunk = blockIdx.x - prefix[j];
  const int col0 = jb.c_begin + TCF_NB * k;
  __shared__ T L[TCF_NB][TCF_NB + 1];
  T* a = A + jb.off;
  const int64_t ld = jb.ld;
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += blockDim.x) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    L[r][c] = (r >= c) ? a[(col0 + r) + (int64_t)(col0 + c) * ld] : T(0);
  }
  __syncthreads();
  const int row = col0 + TCF_NB + chunk * 64 + threadIdx.x;
  if (row >= jb.n) return;
  T x[TCF_NB];
#pragma unroll
  for (int c = 0; c < TCF_NB; ++c) x[c] = a[row + (int64_t)(col0 + c) * ld];
#pragma unroll
  for (int c = 0; c < TCF_NB; ++c) {
    T v = x[c];
#pragma unroll
    for (int l = 0; l < c; ++l) v -= x[l] * L[c][l];
    x[c] = v / L[c][c];
  }
#pragma unroll
  for (int c = 0; c < TCF_NB; ++c) a[row + (int64_t)(col0 + c) * ld] = x[c];
}

// Trailing updates of the blocked Cholesky, C -= L_I L_J^T on 64 x 64 tiles
// (entries on or below the diagonal).  Panels of TCF_NB columns are grouped
// into super-panels of TCF_SP panels.
// mode 0, after panel k: K = the panel's columns [col0, col0 + TCF_NB); rows
//   from trail0 = col0 + TCF_NB to n, columns from trail0 to the end of the
//   super-panel (what the next panels of the super-panel need), tiles
//   enumerated as a rectangle.
// mode 1, after the last panel of super-panel k / TCF_SP: K = all of its
//   columns [p0, p_end); rows and columns from p_end to n (lower tiles):
//   each trailing tile is read and written once per super-panel.
#define TCF_SP 4
template <class T>
__global__ void k_syrk_blk(const FactorJob* jobs, const int* prefix, int njobs, int k, int mode,
                           T* A) {
  const int j = find_job(prefix, njobs, blockIdx.x);
  const FactorJob jb = jobs[j];
  const int t = blockIdx.x - prefix[j];
  const int n = jb.n;
  const int sp = k / TCF_SP;
  const int p0 = jb.c_begin + TCF_NB * TCF_SP * sp;
  const int p_end = min(p0 + TCF_NB * TCF_SP, jb.c_end);
  int k0, k1, row0, cl0, cmax;
  if (mode == 0) {
    const int col0 = jb.c_begin + TCF_NB * k;
    const int trail0 = col0 + TCF_NB;
    const int nJ = (p_end - trail0 + 63) / 64;
    const int I = t / nJ, J = t % nJ;
    k0 = col0;
    k1 = col0 + TCF_NB;
    row0 = trail0 + 64 * I;
    cl0 = trail0 + 64 * J;
    cmax = p_end;
    if (row0 + 63 < cl0) return;  // wholly above the diagonal
  } else {
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    k0 = p0;
    k1 = p_end;
    row0 = p_end + 64 * I;
    cl0 = p_end + 64 * J;
    cmax = n;
  }
  __shared__ T LI[TCF_NB][64 + 1];
  __shared__ T LJ[TCF_NB][64 + 1];
  T* a = A + jb.off;
  const int64_t ld = jb.ld;
  {
    // On the matrix cores (Mfma16<T>: FP64 in FP64, FP32 accumulating in
    // FP32): wave w owns rows 32 (w & 1) .. + 32 and columns
    // 32 (w >> 1) .. + 32 of the tile as 2 x 2 subtiles of 16 x 16.  The
    // operands are swapped (A from LJ, B from LI), so the accumulator holds
    // C^T: element e of lane l is C[rb + l % 16][cb + row(l / 16, e)], i.e.
    // lanes run along rows and the update of C stays coalesced.
    typedef Mfma16<T> M;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
    const int rb = 32 * (w & 1), cb = 32 * (w >> 1);
    typename M::acc acc4[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc4[u][v] = typename M::acc{T(0), T(0), T(0), T(0)};
    for (int kc = k0; kc < k1; kc += TCF_NB) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < TCF_NB * 64; idx += blockDim.x) {
        const int r = idx % 64, c = idx / 64;
        LI[c][r] = (row0 + r < n) ? a[(row0 + r) + (int64_t)(kc + c) * ld] : T(0);
        LJ[c][r] = (cl0 + r < cmax) ? a[(cl0 + r) + (int64_t)(kc + c) * ld] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int k4 = 0; k4 < TCF_NB; k4 += 4) {
        const T b0 = LI[k4 + lk][rb + li], b1 = LI[k4 + lk][rb + 16 + li];
        const T a0 = LJ[k4 + lk][cb + li], a1 = LJ[k4 + lk][cb + 16 + li];
        acc4[0][0] = M::mma(a0, b0, acc4[0][0]);
        acc4[0][1] = M::mma(a1, b0, acc4[0][1]);
        acc4[1][0] = M::mma(a0, b1, acc4[1][0]);
        acc4[1][1] = M::mma(a1, b1, acc4[1][1]);
      }
    }
    // acc4[u][v]: rows rb + 16 u + li, columns cb + 16 v + row(lk, e)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int R = row0 + rb + 16 * u + li;
          const int C = cl0 + cb + 16 * v + M::row(lk, e);
          if (R < n && C < cmax && R >= C) a[R + (int64_t)C * ld] -= acc4[u][v][e];
        }
  }
}

// ===========================================================================
// Fills between factorisation phases
// ===========================================================================
// S_bb (full symmetric, ld nb_pad) from the Schur block left after the
// interior columns were eliminated.
template <class T>
__global__ void k_copy_sbb(const DevPatch* P, const int* col_prefix, int np, const T* A, T* S) {
  const int s = find_job(col_prefix, np, blockIdx.x);
  const DevPatch& pp = P[s];
  const int c = blockIdx.x - col_prefix[s];
  const T* a = A + pp.A_off;
  T* o = S + pp.S_off + (int64_t)c * pp.nb_pad;
  for (int r = threadIdx.x; r < pp.nb_pad; r += blockDim.x) {
    T v = T(0);
    if (r < pp.n_b) {
      const int R = pp.ni_pad + max(r, c), C = pp.ni_pad + min(r, c);
      v = a[R + (int64_t)C * pp.nr_pad];
    }
    o[r] = v;
  }
}

// G = [I | L_pb^T] over nb_pad rows, n_b + n_p columns.
template <class T>
__global__ void k_fill_G(const DevPatch* P, const int* col_prefix, int np, const T* A, T* G) {
  const int s = find_job(col_prefix, np, blockIdx.x);
  const DevPatch& pp = P[s];
  const int c = blockIdx.x - col_prefix[s];
  const T* a = A + pp.A_off;
  T* o = G + pp.G_off + (int64_t)c * pp.nb_pad;
  for (int r = threadIdx.x; r < pp.nb_pad; r += blockDim.x) {
    T v = T(0);
    if (r < pp.n_b) {
      if (c < pp.n_b) v = (r == c) ? T(1) : T(0);
      else v = a[(pp.ni_pad + pp.nb_pad + (c - pp.n_b)) + (int64_t)(pp.ni_pad + r) * pp.nr_pad];
    }
    o[r] = v;
  }
}

// Q^T right-hand side [I | L_bi^T | L_pi^T] over ni_pad rows, n_r columns.
template <class T>
__global__ void k_fill_Q(const DevPatch* P, const int* col_prefix, int np, const T* A, T* Q) {
  const int s = find_job(col_prefix, np, blockIdx.x);
  const DevPatch& pp = P[s];
  const int c = blockIdx.x - col_prefix[s];
  const T* a = A + pp.A_off;
  T* o = Q + pp.Q_off + (int64_t)c * pp.ni_pad;
  int srcrow = -1;
  if (c >= pp.n_i && c < pp.n_i + pp.n_b) srcrow = pp.ni_pad + (c - pp.n_i);
  else if (c >= pp.n_i + pp.n_b) srcrow = pp.ni_pad + pp.nb_pad + (c - pp.n_i - pp.n_b);
  for (int r = threadIdx.x; r < pp.ni_pad; r += blockDim.x) {
    T v = T(0);
    if (r < pp.n_i) {
      if (srcrow < 0) v = (r == c) ? T(1) : T(0);
      else v = a[srcrow + (int64_t)r * pp.nr_pad];
    }
    o[r] = v;
  }
}

// S_Pi += N_s^T S_pp N_s for one patch (launched per patch in sequence).
template <class T>
__global__ void k_coarse_add(const DevPatch* P, int s, const int* p_rank, const T* A, double* SPi,
                             int ldc) {
  const DevPatch& pp = P[s];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pp.n_p * pp.n_p) return;
  const int i = idx % pp.n_p, j = idx / pp.n_p;
  const int R = pp.ni_pad + pp.nb_pad + max(i, j), C = pp.ni_pad + pp.nb_pad + min(i, j);
  const double v = (double)A[pp.A_off + R + (int64_t)C * pp.nr_pad];
  const int gi = p_rank[pp.p_off + i], gj = p_rank[pp.p_off + j];
  SPi[gi + (int64_t)gj * ldc] += v;
}

__global__ void k_set_identity_pad(double* M, int ld, int n0, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - n0) return;
  M[(n0 + i) + (int64_t)(n0 + i) * ld] = 1.0;
}


// ---------------------------------------------------------------------------
// Triangular solves on the matrix cores: FP64 in FP64, FP32 accumulating
// in FP32 (Mfma16<T> holds the instruction and its lane layout).
// ---------------------------------------------------------------------------

// Inverses of the 32 x 32 diagonal blocks of each job's lower factor:
// D[(dprefix[job] + kb) * 1024 + r + 32 c] = (L_kb,kb)^-1 [r][c].  One block
// of 64 threads per diagonal block; thread c < 32 forward-substitutes the
// unit vector e_c.
template <class T>
__global__ void __launch_bounds__(64) k_trsm_dinv(const TrsmJob* jobs, const int* dprefix,
                                                  int njobs, const T* Lb, T* D) {
  const int jx = find_job(dprefix, njobs, blockIdx.x);
  const TrsmJob jb = jobs[jx];
  const int kb = blockIdx.x - dprefix[jx];
  __shared__ T Ls[TCF_NB][TCF_NB + 1];
  __shared__ T Ys[TCF_NB][TCF_NB + 1];
  const T* L = Lb + jb.l_off;
  const int64_t ldl = jb.ldl;
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += 64) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    Ls[r][c] = L[(jb.l_row0 + kb * TCF_NB + r) + (int64_t)(jb.l_row0 + kb * TCF_NB + c) * ldl];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < TCF_NB) {
    for (int r = 0; r < TCF_NB; ++r) {
      T v = (r == c) ? T(1) : T(0);
      if (r >= c) {
        for (int l = c; l < r; ++l) v -= Ls[r][l] * Ys[l][c];
        v /= Ls[r][r];
      }
      Ys[r][c] = v;
    }
  }
  __syncthreads();
  T* out = D + (int64_t)blockIdx.x * TCF_NB * TCF_NB;
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += 64) {
    const int r = idx % TCF_NB, cc = idx / TCF_NB;
    out[idx] = Ys[r][cc];
  }
}

// Solves L X = B (forward) or L^T X = B (backward) for a batch of jobs,
// right-looking over panels of TCF_RL_PANEL row blocks (32 rows each): step
// s takes the panel of row blocks kb = P s + i, i < P (forward; backward
// kb = nblk - 1 - P s - i) of every job in two launches.  The first, per
// column block, solves the panel's blocks in order, X_kb = D_kb (B_kb -
// sum of the panel's earlier blocks L_kb,kb' X_kb') (D_kb^T and L^T
// backward).  The second subtracts the whole panel from every row block
// after it (before it backward), B_j -= sum_i L_j,kb_i X_kb_i, each output
// tile read and written once per panel, every tile of every job in
// parallel.  With identity right-hand sides (tri > 0) the blocks that stay
// zero are skipped.
#define TCF_RL_PANEL 4
__device__ inline int rl_kb(const TrsmJob& jb, int s, int i, int fwd) {
  const int nblk = jb.n / TCF_NB;
  return fwd ? TCF_RL_PANEL * s + i : nblk - 1 - TCF_RL_PANEL * s - i;
}
__device__ inline bool rl_zero_block(const TrsmJob& jb, int kb, int c0, int fwd) {
  if (c0 + 64 > jb.tri) return false;
  if (fwd) return kb < c0 / TCF_NB;
  return kb > (c0 + 63) / TCF_NB;
}

// Stage the 32 x 32 block of L at row block lr, column block lc into Ls and
// the 32 x 64 block of B at row block kb, columns c0.., into Xs.
template <class T>
__device__ inline void rl_stage(const TrsmJob& jb, const T* L, const T* B, int lr, int lc, int kb,
                                int c0, T (*Ls)[TCF_NB + 1], T (*Xs)[64 + 1]) {
  const int64_t ldl = jb.ldl, ldb = jb.ldb;
  for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += 256) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    Ls[r][c] = L[(jb.l_row0 + lr * TCF_NB + r) + (int64_t)(jb.l_row0 + lc * TCF_NB + c) * ldl];
  }
  for (int idx = threadIdx.x; idx < TCF_NB * 64; idx += 256) {
    const int r = idx % TCF_NB, c = idx / TCF_NB;
    Xs[r][c] = (c0 + c < jb.ncols) ? B[(kb * TCF_NB + r) + (int64_t)(c0 + c) * ldb] : T(0);
  }
}

// acc -= A X with A = Ls (forward) or Ls^T (backward), X = Xs, for the
// wave's 16 columns and both 16-row halves
template <class T>
__device__ inline void rl_mfma_sub(const T (*Ls)[TCF_NB + 1], const T (*Xs)[64 + 1], int fwd, int w,
                                   int li, int lk, typename Mfma16<T>::acc& a0,
                                   typename Mfma16<T>::acc& a1) {
#pragma unroll
  for (int k0 = 0; k0 < TCF_NB; k0 += 4) {
    const T bv = Xs[k0 + lk][16 * w + li];
    const T v0 = fwd ? Ls[li][k0 + lk] : Ls[k0 + lk][li];
    const T v1 = fwd ? Ls[16 + li][k0 + lk] : Ls[k0 + lk][16 + li];
    a0 = Mfma16<T>::mma(-v0, bv, a0);
    a1 = Mfma16<T>::mma(-v1, bv, a1);
  }
}

template <class T>
__global__ void __launch_bounds__(256) k_trsm_rl_diag(const TrsmJob* jobs, const int* cprefix,
                                                      const int* dprefix, int njobs, int s,
                                                      int fwd, const T* Lb, const T* D, T* Bb) {
  typedef Mfma16<T> M;
  const int jx = find_job(cprefix, njobs, blockIdx.x);
  const TrsmJob jb = jobs[jx];
  const int nblk = jb.n / TCF_NB;
  const int c0 = (blockIdx.x - cprefix[jx]) * 64;
  __shared__ T Ls[TCF_NB][TCF_NB + 1];
  __shared__ T Xs[TCF_NB][64 + 1];
  const T* L = Lb + jb.l_off;
  T* B = Bb + jb.b_off;
  const int64_t ldb = jb.ldb;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  const int col = c0 + 16 * w + li;
  const bool colok = col < jb.ncols;
  for (int i = 0; i < TCF_RL_PANEL; ++i) {
    const int kb = rl_kb(jb, s, i, fwd);
    if (kb < 0 || kb >= nblk) break;
    if (rl_zero_block(jb, kb, c0, fwd)) continue;
    typename M::acc a0, a1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a0[e] = colok ? B[(kb * TCF_NB + M::row(lk, e)) + (int64_t)col * ldb] : T(0);
      a1[e] = colok ? B[(kb * TCF_NB + 16 + M::row(lk, e)) + (int64_t)col * ldb] : T(0);
    }
    // earlier blocks of this panel (already solved and stored by this block)
    for (int q = 0; q < i; ++q) {
      const int kq = rl_kb(jb, s, q, fwd);
      if (rl_zero_block(jb, kq, c0, fwd)) continue;
      __syncthreads();
      rl_stage(jb, L, B, fwd ? kb : kq, fwd ? kq : kb, kq, c0, Ls, Xs);
      __syncthreads();
      rl_mfma_sub(Ls, Xs, fwd, w, li, lk, a0, a1);
    }
    // X_kb = D_kb acc (D_kb^T backward) through LDS
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Xs[M::row(lk, e)][16 * w + li] = a0[e];
      Xs[16 + M::row(lk, e)][16 * w + li] = a1[e];
    }
    const T* Dk = D + ((int64_t)dprefix[jx] + kb) * TCF_NB * TCF_NB;
    for (int idx = threadIdx.x; idx < TCF_NB * TCF_NB; idx += 256)
      Ls[idx % TCF_NB][idx / TCF_NB] = Dk[idx];
    __syncthreads();
    typename M::acc x0 = {T(0), T(0), T(0), T(0)}, x1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k0 = 0; k0 < TCF_NB; k0 += 4) {
      const T bv = Xs[k0 + lk][16 * w + li];
      const T v0 = fwd ? Ls[li][k0 + lk] : Ls[k0 + lk][li];
      const T v1 = fwd ? Ls[16 + li][k0 + lk] : Ls[k0 + lk][16 + li];
      x0 = M::mma(v0, bv, x0);
      x1 = M::mma(v1, bv, x1);
    }
    if (colok) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        B[(kb * TCF_NB + M::row(lk, e)) + (int64_t)col * ldb] = x0[e];
        B[(kb * TCF_NB + 16 + M::row(lk, e)) + (int64_t)col * ldb] = x1[e];
      }
    }
    __syncthreads();  // the stores are read back by the next block of the panel
  }
}

// tprefix: row s of a (steps x (njobs + 1)) table, the prefix over jobs of
// the tiles that step s updates (row blocks after the panel forward, before
// it backward, times column blocks)
template <class T>
__global__ void __launch_bounds__(256) k_trsm_rl_update(const TrsmJob* jobs, const int* tprefix,
                                                        int njobs, int s, int fwd, const T* Lb,
                                                        T* Bb) {
  typedef Mfma16<T> M;
  const int jx = find_job(tprefix, njobs, blockIdx.x);
  const TrsmJob jb = jobs[jx];
  const int nblk = jb.n / TCF_NB;
  const int ncb = (jb.ncols + 63) / 64;
  const int t = blockIdx.x - tprefix[jx];
  const int first = fwd ? TCF_RL_PANEL * (s + 1) : 0;  // first row block updated
  const int j = first + t / ncb;
  const int c0 = (t % ncb) * 64;
  __shared__ T Ls[TCF_NB][TCF_NB + 1];
  __shared__ T Xs[TCF_NB][64 + 1];
  const T* L = Lb + jb.l_off;
  T* B = Bb + jb.b_off;
  const int64_t ldb = jb.ldb;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  const int col = c0 + 16 * w + li;
  const bool colok = col < jb.ncols;
  typename M::acc a0 = {T(0), T(0), T(0), T(0)}, a1 = {T(0), T(0), T(0), T(0)};
  bool any = false;
  for (int i = 0; i < TCF_RL_PANEL; ++i) {
    const int kb = rl_kb(jb, s, i, fwd);
    if (kb < 0 || kb >= nblk) break;
    if (rl_zero_block(jb, kb, c0, fwd)) continue;
    any = true;
    __syncthreads();
    rl_stage(jb, L, B, fwd ? j : kb, fwd ? kb : j, kb, c0, Ls, Xs);
    __syncthreads();
    rl_mfma_sub(Ls, Xs, fwd, w, li, lk, a0, a1);
  }
  if (!any || !colok) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    B[(j * TCF_NB + M::row(lk, e)) + (int64_t)col * ldb] += a0[e];
    B[(j * TCF_NB + 16 + M::row(lk, e)) + (int64_t)col * ldb] += a1[e];
  }
}


// ===========================================================================
// Per-step matrix-vector products (FP64 vectors, T-typed matrices)
// ===========================================================================
__device__ inline double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Column dots over jobs: out[j] = sum_r M[r + j ld] x[r].  A block of 4
// waves covers TCF_DOT_CPB columns, each wave TCF_DOT_CPW columns at once;
// each lane reads 16 bytes (2 doubles / 4 floats) of a column per load, so a
// wave load covers 128 / 256 rows.  Columns are zero beyond nrows up to the
// padded leading dimension, and x is staged through LDS (zero padded) in
// chunks of TCF_XCH entries.
// xmode 0: x[r] = xv[x_off + r]; xmode 1: x[r] = xscale * sgn * xv[gidx].
#define TCF_XCH 4096
#define TCF_DOT_CPW 8
#define TCF_DOT_CPB (4 * TCF_DOT_CPW)
template <class T> struct Vec16;
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };

template <class T>
__device__ inline void vdot(const typename Vec16<T>::type& v, const double* x, double& acc);
template <>
__device__ inline void vdot<double>(const double2& v, const double* x, double& acc) {
  acc += v.x * x[0] + v.y * x[1];
}
template <>
__device__ inline void vdot<float>(const float4& v, const double* x, double& acc) {
  acc += (double)v.x * x[0] + (double)v.y * x[1] + (double)v.z * x[2] + (double)v.w * x[3];
}

template <class T>
__global__ void __launch_bounds__(256) k_dotcols(const DotJob* jobs, const int* prefix, int njobs,
                                                 const T* Mb, int xmode, const double* xv,
                                                 const int* gidx, const signed char* gsgn,
                                                 double xscale, double* out, const int* done) {
  if (done && *done) return;
  typedef typename Vec16<T>::type VT;
  constexpr int V = Vec16<T>::n;
  const int jx = find_job(prefix, njobs, blockIdx.x);
  const DotJob jb = jobs[jx];
  const int cblk = (blockIdx.x - prefix[jx]) * TCF_DOT_CPB;
  __shared__ double xs[TCF_XCH];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const T* M = Mb + jb.m_off;
  const int64_t ld = jb.ld;
  const int cA = cblk + wave * TCF_DOT_CPW;
  double acc[TCF_DOT_CPW];
  const VT* colp[TCF_DOT_CPW];
#pragma unroll
  for (int q = 0; q < TCF_DOT_CPW; ++q) {
    acc[q] = 0.0;
    const int c = min(cA + q, jb.ncols - 1);
    colp[q] = reinterpret_cast<const VT*>(M + (int64_t)c * ld);
  }
  const int nrv = (jb.nrows + V - 1) / V * V;
  for (int r0 = 0; r0 < nrv; r0 += TCF_XCH) {
    const int rn = min(TCF_XCH, nrv - r0);
    if (r0 > 0) __syncthreads();
    for (int r = threadIdx.x; r < rn; r += blockDim.x) {
      const int R = r0 + r;
      double v = 0.0;
      if (R < jb.nrows)
        v = (xmode == 0) ? xv[jb.x_off + R]
                         : xscale * (double)gsgn[jb.x_off + R] * xv[gidx[jb.x_off + R]];
      xs[r] = v;
    }
    __syncthreads();
    if (cA < jb.ncols) {
      for (int r = lane * V; r < rn; r += 64 * V) {
        VT v[TCF_DOT_CPW];
#pragma unroll
        for (int q = 0; q < TCF_DOT_CPW; ++q) v[q] = colp[q][(r0 + r) / V];
#pragma unroll
        for (int q = 0; q < TCF_DOT_CPW; ++q) vdot<T>(v[q], xs + r, acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TCF_DOT_CPW; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0 && cA + q < jb.ncols) out[jb.out_off + cA + q] = v;
  }
}

// Row stripes: out[r] = base[base_off + r] + alpha * sum_j M[r + (c0+j) ld] y[j].
// A block covers 64*V rows (each lane V consecutive rows, one 16-byte load
// per column); 4 waves split the columns (8 in flight each) and reduce in
// LDS.  y is staged through LDS in chunks.  y[j] = yv[yidx[y_off + j]] or
// yv[y_off + j].  tri != 0: M[r, c0 + j] = 0 for j < r (upper-triangular
// leading block), so each stripe starts at its own first row.
template <class T>
__global__ void __launch_bounds__(256) k_axpyrows(const AxpyJob* jobs, const int* prefix,
                                                  int njobs, const T* Mb, const double* yv,
                                                  const int* yidx, const double* base,
                                                  const int* base_off, double alpha, double* out,
                                                  int tri, const int* done) {
  if (done && *done) return;
  typedef typename Vec16<T>::type VT;
  constexpr int V = Vec16<T>::n;
  const int jx = find_job(prefix, njobs, blockIdx.x);
  const AxpyJob jb = jobs[jx];
  const int r0 = (blockIdx.x - prefix[jx]) * 64 * V;
  __shared__ double ys[TCF_XCH];
  __shared__ double red[4][64 * 4];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = r0 + lane * V;
  const T* M = Mb + jb.m_off;
  const int64_t ld = jb.ld;
  double acc[V];
#pragma unroll
  for (int k = 0; k < V; ++k) acc[k] = 0.0;
  const int jstart = tri ? r0 : 0;
  for (int j0 = jstart; j0 < jb.ncols; j0 += TCF_XCH) {
    const int jn = min(TCF_XCH, jb.ncols - j0);
    if (j0 > jstart) __syncthreads();
    for (int j = threadIdx.x; j < jn; j += blockDim.x)
      ys[j] = yidx ? yv[yidx[jb.y_off + j0 + j]] : yv[jb.y_off + j0 + j];
    __syncthreads();
    if (r < jb.nrows) {
      const T* Mc = M + r + (int64_t)(jb.c0 + j0) * ld;
      int j = wave;
      for (; j + 4 * 7 < jn; j += 4 * 8) {
        VT v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const VT*>(Mc + (int64_t)(j + 4 * u) * ld);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double yj = ys[j + 4 * u];
          const T* e = reinterpret_cast<const T*>(&v[u]);
#pragma unroll
          for (int k = 0; k < V; ++k) acc[k] += (double)e[k] * yj;
        }
      }
      for (; j < jn; j += 4) {
        const VT v = *reinterpret_cast<const VT*>(Mc + (int64_t)j * ld);
        const T* e = reinterpret_cast<const T*>(&v);
        const double yj = ys[j];
#pragma unroll
        for (int k = 0; k < V; ++k) acc[k] += (double)e[k] * yj;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < V; ++k) red[wave][lane * V + k] = acc[k];
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * V; t += blockDim.x) {
    const int R = r0 + t;
    if (R < jb.nrows) {
      const double s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
      const double b = base ? base[base_off[jx] + R] : 0.0;
      out[jb.out_off + R] = b + alpha * s;
    }
  }
}

// Condensation of a kept-ordered right-hand side f (conductor patches):
// ygg[j] += (j < n_i) ? (Q^T[:,j] . f_i) : (f[j] - Q^T[:,j] . f_i),
// where Q^T[:, j] has nonzeros only in rows <= j for j < n_i.
template <class T>
__global__ void __launch_bounds__(256) k_condense(const DevPatch* P, const int* plist,
                                                  const int* prefix, int nlist, const T* Q,
                                                  const double* f, double* ygg, int64_t ldv) {
  const int li = find_job(prefix, nlist, blockIdx.x);
  const DevPatch& pp = P[plist[li]];
  const int rhs = blockIdx.y;
  const int cblk = (blockIdx.x - prefix[li]) * 16;
  __shared__ double xs[TCF_XCH];
  const double* fr = f + (int64_t)rhs * ldv + pp.r_off;
  double* yr = ygg + (int64_t)rhs * ldv + pp.r_off;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const T* M = Q + pp.Q_off;
  const int64_t ld = pp.ni_pad;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int nrq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = cblk + wave * 4 + q;
    nrq[q] = (col >= pp.n_r) ? 0 : ((col < pp.n_i) ? col + 1 : pp.n_i);
  }
  // the wave's 4 columns and 4 row groups per pass: 16 independent loads in
  // flight per lane (addresses clamped into the column, products masked,
  // so no branch separates the loads); the pass count follows the longest
  // of the 4 columns, so the zero part of triangular columns is not read
  int colc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) colc[q] = min(cblk + wave * 4 + q, pp.n_r - 1);
  for (int r0 = 0; r0 < pp.n_i; r0 += TCF_XCH) {
    const int rn = min(TCF_XCH, pp.n_i - r0);
    if (r0 > 0) __syncthreads();
    for (int r = threadIdx.x; r < rn; r += blockDim.x) xs[r] = fr[r0 + r];
    __syncthreads();
    int lim[4], lmax = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lim[q] = max(0, min(rn, nrq[q] - r0));
      lmax = max(lmax, lim[q]);
    }
    for (int base = 0; base < lmax; base += 256) {
      double v[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int rr = min(base + 64 * u + lane, rn - 1);
          v[q][u] = (double)M[(r0 + rr) + (int64_t)colc[q] * ld];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int rr = base + 64 * u + lane;
          if (rr < lim[q]) acc[q] += v[q][u] * xs[rr];
        }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = cblk + wave * 4 + q;
    const double v = wave_sum(acc[q]);
    if (lane == 0 && col < pp.n_r) yr[col] += (col < pp.n_i) ? v : (fr[col] - v);
  }
}

// ---------------------------------------------------------------------------
// The same products for many right-hand sides at once on the matrix cores
// (v_mfma_f64_16x16x4, FP64 accumulation; up to 32 columns, two 16-wide
// accumulators per wave), so that Q^T is read once per step for a whole
// batch of excitations instead of once per excitation.  A block owns 64
// output rows (interior unknowns for the recovery, kept unknowns for the
// condensation) and streams the 64 x 64 blocks of Q^T along the contracted
// index: each lane loads its matrix operands straight from Q^T's column-major
// storage into registers, one block ahead, and only the right-hand sides go
// through LDS (two buffers, one barrier per block).  Loads are issued
// unconditionally, from clamped addresses where they have nothing to read
// (the Q buffers carry 64 elements of slack at their end for the rows past a
// patch's last column), so the waits stay exact.
// ---------------------------------------------------------------------------

// Condensation of R right-hand sides (columns j of f and ygg at j * ldv):
// ygg[c] += (c < n_i) ? (Q^T[:, c] . f_i) : (f[c] - Q^T[:, c] . f_i).  One
// block per 64 columns of a listed patch (prefix over ceil(n_r / 64)).  The
// contraction runs over interior rows, in an order of its own (the k order
// of a product is free as long as both operands follow it): vector g of
// lane (li, lk) holds the rows 4 V g + V lk .. + V - 1 of the 64-row block
// in column li, so the 4 lanes of one column read 4 V consecutive entries
// per load instruction (64 contiguous bytes per column).
template <class T>
__global__ void __launch_bounds__(256) k_condense_w(const DevPatch* P, const int* plist,
                                                    const int* prefix, int nlist, const T* Q,
                                                    const double* f, double* ygg, int64_t ldv,
                                                    int R) {
  typedef Mfma16<double> M;
  typedef typename TileVec<T>::v VT;
  constexpr int V = TileVec<T>::n, NV = 16 / V;  // vectors per lane per block
  constexpr int XP = 65;                         // column stride of the staged f
  const int li_ = find_job(prefix, nlist, blockIdx.x);
  const DevPatch& pp = P[plist[li_]];
  const int c0 = (blockIdx.x - prefix[li_]) * 64;
  __shared__ double Fs[2][32 * XP];
  const T* Mq = Q + pp.Q_off;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int ie = t & 63, jq = t >> 6;
  // Q^T[:, c] for c < n_i has nonzeros only in rows <= c
  const int rmax = c0 < pp.n_i ? min(pp.n_i, c0 + 64) : pp.n_i;
  const int cl = min(c0 + 16 * w + li, pp.n_r - 1);  // this lane's column (clamped)
  M::acc a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
  VT ra[NV];
  double xg[8];
  auto fetch = [&](int r0) {
    const VT* src = reinterpret_cast<const VT*>(Mq + (int64_t)cl * pp.ni_pad + r0) + lk;
#pragma unroll
    for (int g = 0; g < NV; ++g) ra[g] = __builtin_nontemporal_load(src + 4 * g);
    const int r = min(r0 + ie, pp.n_r - 1);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int j = jq + 4 * m;
      xg[m] = f[(int64_t)(j < R ? j : 0) * ldv + pp.r_off + r];
    }
  };
  if (rmax > 0) fetch(0);
  for (int r0 = 0, it = 0; r0 < rmax; r0 += 64, ++it) {
    const int buf = it & 1;
    VT rc[NV];
#pragma unroll
    for (int g = 0; g < NV; ++g) rc[g] = ra[g];
#pragma unroll
    for (int m = 0; m < 8; ++m) Fs[buf][(jq + 4 * m) * XP + ie] = xg[m];
    __syncthreads();
    if (r0 + 64 < rmax) fetch(r0 + 64);
    const double* fs = Fs[buf] + li * XP + V * lk;
    const int rl = r0 + V * lk;  // row of this lane's first k-step
#pragma unroll
    for (int g = 0; g < NV; ++g)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int k = 4 * V * g + e;  // row offset of this k-step from rl
        // rows past n_i contract with zero (their storage may hold the next
        // column's entries)
        const double a = rl + k < pp.n_i ? (double)rc[g][e] : 0.0;
        a0 = M::mma(a, fs[k], a0);
        if (R > 16) a1 = M::mma(a, fs[16 * XP + k], a1);
      }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = c0 + 16 * w + M::row(lk, e);
    if (c >= pp.n_r) continue;
    for (int h = 0; h < 2; ++h) {
      const int j = 16 * h + li;
      if (j >= R) continue;
      const double v = h ? a1[e] : a0[e];
      const int64_t o = (int64_t)j * ldv + pp.r_off + c;
      ygg[o] += (c < pp.n_i) ? v : (f[o] - v);
    }
  }
}

// Interior recovery of R columns: out[r_off + r] = sum_c Q^T[r, c] z[r_off + c]
// for r < n_i (column j of z and out at j * ldv); Q^T's leading block is
// upper triangular, so column blocks before the row block are skipped.  One
// block per 64 interior rows of a listed patch (prefix over ceil(n_i / 64)).
// Lane (li, lk) loads Q^T[r0 + 16 w + li, c0 + 4 k + lk] for its 16 k-steps:
// per load, 16 consecutive rows of 4 columns.
template <class T>
__global__ void __launch_bounds__(256) k_qapply_w(const DevPatch* P, const int* plist,
                                                  const int* prefix, int nlist, const T* Q,
                                                  const double* z, double* out, int64_t ldv,
                                                  int R) {
  typedef Mfma16<double> M;
  constexpr int XP = 66;  // column stride of the staged z
  const int li_ = find_job(prefix, nlist, blockIdx.x);
  const DevPatch& pp = P[plist[li_]];
  const int r0 = (blockIdx.x - prefix[li_]) * 64;
  __shared__ double Zs[2][32 * XP];
  const T* Mq = Q + pp.Q_off + r0 + 16 * ((threadIdx.x >> 6)) + (threadIdx.x & 15);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int ie = t & 63, jq = t >> 6;
  (void)w;
  M::acc a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
  T ra[16];
  double xg[8];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = min(c0 + 4 * k + lk, pp.n_r - 1);
      ra[k] = __builtin_nontemporal_load(Mq + (int64_t)c * pp.ni_pad);
    }
    const int c = c0 + ie;
    const int cc = min(c, pp.n_r - 1);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int j = jq + 4 * m;
      const double v = z[(int64_t)(j < R ? j : 0) * ldv + pp.r_off + cc];
      // columns past n_r meet clamped (nonzero) matrix columns: zero inputs
      xg[m] = c < pp.n_r ? v : 0.0;
    }
  };
  const int cbeg = r0 / 64 * 64;
  if (cbeg < pp.n_r) fetch(cbeg);
  for (int c0 = cbeg, it = 0; c0 < pp.n_r; c0 += 64, ++it) {
    const int buf = it & 1;
    T rc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) rc[k] = ra[k];
#pragma unroll
    for (int m = 0; m < 8; ++m) Zs[buf][(jq + 4 * m) * XP + ie] = xg[m];
    __syncthreads();
    if (c0 + 64 < pp.n_r) fetch(c0 + 64);
    const double* zs = Zs[buf] + li * XP + lk;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double a = (double)rc[k];
      a0 = M::mma(a, zs[4 * k], a0);
      if (R > 16) a1 = M::mma(a, zs[16 * XP + 4 * k], a1);
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + 16 * (t >> 6) + M::row(lk, e);
    if (r >= pp.n_i) continue;
    for (int h = 0; h < 2; ++h) {
      const int j = 16 * h + li;
      if (j < R) out[(int64_t)j * ldv + pp.r_off + r] = h ? a1[e] : a0[e];
    }
  }
}

// ===========================================================================
// Small vector kernels
// ===========================================================================
__device__ inline double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) r += sh[w];
  }
  return r;  // valid in thread 0
}

// One block of 1024 threads per output: c[i] = sum_t rows[i ld + t] v[t] for
// i < nb (block i), and with a != nullptr one more block writes
// c[extra] = sum_t a[t] b[t].  Plain stores, no atomics.
__global__ void __launch_bounds__(1024) k_rowdot(int n, int nb, const double* rows, int64_t ld,
                                                 const double* v, double* c, const double* a,
                                                 const double* b, int extra) {
  __shared__ double sh[16];
  const int i = blockIdx.x;
  const double* x = i < nb ? rows + (int64_t)i * ld : a;
  const double* y = i < nb ? v : b;
  double acc = 0.0;
  for (int t = threadIdx.x; t < n; t += 1024) acc += x[t] * y[t];
  acc = wave_sum(acc);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += sh[w];
    c[i < nb ? i : extra] = s;
  }
}

// v[t] += sgn * sum_{i < nb} c[i] X[i ld + t]; with FX != nullptr also
// Fv[t] += sgn * sum_{i < nb} c[i] FX[i ld + t]
__global__ void __launch_bounds__(256) k_multiaxpy(int n, int nb, const double* c, double sgn,
                                                   const double* X, const double* FX, int64_t ld,
                                                   double* v, double* Fv) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nb; ++i) {
    const double ci = c[i];
    a += ci * X[(int64_t)i * ld + t];
    if (FX) b += ci * FX[(int64_t)i * ld + t];
  }
  v[t] += sgn * a;
  if (FX) Fv[t] += sgn * b;
}

// x = v / sqrt(nu2), fx = Fv / sqrt(nu2) when nu2 > tol * ref > 0, else zeros
// (a direction that adds nothing beyond the span is stored as zero)
__global__ void __launch_bounds__(256) k_store_dir(int n, const double* nu2, const double* ref,
                                                   double tol, const double* v, const double* Fv,
                                                   double* x, double* fx) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const double q = nu2[0], r = ref[0];
  const bool keep = r > 0.0 && q > tol * r;
  const double sc = keep ? 1.0 / sqrt(q) : 0.0;
  x[t] = v[t] * sc;
  fx[t] = Fv[t] * sc;
}

// v = a, w = b - c (copies of a ring slot, or F lambda = d - r)
__global__ void __launch_bounds__(256) k_copy_sub(int n, const double* a, const double* b,
                                                  const double* c, double* v, double* w) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  v[t] = a[t];
  w[t] = c ? b[t] - c[t] : b[t];
}

// y[i] = scale * (w[pp[i]] - w[pm[i]]); partial[block] = sum y[i] * dotw[i]
__global__ void __launch_bounds__(256) k_jump(int n, const int* pos_p, const int* pos_m,
                                              const double* w, double scale, double* y,
                                              const double* dotw, double* partial,
                                              const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    const double v = scale * (w[pos_p[i]] - w[pos_m[i]]);
    y[i] = v;
    if (dotw) d = v * dotw[i];
  }
  if (partial) {
    const double s = block_sum256(d, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

__device__ inline double sum_partials(const double* p, int n, double* sh) {
  // every block reduces the same partials in the same order (deterministic)
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
  __shared__ double s2[4];
  v = wave_sum(v);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) s2[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) r += s2[w];
    sh[0] = r;
  }
  __syncthreads();
  return sh[0];
}

// Sum of the TCF_QSLOTS quadratic-form slots (256-thread blocks), the same
// fixed order in every block.
__device__ inline double sum_slots(const double* slots, double* sh) {
  __shared__ double s4[4];
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < TCF_QSLOTS / 256; ++k) v += slots[k * 256 + threadIdx.x];
  v = block_sum256(v, s4);
  if (threadIdx.x == 0) sh[0] = v;
  __syncthreads();
  return sh[0];
}

// ---- tile-path PCG on R right-hand sides at once ---------------------------
// Vectors are column-major (column j of an n-vector at j * n); st[0 .. R)
// hold each column's scalars, st[R].done is set when every column is done.
// A converged column is frozen (its lambda and r no longer change).

// lambda = 0, r = d, partial[j * npart + block] = d_j.d_j
template <int R>
__global__ void __launch_bounds__(256) k_pcg_init_t(int n, const double* d, double* lam,
                                                    double* r, double* part_dd, int npart) {
  __shared__ double sh4[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double v = 0.0;
    if (i < n) {
      v = d[(int64_t)j * n + i];
      lam[(int64_t)j * n + i] = 0.0;
      r[(int64_t)j * n + i] = v;
    }
    const double s = block_sum256(v * v, sh4);
    if (threadIdx.x == 0) part_dd[j * npart + blockIdx.x] = s;
    __syncthreads();
  }
}

// Warm start: r0 = d - F lambda0, with F lambda0 = dt (w[pp] - w[pm]) from
// the accumulated w of one F apply on lambda0 (lambda is left as it is);
// partial[j * npart + block] = d_j.d_j (the stopping test stays relative to d).
template <int R>
__global__ void __launch_bounds__(256) k_pcg_init_w(int n, const int* pos_p, const int* pos_m,
                                                    const double* w, int wld, double dt,
                                                    const double* d, double* r, double* part_dd,
                                                    int npart) {
  __shared__ double sh4[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = 0, b = 0;
  if (i < n) {
    a = pos_p[i];
    b = pos_m[i];
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double v = 0.0;
    if (i < n) {
      v = d[(int64_t)j * n + i];
      r[(int64_t)j * n + i] = v - dt * (w[(int64_t)j * wld + a] - w[(int64_t)j * wld + b]);
    }
    const double s = block_sum256(v * v, sh4);
    if (threadIdx.x == 0) part_dd[j * npart + blockIdx.x] = s;
    __syncthreads();
  }
}

// z0 = wp tb[pp] - wm tb[pm] (tb = S_bb (D B)^T r0 from the preconditioner
// tiles; wp = wm = 1 unscaled, else the scaling weights of the two copies),
// p = z0; block 0: dd, r.z (the preconditioner's quadratic-form slots),
// iteration counts and flags.
template <int R>
__global__ void __launch_bounds__(256) k_pcg_init2_t(int n, const int* pos_p, const int* pos_m,
                                                     const double* tb, int tld,
                                                     const double* wp, const double* wm,
                                                     const double* rz_slots,
                                                     const double* part_dd, int npart,
                                                     PcgScalars* st, double* p) {
  __shared__ double sh[1];
  __shared__ double sh1[1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int a = pos_p[i], b = pos_m[i];
    const double ca = wp ? wp[i] : 1.0, cb = wm ? wm[i] : 1.0;
#pragma unroll
    for (int j = 0; j < R; ++j)
      p[(int64_t)j * n + i] = ca * tb[(int64_t)j * tld + a] - cb * tb[(int64_t)j * tld + b];
  }
  if (blockIdx.x == 0) {
    int all = 1;
    for (int j = 0; j < R; ++j) {
      const double dd = sum_partials(part_dd + j * npart, npart, sh1);
      const double rz = sum_slots(rz_slots + j * TCF_QSLOTS, sh);
      if (threadIdx.x == 0) {
        st[j].dd = dd;
        st[j].rz[0] = rz;
        st[j].rz[1] = 0.0;
        st[j].rr = dd;
        st[j].done = dd == 0.0 ? 1 : 0;
        st[j].iters = 0;
      }
      all &= dd == 0.0 ? 1 : 0;
      __syncthreads();
    }
    if (threadIdx.x == 0) st[R].done = all;
  }
}

// p.Fp from the F apply's quadratic-form slots (x^T S_bb^-1 x + cv^T S_Pi^-1
// cv, x = Bhat^T p); Fp = dt (w[pp] - w[pm]) formed on the fly from the
// accumulated w; alpha = rz[par] / p.Fp; lambda += alpha p; r -= alpha Fp;
// ||r||^2 partials.  Also clears zero[0 .. nzero) (the preconditioner
// accumulator and its slots).
template <int R>
__global__ void __launch_bounds__(256) k_pcg_update_t(int n, const int* pos_p, const int* pos_m,
                                                      const double* w, int wld, double dt,
                                                      const double* pq_slots, PcgScalars* st,
                                                      int par, double* lam, double* r,
                                                      const double* p, double* part_rr,
                                                      int npart, double* zero, int64_t nzero) {
  // no early exit on the all-done flag: that read would sit in front of every
  // other load; the per-column flags below already guard all updates
  __shared__ double sh[1];
  __shared__ double sh4[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = 0, b = 0;
  // up to 4 columns the vectors are loaded ahead (in flight during the slot
  // reductions); wider batches load each column in its turn
  constexpr int RC = R <= 4 ? R : 1;
  double pi[RC], ri[RC], li[RC];
  if (i < n) {
    a = pos_p[i];
    b = pos_m[i];
  }
  if (R <= 4) {
#pragma unroll
    for (int j = 0; j < RC; ++j) {
      pi[j] = i < n ? p[(int64_t)j * n + i] : 0.0;
      ri[j] = i < n ? r[(int64_t)j * n + i] : 0.0;
      li[j] = i < n ? lam[(int64_t)j * n + i] : 0.0;
    }
  }
  for (int64_t k = i; k < nzero; k += (int64_t)gridDim.x * blockDim.x) zero[k] = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int jc = R <= 4 ? j : 0;
    if (R > 4) {
      pi[0] = i < n ? p[(int64_t)j * n + i] : 0.0;
      ri[0] = i < n ? r[(int64_t)j * n + i] : 0.0;
      li[0] = i < n ? lam[(int64_t)j * n + i] : 0.0;
    }
    const double pq = sum_slots(pq_slots + j * TCF_QSLOTS, sh);
    const bool live = !st[j].done;
    double v = 0.0;
    if (i < n) {
      if (live) {
        const double alpha = st[j].rz[par] / pq;
        const double fi = dt * (w[(int64_t)j * wld + a] - w[(int64_t)j * wld + b]);
        lam[(int64_t)j * n + i] = li[jc] + alpha * pi[jc];
        ri[jc] -= alpha * fi;
        r[(int64_t)j * n + i] = ri[jc];
      }
      v = ri[jc] * ri[jc];
    }
    const double s = block_sum256(v, sh4);
    if (threadIdx.x == 0) part_rr[j * npart + blockIdx.x] = s;
    __syncthreads();
  }
}

// r.z from the preconditioner's quadratic-form slots, z = wp tb[pp] -
// wm tb[pm] on the fly (weights as in k_pcg_init2_t); beta = (r.z) / rz[par]; p = z + beta p.  Block 0 records
// rz[par ^ 1], sums the ||r||^2 partials and sets each column's iteration
// count and flag and the all-done flag (other blocks may then stop early: p
// is not used after convergence).  Also clears zero[0 .. nzero) (the F-apply
// accumulators and their slots).
template <int R>
__global__ void __launch_bounds__(256) k_pcg_pupdate_t(int n, const int* pos_p, const int* pos_m,
                                                       const double* tb, int tld,
                                                       const double* wp, const double* wm,
                                                       const double* rz_slots,
                                                       const double* part_rr, int npart,
                                                       PcgScalars* st, int par, double tol2,
                                                       double* p, double* zero, int64_t nzero) {
  // no early exit on the all-done flag (see k_pcg_update_t)
  __shared__ double sh[1];
  __shared__ double sh1[1];
  __shared__ double rzs[R];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = 0, b = 0;
  constexpr int RC = R <= 4 ? R : 1;
  double pi[RC], ca = 1.0, cb = 1.0;
  if (i < n) {
    a = pos_p[i];
    b = pos_m[i];
    if (wp) ca = wp[i];
    if (wm) cb = wm[i];
  }
  if (R <= 4) {
#pragma unroll
    for (int j = 0; j < RC; ++j) pi[j] = i < n ? p[(int64_t)j * n + i] : 0.0;
  }
  for (int64_t k = i; k < nzero; k += (int64_t)gridDim.x * blockDim.x) zero[k] = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int jc = R <= 4 ? j : 0;
    if (R > 4) pi[0] = i < n ? p[(int64_t)j * n + i] : 0.0;
    const double rz_new = sum_slots(rz_slots + j * TCF_QSLOTS, sh);
    if (threadIdx.x == 0) rzs[j] = rz_new;
    if (i < n && !st[j].done) {
      const double beta = rz_new / st[j].rz[par];
      p[(int64_t)j * n + i] =
          (ca * tb[(int64_t)j * tld + a] - cb * tb[(int64_t)j * tld + b]) + beta * pi[jc];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    int all = 1;  // meaningful in thread 0, which writes every flag itself
    for (int j = 0; j < R; ++j) {
      const double rr = sum_partials(part_rr + j * npart, npart, sh1);
      if (threadIdx.x == 0) {
        int dn = st[j].done;
        if (!dn) {
          st[j].rz[par ^ 1] = rzs[j];
          st[j].rr = rr;
          st[j].iters += 1;
          if (rr <= tol2 * st[j].dd) {
            st[j].done = 1;
            dn = 1;
          }
        }
        all &= dn;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) st[R].done = all;
  }
}


// out[k] = extra[k] + sa * sum srcA[ia[t]] + sb * sum srcB[ib[t]] over owners t of k
__global__ void __launch_bounds__(256) k_coarse_gather(int n, const int* ptr, const int* ia,
                                                       const double* srcA, double sa,
                                                       const int* ib, const double* srcB,
                                                       double sb, const double* extra,
                                                       double* out, const int* done) {
  if (done && *done) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double v = extra ? extra[k] : 0.0;
  for (int t = ptr[k]; t < ptr[k + 1]; ++t) {
    if (srcA) v += sa * srcA[ia[t]];
    if (srcB) v += sb * srcB[ib[t]];
  }
  out[k] = v;
}

// y = alpha * x + beta * y over n entries
__global__ void k_axpby(int64_t n, double alpha, const double* x, double beta, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = alpha * x[i] + (beta == 0.0 ? 0.0 : beta * y[i]);
}

// out[i] = a[ia[i]] - b[ib[i]] (index maps), used for t = u - v on b-vectors
__global__ void k_sub_gather(int n, const int* ia, const double* a, const int* ib,
                             const double* b, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[ia[i]] - b[ib[i]];
}

// out[dst ? dst[i] : i] = scale * src[sidx ? sidx[i] : i]
__global__ void k_scatter(int n, const int* dst, const int* sidx, const double* src, double scale,
                          double* out, const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[dst ? dst[i] : i] = scale * src[sidx ? sidx[i] : i];
}

// global field: out[gid[i]] = a[i] where gid[i] >= 0 (zero elsewhere beforehand)
__global__ void k_to_global(int64_t n, const int64_t* gid, const double* a, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && gid[i] >= 0) out[gid[i]] = a[i];
}

// ===========================================================================
// Host launch wrappers
// ===========================================================================
#define TCF_GRID(n, b) dim3((unsigned)(((n) + (b)-1) / (b)))

void launch_tables(const DevPatch* P, int np, const double* gx, const double* gw, double* tabs,
                   double* ptab, hipStream_t st) {
  hipLaunchKernelGGL(k_tables1d, dim3(3 * np), dim3(256), 0, st, P, gx, gw, tabs);
  hipLaunchKernelGGL(k_point_tables, dim3(3 * np), dim3(256), 0, st, P, gx, gw, ptab);
}

template <class T>
void launch_assemble(const DevPatch* P, const int* col_prefix, int np, int total_cols,
                     const int* r_loc, const double* tabs, double dt, T* A, hipStream_t st) {
  if (total_cols == 0) return;
  hipLaunchKernelGGL(k_assemble<T>, dim3(total_cols), dim3(256), 0, st, P, col_prefix, np, r_loc,
                     tabs, dt, A);
}

void launch_wapply(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                   int total_rows, int nrhs, const int* r_loc, const int* loc2r,
                   const double* tabs, double dt, int mass_only, const double* x, double* y,
                   int64_t ldv, hipStream_t st) {
  if (total_rows == 0 || nrhs <= 0) return;
  if (nrhs == 1)
    hipLaunchKernelGGL(k_wapply<1>, dim3((total_rows + 127) / 128, 1), dim3(128), 0, st, P,
                       plist, row_prefix, nlist, r_loc, loc2r, tabs, dt, mass_only, nrhs, x, y,
                       ldv);
  else
    hipLaunchKernelGGL(k_wapply<8>, dim3((total_rows + 127) / 128, (nrhs + 7) / 8), dim3(128), 0,
                       st, P, plist, row_prefix, nlist, r_loc, loc2r, tabs, dt, mass_only, nrhs,
                       x, y, ldv);
}


void launch_load_batch(const DevPatch* P, const LoadJob* jobs, const int* prefix, int njobs,
                       int total, int nrhs, const int* r_loc, const double* ptab, const double* F,
                       int vec, double* out, int64_t ldv, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_load_batch, dim3(total, nrhs), dim3(128), 0, st, P, jobs, prefix, njobs,
                     r_loc, ptab, F, vec, out, ldv);
}

template <class T>
void launch_potrf(const FactorJob* jobs, int njobs, int k, T* A, int* fail, hipStream_t st) {
  hipLaunchKernelGGL(k_potrf_panel<T>, dim3(njobs), dim3(256), 0, st, jobs, k, A, fail);
}
template <class T>
void launch_trsm_panel(const FactorJob* jobs, const int* prefix, int njobs, int total, int k, T* A,
                       hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_trsm_panel<T>, dim3(total), dim3(64), 0, st, jobs, prefix, njobs, k, A);
}
template <class T>
void launch_syrk(const FactorJob* jobs, const int* prefix, int njobs, int total, int k, int mode,
                 T* A, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_syrk_blk<T>, dim3(total), dim3(256), 0, st, jobs, prefix, njobs, k, mode, A);
}
int syrk_super_panel() { return TCF_SP; }
template <class T>
void launch_copy_sbb(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* S,
                     hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_copy_sbb<T>, dim3(total), dim3(256), 0, st, P, prefix, np, A, S);
}
template <class T>
void launch_fill_G(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* G,
                   hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_fill_G<T>, dim3(total), dim3(256), 0, st, P, prefix, np, A, G);
}
template <class T>
void launch_fill_Q(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* Q,
                   hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_fill_Q<T>, dim3(total), dim3(256), 0, st, P, prefix, np, A, Q);
}
template <class T>
void launch_coarse_add(const DevPatch* P, int s, int n_p, const int* p_rank, const T* A,
                       double* SPi, int ldc, hipStream_t st) {
  if (n_p == 0) return;
  hipLaunchKernelGGL(k_coarse_add<T>, TCF_GRID(n_p * n_p, 256), dim3(256), 0, st, P, s, p_rank, A,
                     SPi, ldc);
}
void launch_identity_pad(double* M, int ld, int n0, int n, hipStream_t st) {
  if (n <= n0) return;
  hipLaunchKernelGGL(k_set_identity_pad, TCF_GRID(n - n0, 256), dim3(256), 0, st, M, ld, n0, n);
}
template <class T>
void launch_trsm_dinv(const TrsmJob* jobs, const int* dprefix, int njobs, int total, const T* L,
                      T* D, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_trsm_dinv<T>, dim3(total), dim3(64), 0, st, jobs, dprefix, njobs, L, D);
}
int trsm_rl_panel() { return TCF_RL_PANEL; }
template <class T>
void launch_trsm_rl_diag(const TrsmJob* jobs, const int* cprefix, const int* dprefix, int njobs,
                         int total, int s, int fwd, const T* L, const T* D, T* B, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_trsm_rl_diag<T>, dim3(total), dim3(256), 0, st, jobs, cprefix, dprefix,
                     njobs, s, fwd, L, D, B);
}
template <class T>
void launch_trsm_rl_update(const TrsmJob* jobs, const int* tprefix, int njobs, int total, int s,
                           int fwd, const T* L, T* B, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_trsm_rl_update<T>, dim3(total), dim3(256), 0, st, jobs, tprefix, njobs, s,
                     fwd, L, B);
}
// Optional timing events for the next timed launch of this thread: attached
// to the dispatch packet itself (hipExtLaunchKernelGGL), so their interval
// is the kernel's own execution, without the queue latency that separate
// marker packets would add.
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}
bool launch_events_pending() { return t_ev_start != nullptr; }

#define TCF_TIMED_LAUNCH(kernel, grid, block, shm, st, ...)                               \
  do {                                                                                  \
    if (t_ev_start) {                                                                   \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, st, t_ev_start, t_ev_stop, 0u,     \
                            __VA_ARGS__);                                               \
      t_ev_start = t_ev_stop = nullptr;                                                 \
    } else {                                                                            \
      hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                    \
    }                                                                                   \
  } while (0)

template <class T>
void launch_dotcols(const DotJob* jobs, const int* prefix, int njobs, int total, int max_rows,
                    const T* M, int xmode, const double* xv, const int* gidx,
                    const signed char* gsgn, double xscale, double* out, const int* done,
                    hipStream_t st) {
  if (total == 0) return;
  (void)max_rows;
  TCF_TIMED_LAUNCH(k_dotcols<T>, dim3(total), dim3(256), 0, st, jobs, prefix, njobs, M, xmode, xv,
                     gidx, gsgn, xscale, out, done);
}
template <class T>
void launch_axpyrows(const AxpyJob* jobs, const int* prefix, int njobs, int total, int max_cols,
                     const T* M, const double* yv, const int* yidx, const double* base,
                     const int* base_off, double alpha, double* out, int tri_cols,
                     const int* done, hipStream_t st) {
  if (total == 0) return;
  (void)max_cols;
  TCF_TIMED_LAUNCH(k_axpyrows<T>, dim3(total), dim3(256), 0, st, jobs, prefix, njobs, M, yv, yidx,
                     base, base_off, alpha, out, tri_cols, done);
}
template <class T>
void launch_condense(const DevPatch* P, const int* plist, const int* prefix, int nlist, int total,
                     int nrhs, int max_ni, const T* Q, const double* f, double* ygg, int64_t ldv,
                     hipStream_t st) {
  if (total == 0) return;
  (void)max_ni;
  TCF_TIMED_LAUNCH(k_condense<T>, dim3(total, nrhs), dim3(256), 0, st, P, plist, prefix, nlist, Q,
                     f, ygg, ldv);
}

template <class T>
void launch_condense_w(const DevPatch* P, const int* plist, const int* prefix, int nlist,
                       int total, int R, const T* Q, const double* f, double* ygg, int64_t ldv,
                       hipStream_t st) {
  if (total == 0 || R == 0) return;
  TCF_TIMED_LAUNCH(k_condense_w<T>, dim3(total), dim3(256), 0, st, P, plist, prefix, nlist, Q, f,
                   ygg, ldv, R);
}
template <class T>
void launch_qapply_w(const DevPatch* P, const int* plist, const int* prefix, int nlist, int total,
                     int R, const T* Q, const double* z, double* out, int64_t ldv,
                     hipStream_t st) {
  if (total == 0 || R == 0) return;
  TCF_TIMED_LAUNCH(k_qapply_w<T>, dim3(total), dim3(256), 0, st, P, plist, prefix, nlist, Q, z,
                   out, ldv, R);
}
template void launch_condense_w<double>(const DevPatch*, const int*, const int*, int, int, int,
                                        const double*, const double*, double*, int64_t,
                                        hipStream_t);
template void launch_condense_w<float>(const DevPatch*, const int*, const int*, int, int, int,
                                       const float*, const double*, double*, int64_t,
                                       hipStream_t);
template void launch_qapply_w<double>(const DevPatch*, const int*, const int*, int, int, int,
                                      const double*, const double*, double*, int64_t,
                                      hipStream_t);
template void launch_qapply_w<float>(const DevPatch*, const int*, const int*, int, int, int,
                                     const float*, const double*, double*, int64_t, hipStream_t);

void launch_jump(int n, const int* pp, const int* pm, const double* w, double scale, double* y,
                 const double* dotw, double* partial, const int* done, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_jump, TCF_GRID(n, 256), dim3(256), 0, st, n, pp, pm, w, scale, y, dotw,
                     partial, done);
}
#define TCF_R_DISPATCH(R, KERNEL, GRID, ...)                                          \
  switch (R) {                                                                       \
    case 1: hipLaunchKernelGGL(KERNEL<1>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL(KERNEL<2>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    case 3: hipLaunchKernelGGL(KERNEL<3>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    case 16: hipLaunchKernelGGL(KERNEL<16>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<32>, GRID, dim3(256), 0, st, __VA_ARGS__); break; \
  }
void launch_pcg_init_t(int R, int n, const double* d, double* lam, double* r, double* part_dd,
                       int npart, hipStream_t st) {
  TCF_R_DISPATCH(R, k_pcg_init_t, TCF_GRID(max(n, 1), 256), n, d, lam, r, part_dd, npart);
}
void launch_pcg_init_w(int R, int n, const int* pp, const int* pm, const double* w, int wld,
                       double dt, const double* d, double* r, double* part_dd, int npart,
                       hipStream_t st) {
  TCF_R_DISPATCH(R, k_pcg_init_w, TCF_GRID(max(n, 1), 256), n, pp, pm, w, wld, dt, d, r, part_dd,
                 npart);
}
void launch_pcg_init2_t(int R, int n, const int* pp, const int* pm, const double* tb, int tld,
                        const double* wp, const double* wm, const double* rz_slots,
                        const double* part_dd, int npart, PcgScalars* stt, double* p,
                        hipStream_t st) {
  TCF_R_DISPATCH(R, k_pcg_init2_t, TCF_GRID(max(n, 1), 256), n, pp, pm, tb, tld, wp, wm,
                 rz_slots, part_dd, npart, stt, p);
}
void launch_pcg_update_t(int R, int n, const int* pp, const int* pm, const double* w, int wld,
                         double dt, const double* pq_slots, PcgScalars* stt, int par,
                         double* lam, double* r, const double* p, double* part_rr, int npart,
                         double* zero, int64_t nzero, hipStream_t st) {
  TCF_R_DISPATCH(R, k_pcg_update_t, TCF_GRID(max(n, 1), 256), n, pp, pm, w, wld, dt, pq_slots,
                 stt, par, lam, r, p, part_rr, npart, zero, nzero);
}
void launch_pcg_pupdate_t(int R, int n, const int* pp, const int* pm, const double* tb, int tld,
                          const double* wp, const double* wm, const double* rz_slots,
                          const double* part_rr, int npart, PcgScalars* stt, int par,
                          double tol2, double* p, double* zero, int64_t nzero, hipStream_t st) {
  TCF_R_DISPATCH(R, k_pcg_pupdate_t, TCF_GRID(max(n, 1), 256), n, pp, pm, tb, tld, wp, wm,
                 rz_slots, part_rr, npart, stt, par, tol2, p, zero, nzero);
}
void launch_coarse_gather(int n, const int* ptr, const int* ia, const double* srcA, double sa,
                          const int* ib, const double* srcB, double sb, const double* extra,
                          double* out, const int* done, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_coarse_gather, TCF_GRID(n, 256), dim3(256), 0, st, n, ptr, ia, srcA, sa, ib,
                     srcB, sb, extra, out, done);
}
void launch_rowdot(int n, int nb, const double* rows, int64_t ld, const double* v, double* c,
                   const double* a, const double* b, int extra, hipStream_t st) {
  const int nblk = nb + (a ? 1 : 0);
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_rowdot, dim3(nblk), dim3(1024), 0, st, n, nb, rows, ld, v, c, a, b, extra);
}
void launch_multiaxpy(int n, int nb, const double* c, double sgn, const double* X, const double* FX,
                      int64_t ld, double* v, double* Fv, hipStream_t st) {
  if (n == 0 || nb == 0) return;
  hipLaunchKernelGGL(k_multiaxpy, TCF_GRID(n, 256), dim3(256), 0, st, n, nb, c, sgn, X, FX, ld, v,
                     Fv);
}
void launch_store_dir(int n, const double* nu2, const double* ref, double tol, const double* v,
                      const double* Fv, double* x, double* fx, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_store_dir, TCF_GRID(n, 256), dim3(256), 0, st, n, nu2, ref, tol, v, Fv, x,
                     fx);
}
void launch_copy_sub(int n, const double* a, const double* b, const double* c, double* v,
                     double* w, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy_sub, TCF_GRID(n, 256), dim3(256), 0, st, n, a, b, c, v, w);
}
void launch_axpby(int64_t n, double alpha, const double* x, double beta, double* y,
                  hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_axpby, TCF_GRID(n, 256), dim3(256), 0, st, n, alpha, x, beta, y);
}
void launch_sub_gather(int n, const int* ia, const double* a, const int* ib, const double* b,
                       double* out, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_sub_gather, TCF_GRID(n, 256), dim3(256), 0, st, n, ia, a, ib, b, out);
}
void launch_scatter(int n, const int* dst, const int* sidx, const double* src, double scale,
                    double* out, const int* done, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scatter, TCF_GRID(n, 256), dim3(256), 0, st, n, dst, sidx, src, scale, out,
                     done);
}
void launch_to_global(int64_t n, const int64_t* gid, const double* a, double* out,
                      hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_global, TCF_GRID(n, 256), dim3(256), 0, st, n, gid, a, out);
}

#define TCF_INST(T)                                                                              \
  template void launch_assemble<T>(const DevPatch*, const int*, int, int, const int*,            \
                                   const double*, double, T*, hipStream_t);                      \
  template void launch_potrf<T>(const FactorJob*, int, int, T*, int*, hipStream_t);              \
  template void launch_trsm_panel<T>(const FactorJob*, const int*, int, int, int, T*,            \
                                     hipStream_t);                                               \
  template void launch_syrk<T>(const FactorJob*, const int*, int, int, int, int, T*,             \
                               hipStream_t);                                                     \
  template void launch_copy_sbb<T>(const DevPatch*, const int*, int, int, const T*, T*,          \
                                   hipStream_t);                                                 \
  template void launch_fill_G<T>(const DevPatch*, const int*, int, int, const T*, T*,            \
                                 hipStream_t);                                                   \
  template void launch_fill_Q<T>(const DevPatch*, const int*, int, int, const T*, T*,            \
                                 hipStream_t);                                                   \
  template void launch_coarse_add<T>(const DevPatch*, int, int, const int*, const T*, double*,   \
                                     int, hipStream_t);                                          \
  template void launch_trsm_dinv<T>(const TrsmJob*, const int*, int, int, const T*, T*,         \
                                    hipStream_t);                                                \
  template void launch_trsm_rl_diag<T>(const TrsmJob*, const int*, const int*, int, int, int,    \
                                       int, const T*, const T*, T*, hipStream_t);                \
  template void launch_trsm_rl_update<T>(const TrsmJob*, const int*, int, int, int, int,         \
                                         const T*, T*, hipStream_t);                             \
  template void launch_dotcols<T>(const DotJob*, const int*, int, int, int, const T*, int,       \
                                  const double*, const int*, const signed char*, double,         \
                                  double*, const int*, hipStream_t);                             \
  template void launch_axpyrows<T>(const AxpyJob*, const int*, int, int, int, const T*,          \
                                   const double*, const int*, const double*, const int*, double, \
                                   double*, int, const int*, hipStream_t);                       \
  template void launch_condense<T>(const DevPatch*, const int*, const int*, int, int, int, int,  \
                                   const T*, const double*, double*, int64_t, hipStream_t);

TCF_INST(double)
TCF_INST(float)

}  // namespace tcf

namespace tcf {
// zr[i] = is_int[i] ? y[i] : -a[i]  (right-hand side of the interior recovery)
__global__ void k_build_z(int64_t n, const signed char* is_int, const double* y, const double* a,
                          double* zr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) zr[i] = is_int[i] ? y[i] : -a[i];
}
void launch_build_z(int64_t n, const signed char* is_int, const double* y, const double* a,
                    double* zr, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_build_z, TCF_GRID(n, 256), dim3(256), 0, st, n, is_int, y, a, zr);
}
}  // namespace tcf

namespace tcf {
// Assembled squared norm: the global value of kept unknown k is the sum of
// its local copies x[idx[ptr[k] .. ptr[k+1]]]; partial[block] = sum of squares.
// first_copy != 0: the value is the first copy only (vectors whose copies
// agree, such as fields), otherwise the sum of copies (assembled residuals).
__global__ void __launch_bounds__(256) k_asm_norm2(int n, const int* ptr, const int* idx,
                                                   const double* x, int first_copy,
                                                   double* partial) {
  __shared__ double sh[4];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (k < n) {
    const int t1 = first_copy ? ptr[k] + 1 : ptr[k + 1];
    for (int t = ptr[k]; t < t1; ++t) v += x[idx[t]];
    v = v * v;
  }
  const double s = block_sum256(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_sum_partials(const double* partial, int npart,
                                                      double* out) {
  __shared__ double sh[1];
  const double s = sum_partials(partial, npart, sh);
  if (threadIdx.x == 0) *out = s;
}
void launch_asm_norm2(int n, const int* ptr, const int* idx, const double* x, int first_copy,
                      double* partial, double* out, hipStream_t st) {
  const int nb = (n + 255) / 256;
  if (n == 0) return;
  hipLaunchKernelGGL(k_asm_norm2, dim3(nb), dim3(256), 0, st, n, ptr, idx, x, first_copy, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, nb, out);
}
}  // namespace tcf

namespace tcf {
__global__ void k_to_float(int64_t n, const double* a, float* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_float, TCF_GRID(n, 256), dim3(256), 0, st, n, a, b);
}
}  // namespace tcf

namespace tcf {
// Residual r = f - W x on the kept unknowns of every listed patch, with the
// row sums accumulated in double-double (exact products by FMA, error-free
// additions), so that the rounding of a sum with heavy cancellation does not
// leak into the near-kernel of the gauged operator.
__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__global__ void k_residual(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                           const int* r_loc, const int* loc2r, const double* tabs, double dt,
                           const double* f, const double* x, double* r) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= row_prefix[nlist]) return;
  const int li = find_job(row_prefix, nlist, gi);
  const DevPatch& pp = P[plist[li]];
  const int j = gi - row_prefix[li];
  const Tab1 X = make_tab(pp, tabs, 0), Y = make_tab(pp, tabs, 1), Z = make_tab(pp, tabs, 2);
  const EdgeCode u = decode_local(pp, r_loc[pp.r_off + j]);
  const double* xs = x + pp.r_off;
  const int* l2r = loc2r + pp.loc_off;
  double hi = 0.0, lo = 0.0;
  const int px = pp.deg[0], py = pp.deg[1], pz = pp.deg[2];
  const double nudt = pp.nu * dt;
  for (int dir = 0; dir < 3; ++dir) {
    const int na = pp.m[0] - (dir == 0), nb = pp.m[1] - (dir == 1), nc = pp.m[2] - (dir == 2);
    const int a0 = max(0, u.a - px), a1 = min(na - 1, u.a + px);
    const int b0 = max(0, u.b - py), b1 = min(nb - 1, u.b + py);
    const int c0 = max(0, u.c - pz), c1 = min(nc - 1, u.c + pz);
    for (int c = c0; c <= c1; ++c)
      for (int b = b0; b <= b1; ++b)
        for (int a = a0; a <= a1; ++a) {
          const int r2 = l2r[encode_local(pp, dir, a, b, c)];
          if (r2 < 0) continue;
          double M, K;
          mk_entry(X, Y, Z, u, EdgeCode{dir, a, b, c}, M, K);
          const double w = pp.sigma * M + nudt * K;
          const double p = w * xs[r2];
          const double pe = fma(w, xs[r2], -p);
          double s, e;
          two_sum(hi, p, s, e);
          hi = s;
          lo += e + pe;
        }
  }
  // r = f - (hi + lo)
  double s, e;
  two_sum(f[pp.r_off + j], -hi, s, e);
  r[pp.r_off + j] = s + (e - lo);
}
void launch_residual(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                     int total_rows, const int* r_loc, const int* loc2r, const double* tabs,
                     double dt, const double* f, const double* x, double* r, hipStream_t st) {
  if (total_rows == 0) return;
  hipLaunchKernelGGL(k_residual, dim3((total_rows + 127) / 128), dim3(128), 0, st, P, plist,
                     row_prefix, nlist, r_loc, loc2r, tabs, dt, f, x, r);
}
}  // namespace tcf

namespace tcf {
// y[i] += scale * (a[pp[i]] - a[pm[i]])  (jump of a kept-ordered vector)
__global__ void k_jump_add(int n, const int* pos_p, const int* pos_m, const double* a, double scale,
                           double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += scale * (a[pos_p[i]] - a[pos_m[i]]);
}
void launch_jump_add(int n, const int* pp, const int* pm, const double* a, double scale, double* y,
                     hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_jump_add, TCF_GRID(n, 256), dim3(256), 0, st, n, pp, pm, a, scale, y);
}
}  // namespace tcf

namespace tcf {
// Replace every local copy of kept unknown k by (sum of its copies) / count,
// i.e. assemble a residual and split it evenly over the patches sharing k.
__global__ void k_assemble_split(int n, const int* ptr, const int* idx, double* x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int t0 = ptr[k], t1 = ptr[k + 1];
  if (t1 - t0 < 2) return;
  double v = 0.0;
  for (int t = t0; t < t1; ++t) v += x[idx[t]];
  v /= (double)(t1 - t0);
  for (int t = t0; t < t1; ++t) x[idx[t]] = v;
}
void launch_assemble_split(int n, const int* ptr, const int* idx, double* x, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_assemble_split, TCF_GRID(n, 256), dim3(256), 0, st, n, ptr, idx, x);
}
}  // namespace tcf

namespace tcf {
// ===========================================================================
// Tile storage and tile GEMV
// ===========================================================================
template <class TS, class TD>
__global__ void k_pack_tiles(const PackJob* jobs, const TS* src, TD* dst) {
  const PackJob jb = jobs[blockIdx.x];
  TD* o = dst + jb.dst_off;
  const TS* s = src + jb.src_off;
  const int ncs = jb.trans ? jb.nr : jb.nc;  // stored columns
  const int nrs = jb.trans ? jb.nc : jb.nr;  // filled rows
  for (int idx = threadIdx.x; idx < 64 * ncs; idx += blockDim.x) {
    const int r = idx % 64, c = idx / 64;
    TD v = TD(0);
    if (r < nrs) {
      const int br = jb.trans ? c : r, bc = jb.trans ? r : c;
      v = (TD)s[(int64_t)(jb.row0 + br) + (int64_t)(jb.col0 + bc) * jb.ld];
    }
    o[idx] = v;
  }
}

// One tile of a row panel in the matrix cores' operand order (read by
// k_panel_w): the 64 x nc tile (the block at (row0, col0), or its transpose
// when trans) is stored as 4 wave blocks of 16 rows; in wave block w,
// vector g of lane l holds, for e < V = 16 / sizeof(TD), the entry
// (16 w + l % 16, 4 (V g + e) + l / 16).  Columns are padded with zeros to a
// multiple of 4 V: the tile takes 64 * roundup(nc, 4 V) elements.
template <class TS, class TD>
__global__ void k_pack_panel(const PackJob* jobs, const TS* src, TD* dst) {
  constexpr int V = 16 / sizeof(TD), Q = 4 * V;
  const PackJob jb = jobs[blockIdx.x];
  TD* o = dst + jb.dst_off;
  const TS* s = src + jb.src_off;
  const int ncs = jb.trans ? jb.nr : jb.nc;  // stored columns
  const int nrs = jb.trans ? jb.nc : jb.nr;  // filled rows
  const int ncq = (ncs + Q - 1) / Q;
  const int wblk = 16 * Q * ncq;             // elements of one wave block
  for (int idx = threadIdx.x; idx < 4 * wblk; idx += blockDim.x) {
    const int w = idx / wblk, r1 = idx % wblk;
    const int g = r1 / (64 * V), r2 = r1 % (64 * V);
    const int l = r2 / V, e = r2 % V;
    const int r = 16 * w + (l & 15), c = 4 * (V * g + e) + (l >> 4);
    TD v = TD(0);
    if (r < nrs && c < ncs) {
      const int br = jb.trans ? c : r, bc = jb.trans ? r : c;
      v = (TD)s[(int64_t)(jb.row0 + br) + (int64_t)(jb.col0 + bc) * jb.ld];
    }
    o[idx] = v;
  }
}

// Lane exchanges inside a wave without the LDS crossbar: DPP moves of the two
// 32-bit halves of a double.  CTRL is a DPP control word: quad_perm 0xB1 (lane
// i takes lane i^1 of its quad), 0x4E (i^2), row_ror 0x120 + n (rotate by n
// within each row of 16 lanes).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}
// sum over the 4 lanes of a quad, in every lane of it
__device__ inline double quad_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  return v;
}
// v plus the value of lane ^ 32 (resp. ^ 16), in every lane, through the
// permlane swaps: swapping a register with itself leaves (own, partner) in
// one half of the wave and (partner, own) in the other, so the two results
// add up to the pair sum everywhere (the same value: addition commutes)
__device__ inline double xor32_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ inline double xor16_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
// sum over the 64 lanes of a wave, in every lane: rotations within rows of
// 16 lanes, then the two exchanges across rows
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_f64<0x128>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x122>(v);
  v += dpp_f64<0x121>(v);
  v = xor16_sum(v);
  return xor32_sum(v);
}

// One block (256 threads) per tile (nc <= 64 columns of 64 rows, zero-padded).
// Loads are coalesced: load k of thread t reads the 16-byte chunk k*256 + t,
// i.e. V = 16/sizeof(T) consecutive rows (V*(t % RPC) ..) of column
// k*(256/RPC) + t/RPC, RPC = 64/V chunks per column, so each wave reads
// 1 KiB contiguous per instruction.  N part (row sums): each thread sums its
// columns, then threads with equal t % RPC are combined by lane shuffles and
// one LDS row per wave.  T part (column sums): per-thread partials over its
// V rows go through LDS and are summed by 4 threads per column.  Results are
// added to y with FP64 atomics (a tile of a symmetric operator serves A_IJ
// and A_IJ^T).

// Group (the operator) fixes the input mode: 0 (F apply) and 2 (Dirichlet
// preconditioner) take the signed gather scale * gsw[i] * xv[gidx[i]] (gsw:
// the +-1 entries of Bhat, or for a scaled preconditioner those of D Bhat),
// 1 (Phi_b N q) and 4 (the coarse factor's sweeps; a separate instance so
// that profiles tell the two apart) the plain gather xv[gidx[i]], 3 (the
// coarse top block) reads xv[i].
template <class T, int Group, int R>
__global__ void __launch_bounds__(256) k_tiles(const TileJob* jobs, const T* Mb,
                                               const double* xv, int xld, const int* gidx,
                                               const double* gsw, double scale,
                                               double* y, int yld, const int* ymap,
                                               double* qslot, const int* done) {
  constexpr int XM = Group == 3 ? 0 : ((Group == 1 || Group == 4) ? 2 : 1);
  // Blocks are dealt to the 8 XCDs round-robin (block b on XCD b % 8); give
  // each XCD a contiguous run of jobs, so that the tiles of a patch, which
  // share inputs and outputs, stay within one L2.
  const int nb = gridDim.x, per = nb >> 3, rem = nb & 7;
  const int xcd = blockIdx.x & 7, kk = blockIdx.x >> 3;
  const int job = xcd < rem ? xcd * (per + 1) + kk : rem * (per + 1) + (xcd - rem) * per + kk;
  typedef typename TileVec<T>::v VT;
  constexpr int V = TileVec<T>::n;   // rows per chunk
  constexpr int RPC = 64 / V;        // chunks per column
  constexpr int L = 64 * 64 / V / 256;  // loads per thread
  constexpr int CPL = 256 / RPC;     // columns advanced per load
  // column-sum partials per column and RHS: with several RHS, FP64 tiles
  // first combine lane pairs so the LDS array stays 16 wide
  constexpr int PRE = (R > 1 && RPC > 16) ? RPC / 16 : 1;
  constexpr int TPW = RPC / PRE;
  const TileJob jb = jobs[job];
  // the test reads a job field (never negative) so that the descriptor load
  // is issued together with the flag read instead of after it
  if ((done ? *done : 0) | (jb.nc < 0) | (jb.m_off < 0)) return;
  // inputs of RHS j: xs[j][0, 64) row side, xs[j][64, 128) column side
  __shared__ double xs[R][256];
  __shared__ double Tp[R][64][TPW + 1];
  __shared__ double Np[R][4][64];
  const int t = threadIdx.x;
  // the quadratic form is accumulated only when the caller passes its slots
  // (the one-column coarse solves of the per-step setup pass none)
  const bool doN = jb.flags & 1, doT = jb.flags & 2, qf = (jb.flags & 16) && qslot != nullptr;
  const VT* base = reinterpret_cast<const VT*>(Mb + jb.m_off);
  // inputs, step 1: gather indices (threads 0..63 the row side, 64..127 the
  // column side).  Issued before the matrix loads: memory counters retire in
  // order, so an index load issued after them would wait for the whole tile.
  const bool side_r = t < 64;
  const int tt = side_r ? t : t - 64;
  const bool xon = t < 128 && (side_r ? ((doT || qf) && tt < jb.nr) : (doN && tt < jb.nc));
  // lanes without an input read entry 0 (which every table has): no branch
  // around the loads, whose results are only used after the matrix loads
  const int xo = xon ? (side_r ? jb.xr_off : jb.xc_off) + tt : 0;
  int gi = xo;
  double sw = 1.0;
  if (XM != 0) gi = gidx[xo];
  if (XM == 1) sw = gsw[xo];
  // keep the index loads ahead of the matrix loads (straight-line code, so
  // this pins the order the scheduler emits)
  __builtin_amdgcn_sched_barrier(0);
  VT raw[L];
  const int h = t / RPC, lr = t % RPC;
  // only the nc stored columns exist: a lane past them reads its row chunk
  // of column 0 instead (no branch around the loads, which would serialise
  // them).  That value needs no masking: the column's input is zero, so it
  // adds nothing to the row sums, and its column sum is never written.
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const bool ok = k * CPL + h < jb.nc;
    raw[k] = __builtin_nontemporal_load(base + (ok ? k * 256 + t : lr));
  }
  __builtin_amdgcn_sched_barrier(0);
  // inputs, step 2: values, all 256 lanes (no branch): slot t of xs[j]
  {
    const double f = XM == 1 ? scale * sw : 1.0;
    // indices are non-negative: an unsigned index needs no sign extension,
    // which the compiler would otherwise hoist right behind the index load
    const unsigned gu = (unsigned)gi;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const double xg = xv[(size_t)j * (unsigned)xld + gu];
      xs[j][t] = xon ? f * xg : 0.0;
    }
  }
  __syncthreads();
  const int r0 = V * lr;
  double xrv[R][V], n[R][V];
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      xrv[j][v] = xs[j][r0 + v];
      n[j][v] = 0.0;
    }
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int cc = k * CPL + h;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const double xcv = xs[j][64 + cc];
      double tp = 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double a = (double)raw[k][v];
        n[j][v] += a * xcv;
        tp += a * xrv[j][v];
      }
      if (PRE == 2) tp += dpp_f64<0xB1>(tp);
      if (lr % PRE == 0) Tp[j][cc][lr / PRE] = tp;
    }
  }
  // rows r0.. are shared by the lanes of a wave with equal t % RPC
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (RPC == 16) n[j][v] = xor16_sum(n[j][v]);
      n[j][v] = xor32_sum(n[j][v]);
    }
  const int w = t >> 6;
  if ((t & 63) < RPC) {
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int v = 0; v < V; ++v) Np[j][w][r0 + v] = n[j][v];
  }
  __syncthreads();
  if (doT) {
    const int cc = t >> 2, q = t & 3;
    const int yi = (cc < jb.nc) ? ((jb.flags & 4) ? ymap[jb.yc_off + cc] : jb.yc_off + cc) : 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < TPW / 4; ++k) sum += Tp[j][cc][q * (TPW / 4) + k];
      sum = quad_sum(sum);
      if (q == 0 && cc < jb.nc) atomicAdd(y + (int64_t)j * yld + yi, sum);
    }
  }
  if (doN && t < 64) {  // wave 0
    const int yi = (t < jb.nr) ? ((jb.flags & 8) ? ymap[jb.yr_off + t] : jb.yr_off + t) : 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const double sum = (Np[j][0][t] + Np[j][1][t]) + (Np[j][2][t] + Np[j][3][t]);
      if (t < jb.nr) atomicAdd(y + (int64_t)j * yld + yi, sum);
      if (qf) {  // this tile's share of x^T A x (rows past nr carry zeros)
        const double v = wave_sum_dpp(xs[j][t] * sum);
        if (t == 0)
          atomicAdd(qslot + j * TCF_QSLOTS + (blockIdx.x & (TCF_QSLOTS - 1)),
                    (jb.flags & 32) ? 2.0 * v : v);
      }
    }
  }
}

// Row panels on the matrix cores, for batches of up to 32 right-hand sides.
// One block per panel job: wave w owns rows 16w .. 16w + 15 of the panel for
// all R columns (one 16-wide v_mfma_f64_16x16x4 accumulator, two when W32:
// R > 16; FP64 accumulation, FP32 tiles widened as they are used), and the job's
// tiles stream by one after the other, so each output row is formed in one
// block: added once to what the vector holds, with atomics only where another
// job shares the row (a split panel, or an operator whose rows several
// panels add into).  The symmetric operators are stored whole for this path.
//
// Tiles are stored in the matrix cores' operand order (see k_pack_panel):
// the 16 rows of wave w come as consecutive 16-byte vectors, lane l holding
// the entries (16w + l % 16, 4k + l / 16) of V = 16 / sizeof(T) consecutive
// k-steps k, so a wave's loads are contiguous and need no LDS.  They go to
// registers one tile ahead: the next tile is in flight while the matrix
// cores work on the current one.  The column inputs of a tile (64 entries x R)
// are staged in LDS, column-major with a column stride of 66 doubles, which
// keeps both the staging stores (lanes along entries) and the operand reads
// of a half-wave (16 columns x 2 entries) on distinct banks, and lets every
// operand read use one base address plus a constant offset; two buffers,
// one barrier per tile.  Inputs: groups 0 to 3 read
// xv[j * xld + i] directly, group 4 (the coarse factor's sweeps) through
// gidx.
template <class T, int Group, bool W32>
__global__ void __launch_bounds__(256) k_panel_w(const PanelJob* jobs, const PanelTile* tiles,
                                                 const T* Mb, const double* xv, int xld,
                                                 const int* gidx, double* y, int yld,
                                                 const int* ymap, double* qslot, const int* done,
                                                 int R, double* stage, int sld, double* qjob) {
  typedef Mfma16<double> M;
  constexpr int XM = Group == 4 ? 2 : 0;
  typedef typename TileVec<T>::v VT;
  constexpr int V = TileVec<T>::n;  // k-steps per 16-byte vector
  constexpr int Q = 4 * V;          // column quantum of the stored tiles
  constexpr int GM = 64 / Q;        // vectors per lane of a full tile
  // block b takes job b: the hardware deals consecutive blocks to the 8 XCDs
  // in turn, which spreads each XCD's streams over the whole buffer (a
  // contiguous run of jobs per XCD streamed measurably slower)
  const int nbk = gridDim.x, job = blockIdx.x;
  const PanelJob jb = jobs[job];
  if ((done ? *done : 0) | (jb.nt <= 0) | (jb.m_off < 0)) return;
  constexpr int XP = 66;  // column stride of the staged inputs
  __shared__ double Xs[2][32 * XP];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  // input staging: thread t serves entry t & 63, columns (t >> 6) + 4 m
  const int ie = t & 63, jq = t >> 6;
  M::acc a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
  VT ra[GM];
  double xg[8];
  const PanelTile* tp = tiles + jb.t0;
  auto fetch = [&](const PanelTile& tl, int64_t off) {
    // the index load goes first: the input loads wait for it, and the
    // tile's loads issued after it stay in flight meanwhile
    const bool xon = ie < tl.nc;
    const int xo = tl.xc_off + (xon ? ie : 0);
    const int gi = XM != 0 ? gidx[xo] : xo;
    const int ncq = (tl.nc + Q - 1) / Q;  // vectors per lane
    // wave block w: 16 rows x Q ncq columns = 64 ncq vectors.  Addresses are
    // a block-uniform base plus 32-bit byte offsets (one register each).
    const char* base = reinterpret_cast<const char*>(Mb + off);
    const unsigned lo = (unsigned)(w * 64 * ncq + lane) * 16u;
    // every load is issued, from a clamped address where it has nothing to
    // read, so that the number in flight is fixed and the waits are exact.
    // An input past the tile's columns meets zero columns of the stored tile
    // and one past the batch feeds an output column that is dropped, so
    // both may hold any finite value: they are not masked
#pragma unroll
    for (int g = 0; g < GM; ++g)
      ra[g] = __builtin_nontemporal_load(
          reinterpret_cast<const VT*>(base + lo + (unsigned)(g < ncq ? g : 0) * 1024u));
    const char* xb = reinterpret_cast<const char*>(xv);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int j = jq + 4 * m;
      xg[m] = *reinterpret_cast<const double*>(
          xb + ((unsigned)(j < R ? j : 0) * (unsigned)xld + (unsigned)gi) * 8u);
    }
  };
  // Operands of the epilogue: the output rows' current values (rows no other
  // job adds into) and the quadratic form's inputs.  They are loaded during
  // the job's last tile, in place of a next tile, so that their latency
  // hides behind that tile's products instead of following them.
  const bool shared = jb.flags & 1, mapped = jb.flags & 2, staged = jb.flags & 8;
  const bool qf = (jb.flags & 4) && (qslot || qjob);
  int yix[4];
  double yv[4][2], xq[4][2];
  auto load_epilogue = [&] {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * w + M::row(lk, e);
      const bool ok = row < jb.nr;
      const int yi = (mapped && !staged) ? (ok ? ymap[jb.yr_off + row] : 0) : jb.yr_off + row;
      yix[e] = yi;
      int gr = jb.xr_off + row;
      if (qf && XM != 0 && ok) gr = gidx[gr];
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int j = 16 * hh + li;
        const bool okj = ok && j < R;
        yv[e][hh] = (okj && !staged && !shared) ? y[(int64_t)j * yld + yi] : 0.0;
        xq[e][hh] = (okj && qf) ? xv[(size_t)j * (unsigned)xld + (unsigned)gr] : 0.0;
      }
    }
  };
  PanelTile tl = tp[0];
  int64_t off = jb.m_off;
  fetch(tl, off);
  // one tile: its inputs staged, the next tile (or, for the last one, the
  // epilogue's operands) requested, then its products
  auto step = [&](int it, auto last) {
    const int buf = it & 1;
    const int ncq = (tl.nc + Q - 1) / Q;
    VT rc[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) rc[g] = ra[g];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int j = jq + 4 * m;
      Xs[buf][j * XP + ie] = xg[m];
    }
    // the tile's inputs are staged; every wave is past the reads of this
    // buffer two tiles ago
    __syncthreads();
    if constexpr (decltype(last)::value) {
      load_epilogue();
    } else {
      off += 64 * (int64_t)(ncq * Q);
      tl = tp[it + 1];
      fetch(tl, off);
    }
    const double* xs = Xs[buf] + li * XP + lk;
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      if (g < ncq) {
        // the group's operand reads first, then its products
        double b0[V], b1[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          b0[e] = xs[4 * (V * g + e)];
          if (W32) b1[e] = xs[16 * XP + 4 * (V * g + e)];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const double a = (double)rc[g][e];
          a0 = M::mma(a, b0[e], a0);
          if (W32) a1 = M::mma(a, b1[e], a1);
        }
      }
    }
  };
  for (int it = 0; it + 1 < jb.nt; ++it) step(it, std::false_type());
  step(jb.nt - 1, std::true_type());
  // outputs: lane (li, lk), element e is row 16 w + row(lk, e), column li (+16).
  // A staged job (flag 8) stores its rows into its own rows of the staging
  // block, summed into their targets afterwards in a fixed order; with qjob
  // the quadratic form of each job goes to its own entry (summed likewise).
  double q0 = 0.0, q1 = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = 16 * w + M::row(lk, e);
    if (row >= jb.nr) continue;
    const int yi = yix[e];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int j = 16 * hh + li;
      if (j >= R) continue;
      const double v = hh ? a1[e] : a0[e];
      if (staged) {
        stage[(int64_t)j * sld + yi] = v;
      } else {
        double* dst = y + (int64_t)j * yld + yi;
        if (shared) atomicAdd(dst, v);
        else *dst = yv[e][hh] + v;
      }
      if (qf) {
        if (hh) q1 += xq[e][hh] * v; else q0 += xq[e][hh] * v;
      }
    }
  }
  if (qf) {
    q0 = xor32_sum(xor16_sum(q0));
    q1 = xor32_sum(xor16_sum(q1));
    __syncthreads();  // every wave is done with the staged inputs
    double* Qs = Xs[0];  // 4 x 32
    if (lk == 0) {
      Qs[w * 32 + li] = q0;
      Qs[w * 32 + 16 + li] = q1;
    }
    __syncthreads();
    if (t < 32 && t < R) {
      const double qv = (Qs[t] + Qs[32 + t]) + (Qs[64 + t] + Qs[96 + t]);
      if (qjob) qjob[(int64_t)t * nbk + job] = qv;
      else atomicAdd(qslot + t * TCF_QSLOTS + (blockIdx.x & (TCF_QSLOTS - 1)), qv);
    }
  } else if (qjob && t < 32 && t < R) {
    qjob[(int64_t)t * nbk + job] = 0.0;
  }
}

// Fixed-order sums of staged rows: y[j * yld + tgt[i]] += sum over
// p in [ptr[i], ptr[i+1]) of stage[j * sld + idx[p]], for R columns (the
// entries of each target in the order the plan lists them).
__global__ void k_stage_add(int n, const int* tgt, const int* ptr, const int* idx,
                            const double* stage, int sld, int R, double* y, int yld,
                            const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = ptr[i], p1 = ptr[i + 1], t = tgt[i];
  for (int j = 0; j < R; ++j) {
    double v = 0.0;
    for (int p = p0; p < p1; ++p) v += stage[(int64_t)j * sld + idx[p]];
    y[(int64_t)j * yld + t] += v;
  }
}

// slots[j * TCF_QSLOTS] += the sum of the njobs per-job quadratic forms of
// column j (one block per column, a fixed summation order).
__global__ void __launch_bounds__(256) k_qjob_add(int njobs, const double* qjob, double* slots,
                                                  const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < njobs; k += 256) v += qjob[(int64_t)j * njobs + k];
  v = block_sum256(v, sh);
  if (threadIdx.x == 0) slots[(int64_t)j * TCF_QSLOTS] += v;
}

__global__ void k_zero(int64_t n, double* a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

template <class TS, class TD>
void launch_pack_tiles(const PackJob* jobs, int njobs, const TS* src, TD* dst, hipStream_t st) {
  if (njobs == 0) return;
  hipLaunchKernelGGL((k_pack_tiles<TS, TD>), dim3(njobs), dim3(256), 0, st, jobs, src, dst);
}
template <class TS, class TD>
void launch_pack_panel(const PackJob* jobs, int njobs, const TS* src, TD* dst, hipStream_t st) {
  if (njobs == 0) return;
  hipLaunchKernelGGL((k_pack_panel<TS, TD>), dim3(njobs), dim3(256), 0, st, jobs, src, dst);
}
template void launch_pack_panel<double, double>(const PackJob*, int, const double*, double*,
                                                hipStream_t);
template void launch_pack_panel<float, float>(const PackJob*, int, const float*, float*,
                                              hipStream_t);
// group only names the kernel instance (apply / phi / precond / coarse) so
// that traces attribute each operator separately
template <class T, int G>
static void launch_tiles_g(int R, const TileJob* jobs, int njobs, const T* M, const double* xv,
                           int xld, const int* gidx, const double* gsgn, double scale,
                           double* y, int yld, const int* ymap, double* qslot, const int* done,
                           hipStream_t st) {
  switch (R) {
    case 1:
      TCF_TIMED_LAUNCH((k_tiles<T, G, 1>), dim3(njobs), dim3(256), 0, st, jobs, M, xv, xld, gidx,
                       gsgn, scale, y, yld, ymap, qslot, done);
      break;
    case 2:
      TCF_TIMED_LAUNCH((k_tiles<T, G, 2>), dim3(njobs), dim3(256), 0, st, jobs, M, xv, xld, gidx,
                       gsgn, scale, y, yld, ymap, qslot, done);
      break;
    case 3:
      TCF_TIMED_LAUNCH((k_tiles<T, G, 3>), dim3(njobs), dim3(256), 0, st, jobs, M, xv, xld, gidx,
                       gsgn, scale, y, yld, ymap, qslot, done);
      break;
    default:
      TCF_TIMED_LAUNCH((k_tiles<T, G, 4>), dim3(njobs), dim3(256), 0, st, jobs, M, xv, xld, gidx,
                       gsgn, scale, y, yld, ymap, qslot, done);
      break;
  }
}

template <class T>
void launch_panels(int group, int R, const PanelJob* jobs, const PanelTile* tiles, int njobs,
                   const T* M, const double* xv, int xld, const int* gidx, double* y, int yld,
                   const int* ymap, double* qslot, const int* done, hipStream_t st,
                   double* stage, int sld, double* qjob) {
  if (njobs == 0) return;
#define TCF_PANEL_CASE(G)                                                                     \
  case G:                                                                                     \
    if (R > 16)                                                                               \
      TCF_TIMED_LAUNCH((k_panel_w<T, G, true>), dim3(njobs), dim3(256), 0, st, jobs, tiles, M, \
                       xv, xld, gidx, y, yld, ymap, qslot, done, R, stage, sld, qjob);        \
    else                                                                                      \
      TCF_TIMED_LAUNCH((k_panel_w<T, G, false>), dim3(njobs), dim3(256), 0, st, jobs, tiles,  \
                       M, xv, xld, gidx, y, yld, ymap, qslot, done, R, stage, sld, qjob);     \
    break;
  switch (group) {
    TCF_PANEL_CASE(0)
    TCF_PANEL_CASE(1)
    TCF_PANEL_CASE(2)
    TCF_PANEL_CASE(3)
    TCF_PANEL_CASE(4)
    default:
      break;
  }
#undef TCF_PANEL_CASE
}
template void launch_panels<double>(int, int, const PanelJob*, const PanelTile*, int,
                                    const double*, const double*, int, const int*, double*, int,
                                    const int*, double*, const int*, hipStream_t, double*, int,
                                    double*);
template void launch_panels<float>(int, int, const PanelJob*, const PanelTile*, int, const float*,
                                   const double*, int, const int*, double*, int, const int*,
                                   double*, const int*, hipStream_t, double*, int, double*);
void launch_stage_add(int n, const int* tgt, const int* ptr, const int* idx, const double* stage,
                      int sld, int R, double* y, int yld, const int* done, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_stage_add, dim3((n + 255) / 256), dim3(256), 0, st, n, tgt, ptr, idx, stage,
                     sld, R, y, yld, done);
}
void launch_qjob_add(int R, int njobs, const double* qjob, double* slots, const int* done,
                     hipStream_t st) {
  if (njobs == 0 || R == 0) return;
  hipLaunchKernelGGL(k_qjob_add, dim3(R), dim3(256), 0, st, njobs, qjob, slots, done);
}

template <class T>
void launch_tiles(int group, int R, const TileJob* jobs, int njobs, const T* M, const double* xv,
                  int xld, const int* gidx, const double* gsgn, double scale, double* y,
                  int yld, const int* ymap, double* qslot, const int* done, hipStream_t st) {
  if (njobs == 0) return;
  switch (group) {
    case 0:
      launch_tiles_g<T, 0>(R, jobs, njobs, M, xv, xld, gidx, gsgn, scale, y, yld, ymap, qslot,
                           done, st);
      break;
    case 1:
      launch_tiles_g<T, 1>(R, jobs, njobs, M, xv, xld, gidx, gsgn, scale, y, yld, ymap, qslot,
                           done, st);
      break;
    case 2:
      launch_tiles_g<T, 2>(R, jobs, njobs, M, xv, xld, gidx, gsgn, scale, y, yld, ymap, qslot,
                           done, st);
      break;
    case 3:
      launch_tiles_g<T, 3>(R, jobs, njobs, M, xv, xld, gidx, gsgn, scale, y, yld, ymap, qslot,
                           done, st);
      break;
    default:
      launch_tiles_g<T, 4>(R, jobs, njobs, M, xv, xld, gidx, gsgn, scale, y, yld, ymap, qslot,
                           done, st);
      break;
  }
}

// Range of the Cholesky factor's diagonal over each patch's real interior
// and dual rows (padding rows excluded): out[2 s] = min |L_kk|, out[2 s + 1]
// = max |L_kk|.  (max / min)^2 is the ratio of the largest to the smallest
// pivot, a lower bound on the condition number of the factored block.
template <class T>
__global__ void k_diag_range(const DevPatch* P, int np, const T* A, double* out) {
  const int s = blockIdx.x;
  if (s >= np) return;
  const DevPatch& d = P[s];
  const T* a = A + d.A_off;
  __shared__ double smin[256], smax[256];
  double lo = DBL_MAX, hi = 0.0;
  for (int k = threadIdx.x; k < d.n_i + d.n_b; k += blockDim.x) {
    const int row = k < d.n_i ? k : d.ni_pad + (k - d.n_i);
    const double v = fabs((double)a[(int64_t)row * (d.nr_pad + 1)]);
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * s] = smin[0];
    out[2 * s + 1] = smax[0];
  }
}
template <class T>
void launch_diag_range(const DevPatch* P, int np, const T* A, double* out, hipStream_t st) {
  if (np == 0) return;
  hipLaunchKernelGGL(k_diag_range<T>, dim3(np), dim3(256), 0, st, P, np, A, out);
}
template void launch_diag_range<double>(const DevPatch*, int, const double*, double*, hipStream_t);
template void launch_diag_range<float>(const DevPatch*, int, const float*, double*, hipStream_t);

// Diagonal of each patch's dual block, read from the assembled [i|b|p]
// matrix before it is factored: out[b_off + k] = A[(ni_pad + k), (ni_pad + k)].
template <class T>
__global__ void k_bdiag(const DevPatch* P, int np, const T* A, double* out) {
  const int s = blockIdx.x;
  if (s >= np) return;
  const DevPatch& d = P[s];
  const T* a = A + d.A_off;
  for (int k = threadIdx.x; k < d.n_b; k += blockDim.x)
    out[d.b_off + k] = (double)a[(int64_t)(d.ni_pad + k) * (d.nr_pad + 1)];
}
template <class T>
void launch_bdiag(const DevPatch* P, int np, const T* A, double* out, hipStream_t st) {
  if (np == 0) return;
  hipLaunchKernelGGL(k_bdiag<T>, dim3(np), dim3(256), 0, st, P, np, A, out);
}
template void launch_bdiag<double>(const DevPatch*, int, const double*, double*, hipStream_t);
template void launch_bdiag<float>(const DevPatch*, int, const float*, double*, hipStream_t);

// Plain streaming copy (measurement reference for traffic counters).
__global__ void k_copy_probe(int64_t n, const double4* a, double4* b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
void launch_copy_probe(int64_t n32, const void* a, void* b, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_probe, dim3(8192), dim3(256), 0, st, n32, (const double4*)a,
                     (double4*)b);
}

// Streaming read of n 16-byte vectors, 8 non-temporal loads in flight per
// thread (the read ceiling the bandwidth probe measures); the sum is kept
// only to keep the loads.
__global__ void __launch_bounds__(256) k_read_probe(int64_t n, const TileVec<double>::v* a,
                                                    double* out) {
  typedef TileVec<double>::v V2;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256 * 8;
  for (int64_t base = (int64_t)blockIdx.x * 256 * 8 + threadIdx.x; base < n; base += stride) {
    V2 r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = base + (int64_t)u * 256;
      r[u] = i < n ? __builtin_nontemporal_load(a + i) : V2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += r[u][0] + r[u][1];
  }
  if (acc == 1.0e300) out[0] = acc;
}
void launch_read_probe(int64_t n16, const void* a, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_read_probe, dim3(8192), dim3(256), 0, st, n16,
                     (const TileVec<double>::v*)a, out);
}
void launch_zero(int64_t n, double* a, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero, TCF_GRID(n, 256), dim3(256), 0, st, n, a);
}
// ===========================================================================
// Coarse factor: fronts of the nested-dissection elimination tree
// ===========================================================================
// Position of ND index g in the front of node c (g in its own range or in
// its structure; the structure is searched by bisection).
__device__ inline int front_pos(const CoarseNodeDev& c, const int* slist, int g) {
  if (g < c.j0 + c.nj) return g - c.j0;
  int lo = 0, hi = c.ns - 1;
  const int* S = slist + c.s_off;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (S[mid] < g) lo = mid + 1; else hi = mid;
  }
  return c.nj_pad + lo;
}

// Original entries of S_Pi = sum_s N_s^T S_pp N_s from one patch (launched
// per patch in sequence, so every entry sums its patches in one order):
// entry (gi, gj), gi >= gj, goes to the front of the node owning gj (the one
// eliminated first), lower triangle.
template <class T>
__global__ void k_front_add(const DevPatch* P, int s, const int* p_nd, const T* A,
                            const CoarseNodeDev* nodes, const int* node_of, const int* slist,
                            double* F) {
  const DevPatch& pp = P[s];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pp.n_p * pp.n_p) return;
  const int i = idx % pp.n_p, j = idx / pp.n_p;
  const int gi = p_nd[pp.p_off + i], gj = p_nd[pp.p_off + j];
  if (gi < gj) return;
  const int R = pp.ni_pad + pp.nb_pad + max(i, j), C = pp.ni_pad + pp.nb_pad + min(i, j);
  const double v = (double)A[pp.A_off + R + (int64_t)C * pp.nr_pad];
  const CoarseNodeDev c = nodes[node_of[gj]];
  const int row = front_pos(c, slist, gi), col = gj - c.j0;
  if (row < c.nf && col < c.nj) F[c.f_off + row + (int64_t)col * c.nf] += v;
}

// Extend-add of child c's update matrix (the Schur complement left in the
// trailing S x S block of its factored front) into its parent's front.
// cpos[s_off + a] is the parent front position of the child's structure
// entry a; both are ascending, so the lower triangle maps to the lower
// triangle.  One launch per child, in postorder.
__global__ void k_extend_add(const CoarseNodeDev* nodes, int c, const int* cpos, double* F) {
  const CoarseNodeDev ch = nodes[c];
  const CoarseNodeDev pa = nodes[ch.parent];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ch.ns * ch.ns) return;
  const int a = (int)(idx % ch.ns), b = (int)(idx / ch.ns);
  if (a < b) return;
  const double v = F[ch.f_off + (ch.nj_pad + a) + (int64_t)(ch.nj_pad + b) * ch.nf];
  const int* cp = cpos + ch.s_off;
  F[pa.f_off + cp[a] + (int64_t)cp[b] * pa.nf] += v;
}

// Identity diagonal on the padding of each node's own block.
__global__ void k_front_pad(const CoarseNodeDev* nodes, double* F) {
  const CoarseNodeDev c = nodes[blockIdx.x];
  for (int r = c.nj + threadIdx.x; r < c.nj_pad; r += blockDim.x)
    F[c.f_off + r + (int64_t)r * c.nf] = 1.0;
}

// Right-hand sides of the explicit operators of non-root nodes, ld nj_pad:
// columns [0, nj) the identity (for L_JJ^-1), columns nj .. nj + ns the
// negated transpose of L_SJ (for -L_JJ^-T L_SJ^T).  One block per column.
__global__ void k_front_rhs(const CoarseNodeDev* nodes, const int* jobs, const int* prefix,
                            int njobs, const double* F, double* L) {
  const int j = find_job(prefix, njobs, blockIdx.x);
  const CoarseNodeDev c = nodes[jobs[j]];
  const int col = blockIdx.x - prefix[j];
  double* o = L + c.l_off + (int64_t)col * c.nj_pad;
  for (int r = threadIdx.x; r < c.nj_pad; r += blockDim.x) {
    double v;
    if (col < c.nj) v = (r == col) ? 1.0 : 0.0;
    else v = -F[c.f_off + (c.nj_pad + (col - c.nj)) + (int64_t)r * c.nf];
    o[r] = v;
  }
}

// slots[j * TCF_QSLOTS + k] += sum of squares of part of column j of y
// (y[j * ld + i], i < n).  Blocks of 256 threads, grid (chunks, R).
__global__ void __launch_bounds__(256) k_sumsq_slots(int n, const double* y, int ld,
                                                     double* slots, const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int j = blockIdx.y;
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double t = y[(int64_t)j * ld + i];
    v += t * t;
  }
  v = block_sum256(v, sh);
  if (threadIdx.x == 0) atomicAdd(slots + j * TCF_QSLOTS + (blockIdx.x & (TCF_QSLOTS - 1)), v);
}

template <class T>
void launch_front_add(const DevPatch* P, int s, int n_p, const int* p_nd, const T* A,
                      const CoarseNodeDev* nodes, const int* node_of, const int* slist, double* F,
                      hipStream_t st) {
  if (n_p == 0) return;
  hipLaunchKernelGGL(k_front_add<T>, TCF_GRID(n_p * n_p, 256), dim3(256), 0, st, P, s, p_nd, A,
                     nodes, node_of, slist, F);
}
template void launch_front_add<double>(const DevPatch*, int, int, const int*, const double*,
                                       const CoarseNodeDev*, const int*, const int*, double*,
                                       hipStream_t);
template void launch_front_add<float>(const DevPatch*, int, int, const int*, const float*,
                                      const CoarseNodeDev*, const int*, const int*, double*,
                                      hipStream_t);
void launch_extend_add(const CoarseNodeDev* nodes, int c, int ns, const int* cpos, double* F,
                       hipStream_t st) {
  if (ns == 0) return;
  hipLaunchKernelGGL(k_extend_add, TCF_GRID((int64_t)ns * ns, 256), dim3(256), 0, st, nodes, c,
                     cpos, F);
}
void launch_front_pad(const CoarseNodeDev* nodes, int nn, double* F, hipStream_t st) {
  if (nn == 0) return;
  hipLaunchKernelGGL(k_front_pad, dim3(nn), dim3(64), 0, st, nodes, F);
}
void launch_front_rhs(const CoarseNodeDev* nodes, const int* jobs, const int* prefix, int njobs,
                      int total, const double* F, double* L, hipStream_t st) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_front_rhs, dim3(total), dim3(256), 0, st, nodes, jobs, prefix, njobs, F, L);
}
__global__ void __launch_bounds__(256) k_gather_cols(int n, int R, const int* idx,
                                                     const double* w, double scale,
                                                     const double* src, int sld, double* dst,
                                                     int dld, const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int g = idx[i];
  const double f = w ? scale * w[i] : scale;
  for (int j = 0; j < R; ++j)
    dst[(int64_t)j * dld + i] = f * src[(int64_t)j * sld + g];
}
void launch_gather_cols(int R, int n, const int* idx, const double* w, double scale,
                        const double* src, int sld, double* dst, int dld, const int* done,
                        hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3((n + 255) / 256), dim3(256), 0, st, n, R, idx, w, scale,
                     src, sld, dst, dld, done);
}

void launch_sumsq_slots(int R, int n, const double* y, int ld, double* slots, const int* done,
                        hipStream_t st) {
  if (n == 0) return;
  const int chunks = std::min(256, (n + 2047) / 2048);
  hipLaunchKernelGGL(k_sumsq_slots, dim3(chunks, R), dim3(256), 0, st, n, y, ld, slots, done);
}

template void launch_pack_tiles<double, double>(const PackJob*, int, const double*, double*,
                                                hipStream_t);
template void launch_pack_tiles<float, float>(const PackJob*, int, const float*, float*,
                                              hipStream_t);
template void launch_tiles<double>(int, int, const TileJob*, int, const double*, const double*,
                                   int, const int*, const double*, double, double*, int,
                                   const int*, double*, const int*, hipStream_t);
template void launch_tiles<float>(int, int, const TileJob*, int, const float*, const double*, int,
                                  const int*, const double*, double, double*, int, const int*,
                                  double*, const int*, hipStream_t);
}  // namespace tcf
