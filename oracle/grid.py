"""Global control grid of a multi-patch box (oracle).

Patches are axis-aligned boxes arranged in rows.  Row r of direction d has
m = nel + deg control nodes; neighbouring rows share their boundary node
plane, so the global grid has N_d = sum_r (m_r - 1) + 1 nodes per direction
(the conforming-interface requirement of Sec. 2.2).

Numbering conventions:

* node (I, J, K) -> I + Nx (J + Ny K);
* x-edge from (I,J,K) to (I+1,J,K) -> I + (Nx-1)(J + Ny K);
* y-edges follow with offset Ex = (Nx-1) Ny Nz: Ex + I + Nx (J + (Ny-1) K);
* z-edges follow with offset Ex + Ey: Ex + Ey + I + Nx (J + Ny K);
* every edge is oriented from the lower to the higher node index.

Inside a patch the same scheme runs over the patch's own node box.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

WIREBASKET, FACE, INTERIOR = 0, 1, 2


@dataclass
class Grid:
    P: tuple            # patches per direction
    m: list             # m[d][r] = nodes of row r along d
    off: list           # off[d][r] = first global node index of row r
    N: tuple            # global nodes per direction
    planes: list        # planes[d] = sorted global node indices on break planes
    Ex: int
    Ey: int
    Ez: int

    @property
    def n_edges(self) -> int:
        return self.Ex + self.Ey + self.Ez

    @property
    def n_nodes(self) -> int:
        return self.N[0] * self.N[1] * self.N[2]

    # ---- patches -------------------------------------------------------
    def patch_ijk(self, s):
        P0, P1, _ = self.P
        return s % P0, (s // P0) % P1, s // (P0 * P1)

    def patch_box(self, s):
        """Inclusive global node ranges ((I0,I1),(J0,J1),(K0,K1)) of patch s."""
        ijk = self.patch_ijk(s)
        return tuple((self.off[d][ijk[d]], self.off[d][ijk[d]] + self.m[d][ijk[d]] - 1)
                     for d in range(3))

    def patch_m(self, s):
        ijk = self.patch_ijk(s)
        return tuple(int(self.m[d][ijk[d]]) for d in range(3))

    # ---- edges ---------------------------------------------------------
    def edge_id(self, direction, I, J, K):
        Nx, Ny, Nz = self.N
        if direction == 0:
            return I + (Nx - 1) * (J + Ny * K)
        if direction == 1:
            return self.Ex + I + Nx * (J + (Ny - 1) * K)
        return self.Ex + self.Ey + I + Nx * (J + Ny * K)

    def edge_decode(self, e):
        """Global edge id -> (direction, I, J, K) of its lower node (arrays ok)."""
        e = np.asarray(e, dtype=np.int64)
        Nx, Ny, Nz = self.N
        d = np.where(e < self.Ex, 0, np.where(e < self.Ex + self.Ey, 1, 2))
        r = e - np.where(d == 0, 0, np.where(d == 1, self.Ex, self.Ex + self.Ey))
        nx = np.where(d == 0, Nx - 1, Nx)
        ny = np.where(d == 1, Ny - 1, Ny)
        I = r % nx
        J = (r // nx) % ny
        K = r // (nx * ny)
        return d, I, J, K

    def edge_nodes(self, e):
        """Global node ids (tail, head) of edges e."""
        d, I, J, K = self.edge_decode(e)
        Nx, Ny, _ = self.N
        tail = I + Nx * (J + Ny * K)
        hI = I + (d == 0)
        hJ = J + (d == 1)
        hK = K + (d == 2)
        head = hI + Nx * (hJ + Ny * hK)
        return tail, head

    def local_edges(self, s):
        """Global ids of the local edges of patch s, in local order.

        Local order: x-edges (a,b,c) with a fastest, then y-edges, then
        z-edges, over the patch node box of m = (mx, my, mz) nodes.
        Returns (gid, direction, a, b, c) arrays.
        """
        (I0, _), (J0, _), (K0, _) = self.patch_box(s)
        mx, my, mz = self.patch_m(s)
        out = []
        for d, dims in ((0, (mx - 1, my, mz)), (1, (mx, my - 1, mz)), (2, (mx, my, mz - 1))):
            c, b, a = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]),
                                  indexing="ij")
            a, b, c = a.ravel(), b.ravel(), c.ravel()
            gid = self.edge_id(d, I0 + a, J0 + b, K0 + c)
            out.append((gid, np.full(a.shape, d), a, b, c))
        return tuple(np.concatenate([o[k] for o in out]) for k in range(5))

    # ---- classification ------------------------------------------------
    def on_plane(self, d, idx):
        return np.isin(idx, self.planes[d])

    def edge_class(self, e):
        """WIREBASKET / FACE / INTERIOR by how many transverse coordinates
        of the edge lie on patch break planes (2 / 1 / 0)."""
        d, I, J, K = self.edge_decode(e)
        c = [self.on_plane(0, I), self.on_plane(1, J), self.on_plane(2, K)]
        hits = np.zeros(np.shape(d), dtype=np.int64)
        for dd in range(3):
            hits += np.where(d != dd, c[dd], False)
        return np.where(hits == 2, WIREBASKET, np.where(hits == 1, FACE, INTERIOR))

    def node_ijk(self, n):
        Nx, Ny, _ = self.N
        n = np.asarray(n, dtype=np.int64)
        return n % Nx, (n // Nx) % Ny, n // (Nx * Ny)

    def node_on_boundary(self, n):
        I, J, K = self.node_ijk(n)
        Nx, Ny, Nz = self.N
        return (I == 0) | (I == Nx - 1) | (J == 0) | (J == Ny - 1) | (K == 0) | (K == Nz - 1)


def build_grid(prob) -> Grid:
    P = tuple(int(v) for v in prob.np)
    m, off, N, planes = [], [], [], []
    for d in range(3):
        md = [int(prob.nel[d][r]) + int(prob.deg[d][r]) for r in range(P[d])]
        od = [0]
        for r in range(P[d]):
            od.append(od[-1] + md[r] - 1)
        m.append(md)
        off.append(od[:-1])
        N.append(od[-1] + 1)
        planes.append(np.array(od, dtype=np.int64))
    Nx, Ny, Nz = N
    return Grid(P=P, m=m, off=off, N=tuple(N), planes=planes,
                Ex=(Nx - 1) * Ny * Nz, Ey=Nx * (Ny - 1) * Nz, Ez=Nx * Ny * (Nz - 1))


def incidence_G(grid: Grid):
    """Signed edge-node incidence (discrete gradient): +1 at the head (higher
    node), -1 at the tail.  Shape (n_edges, n_nodes), integer CSR."""
    import scipy.sparse as sp
    e = np.arange(grid.n_edges)
    tail, head = grid.edge_nodes(e)
    rows = np.concatenate([e, e])
    cols = np.concatenate([head, tail])
    vals = np.concatenate([np.ones(len(e), np.int64), -np.ones(len(e), np.int64)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.n_edges, grid.n_nodes))


def incidence_C(grid: Grid):
    """Signed face-edge incidence (discrete curl) of the control grid.

    A face spanned by directions (u, v) at lower node (I,J,K) has boundary
    e_u(low) + e_v(low + u) - e_u(low + v) - e_v(low), i.e. counter-clockwise
    circulation in the (u, v) plane with (u, v) in {(x,y), (y,z), (z,x)}.
    """
    import scipy.sparse as sp
    Nx, Ny, Nz = grid.N
    rows, cols, vals = [], [], []
    fid = 0
    for (u, v) in ((0, 1), (1, 2), (2, 0)):
        rng = [range(Nx), range(Ny), range(Nz)]
        rng = [np.arange(Nx - (1 if (u == 0 or v == 0) else 0)),
               np.arange(Ny - (1 if (u == 1 or v == 1) else 0)),
               np.arange(Nz - (1 if (u == 2 or v == 2) else 0))]
        K, J, I = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        n = len(I)
        ids = fid + np.arange(n)
        du = [int(u == 0), int(u == 1), int(u == 2)]
        dv = [int(v == 0), int(v == 1), int(v == 2)]
        terms = [
            (u, I, J, K, +1),
            (v, I + du[0], J + du[1], K + du[2], +1),
            (u, I + dv[0], J + dv[1], K + dv[2], -1),
            (v, I, J, K, -1),
        ]
        for (d, a, b, c, sgn) in terms:
            rows.append(ids)
            cols.append(grid.edge_id(d, a, b, c))
            vals.append(np.full(n, sgn, np.int64))
        fid += n
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fid, grid.n_edges))
