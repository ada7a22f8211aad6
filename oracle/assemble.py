"""Element-loop Galerkin assembly on the multi-patch spline space (oracle).

Sec. 2.2 defines, per subdomain, the curl-curl stiffness
(K)_jk = int nu curl w_k . curl w_j, the conductivity mass
(M)_jk = int sigma w_k . w_j, and the load (j)_j = int J . w_j.
Here every patch is an axis-aligned box with constant sigma and nu, and the
edge basis of a patch is, per Cartesian direction,

    x-edge (a,b,c):  w = D_a(x) N_b(y) N_c(z) e_x,   and cyclically,

so curl w follows from the product rule.  Integrals are computed element by
element with a tensor Gauss-Legendre rule of p_d + 1 points per direction
(exact for these polynomial integrands) and summed into local patch
matrices, which are then added into the global conforming matrices through
the patch's local-to-global edge map.

The source is J = g(t) curl Psi with Psi = (0, 0, phi).  The load uses the
curl form int Psi . curl w_e (equal to int J . w_e whenever n x Psi = 0 on
the boundary of the source region) on a rule of p_d + 3 points; the curl
form makes the load annihilate discrete gradients exactly.

A problem may instead (or also) give the source as a vector field J (the
``jvol`` callback), loaded as written in Sec. 2.2: int J . w_e, on the same
p_d + 3 point rule.  An initial potential A(x, 0) (Sec. 2.1, ``ainit``)
enters the first step through int sigma A(x,0) . w_e, which is M a^(0) for
the sigma-weighted L2 projection a^(0) of the initial value.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import spline
from .grid import Grid, build_grid


def _row_tables(a, b, n, p, nq):
    """Per-element basis tables of one patch row.

    Returns x (n, nq), w (n, nq), N (n, nq, p+1), dN (n, nq, p+1), D (n, nq, p)
    where element e uses H1 functions e..e+p and edge functions e..e+p-1.
    """
    t = spline.open_knots(a, b, n, p)
    x, w = spline.element_points(a, b, n, nq)
    flat = x.ravel()
    Nf = spline.bsplines(t, p, flat).reshape(n, nq, -1)
    dNf = spline.bspline_derivs(t, p, flat).reshape(n, nq, -1)
    Df = spline.dsplines(t, p, flat).reshape(n, nq, -1)
    N = np.stack([Nf[e, :, e:e + p + 1] for e in range(n)])
    dN = np.stack([dNf[e, :, e:e + p + 1] for e in range(n)])
    D = np.stack([Df[e, :, e:e + p] for e in range(n)])
    return x, w, N, dN, D


def _t3(fx, fy, fz):
    """Tensor product over a batch of elements.

    fx (E, qx, A), fy (E, qy, B), fz (E, qz, C) -> (E, qz*qy*qx, C*B*A)
    with the quadrature point index and the basis index both x-fastest.
    """
    E = fx.shape[0]
    T = np.einsum("exa,eyb,ezc->ezyxcba", fx, fy, fz)
    return T.reshape(E, fx.shape[1] * fy.shape[1] * fz.shape[1], -1)


@dataclass
class PatchMatrices:
    gid: np.ndarray      # local edge -> global edge id
    M: sp.csr_matrix     # sigma-weighted mass (local numbering)
    K: sp.csr_matrix     # nu-weighted curl-curl (local numbering)
    jhat: np.ndarray     # (n_local, n_rhs) source load, zero if no source
    m0: np.ndarray       # (n_local, n_rhs) initial load int sigma A(x,0) . w, zero if none


def patch_rows(prob, s):
    """(bounds, n, p) per direction for patch s."""
    ijk = prob.patch_ijk(s)
    out = []
    for d in range(3):
        r = ijk[d]
        out.append(((float(prob.breaks[d][r]), float(prob.breaks[d][r + 1])),
                    int(prob.nel[d][r]), int(prob.deg[d][r])))
    return out


def _local_index_blocks(m, rng_x, rng_y, rng_z, d):
    """Local patch edge indices of a (c,b,a)-meshgrid block of direction d."""
    mx, my, mz = m
    nX = (mx - 1) * my * mz
    nY = mx * (my - 1) * mz
    c, b, a = np.meshgrid(rng_z, rng_y, rng_x, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    if d == 0:
        return a + (mx - 1) * (b + my * c)
    if d == 1:
        return nX + a + mx * (b + (my - 1) * c)
    return nX + nY + a + mx * (b + my * c)


def assemble_patch(prob, grid: Grid, s: int, nu_elem=None, elements=None) -> PatchMatrices:
    """Local matrices of patch s.  ``nu_elem`` (optional, shape (nz, ny, nx))
    gives nu per element in place of the patch's constant nu (a
    field-dependent reluctivity, evaluated per element).  ``elements``
    (optional list) receives, per layer of elements in z, the local indices
    (E, nl) and the curl-curl element matrices with nu = 1 (E, nl, nl),
    elements x-fastest."""
    rows = patch_rows(prob, s)
    (bx, nx, px), (by, ny, py), (bz, nz, pz) = rows
    m = (nx + px, ny + py, nz + pz)
    gid, _, _, _, _ = grid.local_edges(s)
    nloc = len(gid)
    sig = float(prob.sigma[s])
    nu = float(prob.nu[s])

    tx = _row_tables(bx[0], bx[1], nx, px, px + 1)
    ty = _row_tables(by[0], by[1], ny, py, py + 1)
    tz = _row_tables(bz[0], bz[1], nz, pz, pz + 1)

    Mr, Mc, Mv, Kv = [], [], [], []
    ex_all, ey_all = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ex_all, ey_all = ex_all.ravel(), ey_all.ravel()  # ex fastest
    E = len(ex_all)
    for ez in range(nz):
        ezs = np.full(E, ez)
        _, wx, Nx, dNx, Dx = (v[ex_all] if i > 0 else None for i, v in enumerate(tx))
        _, wy, Ny, dNy, Dy = (v[ey_all] if i > 0 else None for i, v in enumerate(ty))
        _, wz, Nz, dNz, Dz = (v[ezs] if i > 0 else None for i, v in enumerate(tz))
        wq = _t3(wx[:, :, None], wy[:, :, None], wz[:, :, None])[:, :, 0]  # (E, nq3)

        blocks = []  # (val(3 comps), curl(3 comps), local idx per element)
        # x-edges: w = D N N e_x ; curl = (0, D N dN, -D dN N)
        z = None
        vx = _t3(Dx, Ny, Nz)
        blocks.append(((vx, z, z), (z, _t3(Dx, Ny, dNz), -_t3(Dx, dNy, Nz)), 0))
        # y-edges: w = N D N e_y ; curl = (-N D dN, 0, dN D N)
        vy = _t3(Nx, Dy, Nz)
        blocks.append(((z, vy, z), (-_t3(Nx, Dy, dNz), z, _t3(dNx, Dy, Nz)), 1))
        # z-edges: w = N N D e_z ; curl = (N dN D, -dN N D, 0)
        vz = _t3(Nx, Ny, Dz)
        blocks.append(((z, z, vz), (_t3(Nx, dNy, Dz), -_t3(dNx, Ny, Dz), z), 2))

        nq3 = wq.shape[1]
        nl = sum(b[0][b[2]].shape[2] for b in blocks)
        V = np.zeros((E, nq3, nl, 3))
        C = np.zeros((E, nq3, nl, 3))
        idx = np.zeros((E, nl), dtype=np.int64)
        col = 0
        for (vals, curls, d) in blocks:
            width = vals[d].shape[2]
            for comp in range(3):
                if vals[comp] is not None:
                    V[:, :, col:col + width, comp] = vals[comp]
                if curls[comp] is not None:
                    C[:, :, col:col + width, comp] = curls[comp]
            for e in range(E):
                ex, ey = ex_all[e], ey_all[e]
                lo = [ex, ey, ez]
                span = [(px + 1), (py + 1), (pz + 1)]
                span[d] -= 1
                idx[e, col:col + width] = _local_index_blocks(
                    m, np.arange(lo[0], lo[0] + span[0]), np.arange(lo[1], lo[1] + span[1]),
                    np.arange(lo[2], lo[2] + span[2]), d)
            col += width
        # element matrices: sum over points q and components c of
        # w_q curl w_i(q)_c curl w_j(q)_c, as a batched product per element
        Cq = C.transpose(0, 1, 3, 2).reshape(E, nq3 * 3, nl)
        Vq = V.transpose(0, 1, 3, 2).reshape(E, nq3 * 3, nl)
        wr = np.repeat(wq, 3, axis=1)[:, :, None]
        nu_l = nu if nu_elem is None else np.asarray(nu_elem, dtype=np.float64)[ez].ravel()[:, None, None]
        K1 = np.matmul((Cq * wr).transpose(0, 2, 1), Cq)
        Ke = nu_l * K1
        if elements is not None:
            elements.append((idx.copy(), K1))
        Me = sig * np.matmul((Vq * wr).transpose(0, 2, 1), Vq)
        Mr.append(np.repeat(idx[:, :, None], nl, axis=2).ravel())
        Mc.append(np.repeat(idx[:, None, :], nl, axis=1).ravel())
        Mv.append(Me.ravel())
        Kv.append(Ke.ravel())
    r_ = np.concatenate(Mr)
    c_ = np.concatenate(Mc)
    Mloc = sp.csr_matrix((np.concatenate(Mv), (r_, c_)), shape=(nloc, nloc))
    Kloc = sp.csr_matrix((np.concatenate(Kv), (r_, c_)), shape=(nloc, nloc))
    jloc = np.zeros((nloc, prob.n_rhs))
    if prob.src_mask[s]:
        if prob.phi is not None:
            jloc = jloc + assemble_patch_load(prob, s, m)
        if getattr(prob, "jvol", None) is not None:
            jloc = jloc + assemble_patch_vec_load(prob, s, m, prob.jvol)
    m0loc = np.zeros((nloc, prob.n_rhs))
    if getattr(prob, "ainit", None) is not None and sig > 0:
        m0loc = sig * assemble_patch_vec_load(prob, s, m, prob.ainit)
    return PatchMatrices(gid=gid, M=Mloc, K=Kloc, jhat=jloc, m0=m0loc)


def assemble_patch_vec_load(prob, s, m, fn):
    """Volume-form load int F . w_e over patch s, one column per RHS.

    F = fn(s, xs, ys, zs, k) on the tensor grid of load points, shape
    (nx, ny, nz, 3).  An edge of direction d pairs with component d only:
    x-edges take F_x D_a(x) N_b(y) N_c(z), y-edges F_y N_a D_b N_c, z-edges
    F_z N_a N_b D_c.  Gauss rule with p_d + 3 points per element and direction.
    """
    rows = patch_rows(prob, s)
    tabs = [_row_tables(r[0][0], r[0][1], r[1], r[2], r[2] + 3) for r in rows]
    (x, wx, Nx, _, Dx), (y, wy, Ny, _, Dy), (zz, wz, Nz, _, Dz) = tabs
    (nx, px), (ny, py), (nz, pz) = [(r[1], r[2]) for r in rows]
    mx, my, mz = m
    nloc = (mx - 1) * my * mz + mx * (my - 1) * mz + mx * my * (mz - 1)
    out = np.zeros((nloc, prob.n_rhs))
    qx, qy, qz = x.shape[1], y.shape[1], zz.shape[1]
    for k in range(prob.n_rhs):
        F = np.asarray(fn(s, x.ravel(), y.ravel(), zz.ravel(), k), dtype=np.float64)
        F = F.reshape(nx, qx, ny, qy, nz, qz, 3)
        for ez in range(nz):
            for ey in range(ny):
                for ex in range(nx):
                    wgt = wx[ex][:, None, None] * wy[ey][None, :, None] * wz[ez][None, None, :]
                    f = F[ex, :, ey, :, ez, :, :] * wgt[..., None]
                    for d, (fa, fb, fc) in enumerate(((Dx[ex], Ny[ey], Nz[ez]),
                                                      (Nx[ex], Dy[ey], Nz[ez]),
                                                      (Nx[ex], Ny[ey], Dz[ez]))):
                        v = np.einsum("xyz,xa,yb,zc->cba", f[..., d], fa, fb, fc).ravel()
                        span = [px + 1, py + 1, pz + 1]
                        span[d] -= 1
                        idx = _local_index_blocks(m, np.arange(ex, ex + span[0]),
                                                  np.arange(ey, ey + span[1]),
                                                  np.arange(ez, ez + span[2]), d)
                        np.add.at(out[:, k], idx, v)
    return out


def assemble_patch_load(prob, s, m):
    """Curl-form load int phi (curl w_e)_z over patch s, one column per RHS.

    (curl w)_z is -D_a dN_b N_c for x-edges, dN_a D_b N_c for y-edges and 0
    for z-edges.  Gauss rule with p_d + 3 points per element and direction.
    """
    rows = patch_rows(prob, s)
    tabs = [_row_tables(r[0][0], r[0][1], r[1], r[2], r[2] + 3) for r in rows]
    (x, wx, Nx, dNx, Dx), (y, wy, Ny, dNy, Dy), (zz, wz, Nz, dNz, Dz) = tabs
    (nx, px), (ny, py), (nz, pz) = [(r[1], r[2]) for r in rows]
    mx, my, mz = m
    nX = (mx - 1) * my * mz
    nloc = nX + mx * (my - 1) * mz + mx * my * (mz - 1)
    out = np.zeros((nloc, prob.n_rhs))
    qx, qy, qz = x.shape[1], y.shape[1], zz.shape[1]
    for k in range(prob.n_rhs):
        phi = np.asarray(prob.phi(x.ravel(), y.ravel(), zz.ravel(), k), dtype=np.float64)
        phi = phi.reshape(nx, qx, ny, qy, nz, qz)
        for ez in range(nz):
            for ey in range(ny):
                for ex in range(nx):
                    f = phi[ex, :, ey, :, ez, :] * (wx[ex][:, None, None] * wy[ey][None, :, None]
                                                   * wz[ez][None, None, :])
                    # x-edges: -D_a(x) dN_b(y) N_c(z)
                    vxe = -np.einsum("xyz,xa,yb,zc->cba", f, Dx[ex], dNy[ey], Nz[ez]).ravel()
                    ix = _local_index_blocks(m, np.arange(ex, ex + px), np.arange(ey, ey + py + 1),
                                             np.arange(ez, ez + pz + 1), 0)
                    np.add.at(out[:, k], ix, vxe)
                    # y-edges: dN_a(x) D_b(y) N_c(z)
                    vye = np.einsum("xyz,xa,yb,zc->cba", f, dNx[ex], Dy[ey], Nz[ez]).ravel()
                    iy = _local_index_blocks(m, np.arange(ex, ex + px + 1), np.arange(ey, ey + py),
                                             np.arange(ez, ez + pz + 1), 1)
                    np.add.at(out[:, k], iy, vye)
    return out


@dataclass
class GlobalSystem:
    grid: Grid
    M: sp.csr_matrix       # sum over patches of sigma-mass
    K: sp.csr_matrix       # sum over patches of nu curl-curl
    jhat: np.ndarray       # (n_edges, n_rhs)
    patches: list          # PatchMatrices per patch
    m0: np.ndarray = None  # (n_edges, n_rhs) initial load, zeros if no initial value

    def W(self, dt):
        return (self.M + dt * self.K).tocsr()


def assemble_global(prob, grid: Grid | None = None, keep_patches=True) -> GlobalSystem:
    """Sum the local patch matrices into the global conforming matrices
    through each patch's local-to-global edge map (one COO build)."""
    grid = grid or build_grid(prob)
    nE = grid.n_edges
    rows, cols, mv, kv = [], [], [], []
    jg = np.zeros((nE, prob.n_rhs))
    m0 = np.zeros((nE, prob.n_rhs))
    pats = []
    for s in range(prob.n_patches):
        pm = assemble_patch(prob, grid, s)
        Mc = pm.M.tocoo()
        Kc = pm.K.tocoo()
        assert np.array_equal(Mc.row, Kc.row) and np.array_equal(Mc.col, Kc.col)
        rows.append(pm.gid[Mc.row])
        cols.append(pm.gid[Mc.col])
        mv.append(Mc.data)
        kv.append(Kc.data)
        np.add.at(jg, pm.gid, pm.jhat)
        np.add.at(m0, pm.gid, pm.m0)
        if keep_patches:
            pats.append(pm)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    Mg = sp.csr_matrix((np.concatenate(mv), (r, c)), shape=(nE, nE))
    Kg = sp.csr_matrix((np.concatenate(kv), (r, c)), shape=(nE, nE))
    return GlobalSystem(grid=grid, M=Mg, K=Kg, jhat=jg, patches=pats, m0=m0)
