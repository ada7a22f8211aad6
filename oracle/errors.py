"""L2 errors of a discrete field against a closed-form solution (oracle).

Sec. 4 checks the discretisation with a prescribed exact potential and
measures two fields.
* The flux density B = curl A, over the whole box.
* The electric field E = -dA/dt, in the conductor only.  In the insulator
  the potential is fixed only up to a gradient (the gauge), so E is not
  defined there.
Both errors should fall like h^p + 1/n_t.

This module evaluates the discrete fields from a global edge vector.
* B_h is the curl of the spline field.  For an x-edge function
  D_a(x) N_b(y) N_c(z) e_x the curl is (0, D_a N_b N'_c, -D_a N'_b N_c),
  and likewise for y and z.
* E_h is the backward difference -(a^(l) - a^(l-1)) / dt of implicit Euler.

Norms are L2 norms, taken with a tensor Gauss rule of p_d + 3 points per
element and direction on every patch.  Reading: the paper cites another work
for the exact error definition.  Here the errors are relative L2 errors,
taken as the maximum over the time levels.  E_h starts at the second level,
because the first step's a^(0) is given only weakly, through its mass
product.  ``field_errors`` gives the errors at one time level.
"""
from __future__ import annotations

import numpy as np

from . import spline
from .assemble import patch_rows
from .grid import Grid, build_grid


def _axis(bounds, n, p):
    t = spline.open_knots(bounds[0], bounds[1], n, p)
    x, w = spline.element_points(bounds[0], bounds[1], n, p + 3)
    xs = x.ravel()
    return xs, w.ravel(), spline.bsplines(t, p, xs), spline.bspline_derivs(t, p, xs), \
        spline.dsplines(t, p, xs)


def _t(fx, fy, fz, coef):
    """sum_abc fx[i,a] fy[j,b] fz[k,c] coef[c,b,a] -> (i, j, k)."""
    return np.einsum("ia,jb,kc,cba->ijk", fx, fy, fz, coef, optimize=True)


def patch_fields(prob, grid: Grid, s: int, a: np.ndarray):
    """Points, weights, A_h and curl A_h of the global edge vector ``a`` on
    the load quadrature grid of patch s.

    Returns (X, Y, Z, W, A, curlA) with A and curlA of shape (nx, ny, nz, 3).
    """
    rows = patch_rows(prob, s)
    (xs, wx, Nx, dNx, Dx), (ys, wy, Ny, dNy, Dy), (zs, wz, Nz, dNz, Dz) = [
        _axis(r[0], r[1], r[2]) for r in rows]
    mx, my, mz = grid.patch_m(s)
    gid = grid.local_edges(s)[0]
    c = np.asarray(a, dtype=np.float64)[gid]
    nX = (mx - 1) * my * mz
    nY = mx * (my - 1) * mz
    cx = c[:nX].reshape(mz, my, mx - 1)
    cy = c[nX:nX + nY].reshape(mz, my - 1, mx)
    cz = c[nX + nY:].reshape(mz - 1, my, mx)
    A = np.stack([_t(Dx, Ny, Nz, cx), _t(Nx, Dy, Nz, cy), _t(Nx, Ny, Dz, cz)], axis=-1)
    curl = np.stack([
        _t(Nx, dNy, Dz, cz) - _t(Nx, Dy, dNz, cy),   # d_y A_z - d_z A_y
        _t(Dx, Ny, dNz, cx) - _t(dNx, Ny, Dz, cz),   # d_z A_x - d_x A_z
        _t(dNx, Dy, Nz, cy) - _t(Dx, dNy, Nz, cx),   # d_x A_y - d_y A_x
    ], axis=-1)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    W = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
    return X, Y, Z, W, A, curl


def field_errors(prob, a_now, a_prev, t, B_exact, E_exact, grid: Grid | None = None):
    """Relative L2 errors of B_h = curl A_h (whole box) and of
    E_h = -(a_now - a_prev) / dt (conductor patches) at time t.

    ``B_exact(X, Y, Z, t)`` and ``E_exact(X, Y, Z, t)`` return (..., 3).
    Returns a dict with the relative errors ``eB``, ``eE`` and the absolute
    errors and reference norms behind them.
    """
    grid = grid or build_grid(prob)
    dt = float(prob.dt)
    eB2 = nB2 = eE2 = nE2 = 0.0
    for s in range(prob.n_patches):
        X, Y, Z, W, _, curl = patch_fields(prob, grid, s, a_now)
        Bx = B_exact(X, Y, Z, t)
        eB2 += float(np.sum(W[..., None] * (curl - Bx) ** 2))
        nB2 += float(np.sum(W[..., None] * Bx ** 2))
        if float(prob.sigma[s]) > 0:
            A1 = patch_fields(prob, grid, s, a_now)[4]
            A0 = patch_fields(prob, grid, s, a_prev)[4]
            Eh = -(A1 - A0) / dt
            Ex = E_exact(X, Y, Z, t)
            eE2 += float(np.sum(W[..., None] * (Eh - Ex) ** 2))
            nE2 += float(np.sum(W[..., None] * Ex ** 2))
    return {"eB": np.sqrt(eB2 / nB2), "eE": np.sqrt(eE2 / nE2) if nE2 > 0 else float("nan"),
            "eB_abs": np.sqrt(eB2), "eE_abs": np.sqrt(eE2), "B_norm": np.sqrt(nB2),
            "E_norm": np.sqrt(nE2)}


def step_errors(prob, fields, B_exact, E_exact, grid: Grid | None = None, chunk: int = 16):
    """Relative L2 errors at every time level t_l = l dt, l = 1 .. len(fields).

    ``fields[l-1]`` is the global edge vector a^(l).  Returns per-level arrays
    ``eB`` and ``eE`` (eE[0] = nan: no a^(0)) and their maxima ``eB_max``
    (over all levels) and ``eE_max`` (from the second level on).  The spline
    evaluation is the one of ``patch_fields``, applied to a block of levels
    at a time.
    """
    grid = grid or build_grid(prob)
    F = np.stack([np.asarray(f, dtype=np.float64).reshape(-1) for f in fields], axis=1)
    m = F.shape[1]
    dt = float(prob.dt)
    eB2 = np.zeros(m)
    nB2 = np.zeros(m)
    eE2 = np.zeros(m)
    nE2 = np.zeros(m)
    for s in range(prob.n_patches):
        rows = patch_rows(prob, s)
        (xs, wx, Nx, dNx, Dx), (ys, wy, Ny, dNy, Dy), (zs, wz, Nz, dNz, Dz) = [
            _axis(r[0], r[1], r[2]) for r in rows]
        mx, my, mz = grid.patch_m(s)
        gid = grid.local_edges(s)[0]
        nX = (mx - 1) * my * mz
        nY = mx * (my - 1) * mz
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        W = (wx[:, None, None] * wy[None, :, None] * wz[None, None, :])[..., None]
        cond = float(prob.sigma[s]) > 0

        def t4(fx, fy, fz, coef):
            return np.einsum("ia,jb,kc,cbam->ijkm", fx, fy, fz, coef, optimize=True)

        for m0 in range(0, m, chunk):
            cols = list(range(max(m0 - 1, 0), min(m0 + chunk, m)))
            C = F[gid][:, cols]
            q = C.shape[1]
            cx = C[:nX].reshape(mz, my, mx - 1, q)
            cy = C[nX:nX + nY].reshape(mz, my - 1, mx, q)
            cz = C[nX + nY:].reshape(mz - 1, my, mx, q)
            curl = np.stack([t4(Nx, dNy, Dz, cz) - t4(Nx, Dy, dNz, cy),
                             t4(Dx, Ny, dNz, cx) - t4(dNx, Ny, Dz, cz),
                             t4(dNx, Dy, Nz, cy) - t4(Dx, dNy, Nz, cx)], axis=-1)
            A = np.stack([t4(Dx, Ny, Nz, cx), t4(Nx, Dy, Nz, cy), t4(Nx, Ny, Dz, cz)], axis=-1) \
                if cond else None
            for c_i, l in enumerate(cols):
                if l < m0:
                    continue  # the overlap column only supplies a^(l-1)
                t = (l + 1) * dt
                Bx = B_exact(X, Y, Z, t)
                eB2[l] += float(np.sum(W * (curl[:, :, :, c_i] - Bx) ** 2))
                nB2[l] += float(np.sum(W * Bx ** 2))
                if cond and l >= 1:
                    Eh = -(A[:, :, :, c_i] - A[:, :, :, c_i - 1]) / dt
                    Ex = E_exact(X, Y, Z, t)
                    eE2[l] += float(np.sum(W * (Eh - Ex) ** 2))
                    nE2[l] += float(np.sum(W * Ex ** 2))
    eB = np.sqrt(eB2 / nB2)
    eE = np.full(m, np.nan)
    ok = nE2 > 0
    eE[ok] = np.sqrt(eE2[ok] / nE2[ok])
    return {"eB": eB, "eE": eE, "eB_max": float(np.max(eB)),
            "eE_max": float(np.nanmax(eE)) if np.any(ok) else float("nan")}
