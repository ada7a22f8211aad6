"""Field-dependent reluctivity nu(|B|), one fixed-point iteration per time
step (oracle; test infrastructure).

Sec. 2 notes that a nonlinear material law nu(|B|) extends the linear
setting in a straightforward way: each implicit-Euler step becomes a
nonlinear system, solved by a sequence of linear ones of the same form.
The paper fixes neither the material curve nor the linearisation; the
readings taken here:
* the curve is the exponential (Brauer) form nu(b2) = k1 exp(k2 b2) + k3 of
  the squared flux density b2 = |B|^2, applied in the patches marked
  nonlinear (the other patches keep their constant nu);
* nu is constant per element, evaluated at the element's mean of |B|^2
  (an integral average over the element, B = curl A of the current iterate);
* the linearisation is the fixed-point (Picard) iteration: assemble K with
  the current nu, solve the step's linear system W a = f, re-evaluate nu,
  until the relative change of a is below ``tol``; the first iterate of a
  step takes nu from the previous step's field.
The linear systems are solved exactly as the linear oracle does (global
assembly, the same gauge and kept edges, SuperLU).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .assemble import assemble_global, assemble_patch
from .errors import patch_fields
from .gauge import compute_topology
from .grid import build_grid
from .solve import GaugedSolver


def brauer_nu(b2, k1, k2, k3):
    """nu(|B|^2) = k1 exp(k2 |B|^2) + k3."""
    return k1 * np.exp(k2 * np.asarray(b2, dtype=np.float64)) + k3


def element_b2(prob, grid, s, a):
    """Mean of |curl A|^2 over each element of patch s, shape (nz, ny, nx),
    for the global edge vector ``a`` (one column): the integral of |B|^2 on a
    tensor Gauss rule of p_d + 3 points (exact for these polynomials) divided
    by the element's volume."""
    _, _, _, W, _, curl = patch_fields(prob, grid, s, a)
    b2 = np.sum(curl * curl, axis=-1) * W          # (nxq, nyq, nzq)
    nel = [int(prob.nel[d][prob.patch_ijk(s)[d]]) for d in range(3)]
    q = [b2.shape[d] // nel[d] for d in range(3)]
    e = b2.reshape(nel[0], q[0], nel[1], q[1], nel[2], q[2]).sum(axis=(1, 3, 5))
    vol = W.reshape(nel[0], q[0], nel[1], q[1], nel[2], q[2]).sum(axis=(1, 3, 5))
    return np.transpose(e / vol, (2, 1, 0))        # (nz, ny, nx)


def assemble_K(prob, grid, nu_elems, cache=None):
    """Global curl-curl matrix with nu per element on the patches where
    nu_elems[s] is given (shape (nz, ny, nx)), the patch's constant nu
    elsewhere.  ``cache`` (dict) keeps the constant patches' matrices."""
    nE = grid.n_edges
    rows, cols, vals = [], [], []
    for s in range(prob.n_patches):
        if nu_elems[s] is None and cache is not None and s in cache:
            pm = cache[s]
        else:
            pm = assemble_patch(prob, grid, s, nu_elem=nu_elems[s])
            if nu_elems[s] is None and cache is not None:
                cache[s] = pm
        Kc = pm.K.tocoo()
        rows.append(pm.gid[Kc.row])
        cols.append(pm.gid[Kc.col])
        vals.append(Kc.data)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nE, nE))


@dataclass
class PicardRun:
    fields: list        # a^(l+1), l = 0..n_steps-1, each (n_edges, n_rhs)
    iterations: list    # per step and excitation: fixed-point iterations taken
    nu: list            # per step: the last iterate's nu per nonlinear patch (excitation 0)


def run_picard(prob, curve, nonlinear, n_steps=None, tol=1e-12, maxit=60) -> PicardRun:
    """Implicit Euler with nu(|B|) in the patches where ``nonlinear[s]`` is
    true, ``curve`` = (k1, k2, k3).  Each excitation is its own nonlinear
    problem (nu follows its own field)."""
    grid = build_grid(prob)
    sys = assemble_global(prob, grid)
    topo = compute_topology(prob, grid)
    K_kept = topo.kept
    cache = {}
    nE = grid.n_edges
    steps = prob.n_steps if n_steps is None else int(n_steps)
    a = np.zeros((nE, prob.n_rhs))
    fields, iters, nus = [], [], []
    for l in range(steps):
        f = sys.M @ a + prob.dt * sys.jhat * prob.amp[:, l][None, :]
        if l == 0 and sys.m0 is not None:
            f = f + sys.m0
        a_new = np.zeros_like(a)
        it_l = []
        nu_l = None
        for k in range(prob.n_rhs):
            x = a[:, k].copy()
            for it in range(1, maxit + 1):
                nu_e = [brauer_nu(element_b2(prob, grid, s, x), *curve) if nonlinear[s] else None
                        for s in range(prob.n_patches)]
                Kg = assemble_K(prob, grid, nu_e, cache)
                W = (sys.M + prob.dt * Kg).tocsr()
                Wg = W[K_kept][:, K_kept].tocsc()
                y = np.zeros(nE)
                y[K_kept] = GaugedSolver(Wg, grid, K_kept).solve(np.ascontiguousarray(f[K_kept, k]))
                done = np.linalg.norm(y - x) <= tol * np.linalg.norm(y)
                x = y
                if done:
                    break
            else:
                raise RuntimeError(f"fixed point not reached in {maxit} iterations (step {l})")
            a_new[:, k] = x
            it_l.append(it)
            if k == 0:
                nu_l = nu_e
        a = a_new
        fields.append(a.copy())
        iters.append(it_l)
        nus.append(nu_l)
    return PicardRun(fields=fields, iterations=iters, nu=nus)


def nonlinear_residual(prob, curve, nonlinear, a_now, a_prev, l, k=0):
    """|W(nu(a)) a - f|_K / |f|_K for step l of excitation k, with nu taken
    from a_now itself: zero at a fixed point of the iteration."""
    grid = build_grid(prob)
    sys = assemble_global(prob, grid)
    topo = compute_topology(prob, grid)
    nu_e = [brauer_nu(element_b2(prob, grid, s, a_now[:, k]), *curve) if nonlinear[s] else None
            for s in range(prob.n_patches)]
    Kg = assemble_K(prob, grid, nu_e)
    f = sys.M @ a_prev[:, k] + prob.dt * sys.jhat[:, k] * prob.amp[k, l]
    if l == 0 and sys.m0 is not None:
        f = f + sys.m0[:, k]
    r = (sys.M + prob.dt * Kg) @ a_now[:, k] - f
    K = topo.kept
    return float(np.linalg.norm(r[K]) / np.linalg.norm(f[K]))
