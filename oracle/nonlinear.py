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


# --------------------------------------------------------------------------
# Newton's method for the same nonlinear step.
#
# With nu constant per element at b2_e = (1/|e|) int_e |curl a|^2 =
# a_e^T K1_e a_e / |e| (K1_e the element's curl-curl matrix for nu = 1), the
# step's residual is R(a) = (M + dt K(nu(a))) a - f and its Jacobian is
#   J(a) = M + dt [ K(nu(a)) + sum_e (2 nu'(b2_e) / |e|) g_e g_e^T ],
# g_e = K1_e a_e (the derivative of nu_e K1_e a_e with respect to a brings
# K1_e a_e times the derivative of nu_e, which is nu'(b2_e) 2 g_e^T / |e|).
# --------------------------------------------------------------------------

def brauer_dnu(b2, k1, k2, k3):
    """d nu / d(|B|^2) of the exponential curve."""
    return k1 * k2 * np.exp(k2 * np.asarray(b2, dtype=np.float64))


def element_data(prob, grid, s):
    """(global edge ids per element (E, nl), K1 (E, nl, nl), element volume)
    of patch s, elements in (z, y, x) order with x fastest."""
    els = []
    pm = assemble_patch(prob, grid, s, elements=els)
    idx = np.concatenate([e[0] for e in els])
    K1 = np.concatenate([e[1] for e in els])
    ijk = prob.patch_ijk(s)
    vol = 1.0
    for d in range(3):
        r = ijk[d]
        vol *= (float(prob.breaks[d][r + 1]) - float(prob.breaks[d][r])) / int(prob.nel[d][r])
    return pm.gid[idx], K1, vol


def _element_state(x, edata, curve):
    """b2, nu, nu' and g_e = K1_e a_e per element of one nonlinear patch."""
    gidx, K1, vol = edata
    ae = x[gidx]                                   # (E, nl)
    g = np.einsum("eij,ej->ei", K1, ae)
    b2 = np.einsum("ei,ei->e", ae, g) / vol
    return b2, brauer_nu(b2, *curve), brauer_dnu(b2, *curve), g


def _k_nu(prob, grid, x, curve, nonlinear, edatas, cache):
    nu_e = [None] * prob.n_patches
    for s in range(prob.n_patches):
        if nonlinear[s]:
            _, nu, _, _ = _element_state(x, edatas[s], curve)
            nel = [int(prob.nel[d][prob.patch_ijk(s)[d]]) for d in range(3)]
            nu_e[s] = nu.reshape(nel[2], nel[1], nel[0])
    return assemble_K(prob, grid, nu_e, cache)


def step_residual(prob, grid, sys, x, f, curve, nonlinear, edatas, cache=None):
    """R(x) = (M + dt K(nu(x))) x - f (all edges)."""
    return (sys.M + prob.dt * _k_nu(prob, grid, x, curve, nonlinear, edatas, cache)) @ x - f


def step_jacobian(prob, grid, sys, x, curve, nonlinear, edatas, cache=None):
    """J(x) of the step residual (all edges, sparse)."""
    Kg = _k_nu(prob, grid, x, curve, nonlinear, edatas, cache)
    rows, cols, vals = [], [], []
    for s in range(prob.n_patches):
        if not nonlinear[s]:
            continue
        gidx, _, vol = edatas[s]
        _, _, dnu, g = _element_state(x, edatas[s], curve)
        w = 2.0 * dnu / vol
        nl = gidx.shape[1]
        rows.append(np.repeat(gidx[:, :, None], nl, axis=2).ravel())
        cols.append(np.repeat(gidx[:, None, :], nl, axis=1).ravel())
        vals.append((w[:, None, None] * g[:, :, None] * g[:, None, :]).ravel())
    nE = grid.n_edges
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nE, nE)) if rows else sp.csr_matrix((nE, nE))
    return (sys.M + prob.dt * (Kg + D)).tocsr()


@dataclass
class NewtonRun:
    fields: list        # a^(l+1) per step, (n_edges, n_rhs)
    iterations: list    # per step and excitation: Newton iterations taken
    residuals: list     # per step, excitation 0: |R|_K / |f|_K before each iteration


def run_newton(prob, curve, nonlinear, n_steps=None, tol=1e-12, maxit=40) -> NewtonRun:
    """Implicit Euler with nu(|B|) solved per step by Newton's method from
    the previous step's field; stops when the update is below ``tol``
    relative to the field."""
    grid = build_grid(prob)
    sys = assemble_global(prob, grid)
    topo = compute_topology(prob, grid)
    Kk = topo.kept
    edatas = [element_data(prob, grid, s) if nonlinear[s] else None
              for s in range(prob.n_patches)]
    cache = {}
    nE = grid.n_edges
    steps = prob.n_steps if n_steps is None else int(n_steps)
    a = np.zeros((nE, prob.n_rhs))
    fields, iters, res = [], [], []
    for l in range(steps):
        f = sys.M @ a + prob.dt * sys.jhat * prob.amp[:, l][None, :]
        if l == 0 and sys.m0 is not None:
            f = f + sys.m0
        a_new = np.zeros_like(a)
        it_l, res_l = [], []
        for k in range(prob.n_rhs):
            x = a[:, k].copy()
            fk = f[:, k]
            fn = np.linalg.norm(fk[Kk])
            for it in range(1, maxit + 1):
                R = step_residual(prob, grid, sys, x, fk, curve, nonlinear, edatas, cache)
                if k == 0:
                    res_l.append(float(np.linalg.norm(R[Kk]) / fn))
                J = step_jacobian(prob, grid, sys, x, curve, nonlinear, edatas, cache)
                Jg = J[Kk][:, Kk].tocsc()
                d = np.zeros(nE)
                d[Kk] = -GaugedSolver(Jg, grid, Kk).solve(np.ascontiguousarray(R[Kk]))
                x = x + d
                if np.linalg.norm(d) <= tol * np.linalg.norm(x):
                    break
            else:
                raise RuntimeError(f"Newton did not converge in {maxit} iterations (step {l})")
            a_new[:, k] = x
            it_l.append(it)
        a = a_new
        fields.append(a.copy())
        iters.append(it_l)
        res.append(res_l)
    return NewtonRun(fields=fields, iterations=iters, residuals=res)
