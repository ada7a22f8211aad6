"""Implicit Euler on the globally assembled, gauged system (oracle).

Sec. 2.2 (implicit Euler system): with W = M + dt K and
f^(l+1) = M a^(l) + dt j^(l+1), each step solves the coupled system for the
new potential.  Because every interface unknown left after the split of
Sec. 3 is either primal (one shared value) or tied by a multiplier, the
dual-primal solution equals the solution of the conforming global system
restricted to the kept edges K = all edges - Dirichlet - gauge tree, with
the eliminated edges at zero.  The oracle solves exactly that:

    W_g a_K^(l+1) = (M a^(l) + dt g(t_{l+1}) jhat)_K,   a^(0) = 0,

with one sparse LU factorisation of W_g reused for every step.  With an
initial value A(x, 0) (Sec. 2.1) the first step's M a^(0) is the load
int sigma A(x,0) . w_e (a^(0) = its sigma-weighted L2 projection).

The factorisation takes W_g symmetrically permuted by a geometric nested
dissection of its unknowns (``ordering.py``), with SuperLU told to keep
that order and the diagonal pivots (W_g is symmetric positive definite).
The permutation changes only the fill of the factor, and so whether the
full-size systems fit one CPU; the solution is that of W_g itself.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import GlobalSystem, assemble_global
from .gauge import Topology, compute_topology
from .grid import build_grid
from .ordering import edge_midpoints, nested_dissection


@dataclass
class OracleRun:
    sys: GlobalSystem
    topo: Topology
    fields: list                  # a^(l+1), l = 0..n_steps-1, each (n_edges, n_rhs)
    timings: dict = field(default_factory=dict)


def gauged_matrix(sys: GlobalSystem, topo: Topology, dt: float):
    K = topo.kept
    W = sys.W(dt)
    return W[K][:, K].tocsc(), K


class GaugedSolver:
    """Factor of W_g in nested-dissection order; solve(f_K) returns a_K."""

    def __init__(self, Wg, grid, K):
        self.perm = nested_dissection(Wg, edge_midpoints(grid, K))
        Wp = Wg[self.perm][:, self.perm].tocsc()
        self.lu = spla.splu(Wp, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def solve(self, f):
        x = np.empty_like(f)
        x[self.perm] = self.lu.solve(np.ascontiguousarray(f[self.perm]))
        return x


def run(prob, n_steps=None, keep_fields=True) -> OracleRun:
    t0 = time.perf_counter()
    grid = build_grid(prob)
    sys = assemble_global(prob, grid)
    t1 = time.perf_counter()
    topo = compute_topology(prob, grid)
    t2 = time.perf_counter()
    Wg, K = gauged_matrix(sys, topo, prob.dt)
    lu = GaugedSolver(Wg, grid, K)
    t3 = time.perf_counter()
    nE = grid.n_edges
    a = np.zeros((nE, prob.n_rhs))
    fields = []
    steps = prob.n_steps if n_steps is None else int(n_steps)
    t_solve = 0.0
    for l in range(steps):
        ts = time.perf_counter()
        f = sys.M @ a + prob.dt * sys.jhat * prob.amp[:, l][None, :]
        if l == 0 and sys.m0 is not None:
            f = f + sys.m0
        a = np.zeros((nE, prob.n_rhs))
        a[K] = lu.solve(np.ascontiguousarray(f[K]))
        t_solve += time.perf_counter() - ts
        if keep_fields:
            fields.append(a.copy())
    if not keep_fields:
        fields.append(a.copy())
    return OracleRun(sys=sys, topo=topo, fields=fields,
                     timings={"assemble": t1 - t0, "tree": t2 - t1, "factor": t3 - t2,
                              "solve": t_solve, "steps": steps})
