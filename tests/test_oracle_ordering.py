"""The oracle's nested-dissection ordering changes nothing but the fill.

* it is a permutation of the gauged unknowns;
* every split leaves no structural nonzero of W_g between its two halves
  (the dissection property that confines the fill);
* the factor in that order solves W_g: the same field as a dense
  numpy solve of the gauged system, and as SuperLU in its default order.
"""
import numpy as np
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble, gauge, grid as G, solve
from oracle.ordering import edge_midpoints, nested_dissection
from tests.test_oracle_gauge import CASES, tiny


def _system(prob):
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    Wg, K = solve.gauged_matrix(sysm, topo, prob.dt)
    return g, sysm, topo, Wg, K


def test_dissection_splits_decouple():
    prob = W.subproblem(W.uneven_fp64(), P=(2, 2, 2))
    g, sysm, topo, Wg, K = _system(prob)
    splits = []
    perm = nested_dissection(Wg, edge_midpoints(g, K), leaf=64, splits=splits)
    assert np.array_equal(np.sort(perm), np.arange(Wg.shape[0]))
    assert len(splits) > 10
    A = Wg.tocsr()
    for lo, hi, sep in splits:
        if len(lo) and len(hi):
            assert A[lo][:, hi].nnz == 0
        # the separator really is needed: it couples to the upper half
        if len(sep) and len(hi):
            assert A[sep][:, hi].nnz > 0


def test_ordered_factor_solves_the_gauged_system():
    for name in ("cond_bottom_p2", "floating_p2", "checker"):
        P, n, p, sig = CASES[name]
        prob = tiny(P, n, p, sig)
        g, sysm, topo, Wg, K = _system(prob)
        rng = np.random.default_rng(5)
        f = rng.standard_normal((len(K), 2))
        x = solve.GaugedSolver(Wg, g, K).solve(f)
        x_dense = np.linalg.solve(Wg.toarray(), f)
        assert np.abs(x - x_dense).max() <= 1e-11 * np.abs(x_dense).max()
        x_default = spla.splu(Wg.tocsc()).solve(f)
        assert np.abs(x - x_default).max() <= 1e-11 * np.abs(x_default).max()
