"""Pins of the patch-by-patch step residual (oracle/residual.py).

* Translation invariance, the fact the residual's reuse of local matrices
  rests on: patches of the same shape and material assembled one by one
  give the same local M and K.
* The oracle's own direct solution has a residual at rounding level, and
  the residual equals the one computed with the globally assembled W.
* A planted error in the field is seen.
"""
import numpy as np

import workloads as W
from oracle import residual, solve
from oracle.assemble import assemble_global, assemble_patch
from oracle.grid import build_grid


def test_same_shape_patches_have_the_same_local_matrices():
    prob = W.largest_multirhs(P=(4, 2, 2), n=3, p=2, n_rhs=1, n_steps=1)
    grid = build_grid(prob)
    keys = [residual.shape_key(prob, s) for s in range(prob.n_patches)]
    pairs = [(0, 2), (1, 3), (0, 5)]   # same parity of i + j + k: same sigma
    for a, b in pairs:
        assert keys[a] == keys[b]
        A, B = assemble_patch(prob, grid, a), assemble_patch(prob, grid, b)
        for X, Y in ((A.M, B.M), (A.K, B.K)):
            d = abs(X - Y).max()
            assert d <= 1e-13 * abs(X).max(), d
    assert keys[0] != keys[1]               # conductor and insulator differ


def _residuals(prob, steps):
    run = solve.run(prob, n_steps=steps)
    grid = run.sys.grid
    K = run.topo.kept
    ops, keys = residual.local_operators(prob, grid)
    out = []
    for k in range(prob.n_rhs):
        loads = [residual.patch_load(prob, s, [k])[:, 0] for s in range(prob.n_patches)]
        prev = np.zeros(grid.n_edges)
        for l in range(steps):
            a = run.fields[l][:, k]
            g = prob.amp[k, l]
            out.append((residual.step_residual(prob, grid, K, ops, keys, loads, prev, a, g),
                        run, k, l, loads, prev.copy(), a.copy()))
            prev = a
    return out, ops, keys


def test_oracle_solution_has_rounding_level_residual_and_matches_global_assembly():
    prob = W.largest_multirhs(P=(2, 2, 2), n=3, p=2, n_rhs=2, n_steps=2)
    rows, ops, keys = _residuals(prob, 2)
    gsys = assemble_global(prob)
    Wg = gsys.W(prob.dt)
    for r, run, k, l, loads, prev, a in rows:
        assert r <= 1e-12, r
        K = run.topo.kept
        f = gsys.M @ prev + prob.dt * prob.amp[k, l] * gsys.jhat[:, k]
        rg = np.linalg.norm(f[K] - (Wg @ a)[K]) / np.linalg.norm(f[K])
        assert abs(r - rg) <= 1e-12


def test_planted_field_error_is_seen():
    prob = W.largest_multirhs(P=(2, 2, 2), n=3, p=2, n_rhs=1, n_steps=1)
    rows, ops, keys = _residuals(prob, 1)
    r, run, k, l, loads, prev, a = rows[0]
    b = a.copy()
    e = run.topo.kept[len(run.topo.kept) // 2]
    b[e] *= 1.0 + 1e-6
    grid = run.sys.grid
    rb = residual.step_residual(prob, grid, run.topo.kept, ops, keys, loads, prev, b,
                                prob.amp[k, l])
    assert rb > 1e3 * max(r, 1e-16)
