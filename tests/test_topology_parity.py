"""Bit-exact parity of the library's host combinatorics with the oracle.

The gauge tree, the interface trees, the primal / dual / interior sets, the
multiplier table (edge, +patch, -patch) and the primal assembly N must be
identical, integer for integer.  tcf_create does host work only, so these
run without a GPU.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import gauge, grid as G
from paper_2510_23446_amd import tcf
from tests.test_oracle_gauge import CASES, tiny


def _compare(prob):
    g = G.build_grid(prob)
    topo = gauge.compute_topology(prob, g)
    p = tcf.Problem(prob)
    c = p.counts()
    assert c["n_edges"] == g.n_edges
    assert c["n_nodes"] == g.n_nodes
    assert c["n_vertices_H"] == topo.n_vertices_H
    assert c["n_plain"] == topo.n_plain
    assert c["n_floating"] == topo.n_floating
    assert c["n_lambda"] == len(topo.dual)
    assert c["n_primal"] == len(topo.primal)
    assert c["n_kept"] == len(topo.kept)
    for kind, ref in [(tcf.TCF_TOPO_DIRICHLET, topo.dirichlet), (tcf.TCF_TOPO_TREE_I, topo.tree_I),
                      (tcf.TCF_TOPO_TREE_GAMMA, topo.tree_gamma), (tcf.TCF_TOPO_PRIMAL, topo.primal),
                      (tcf.TCF_TOPO_DUAL, topo.dual), (tcf.TCF_TOPO_INTERIOR, topo.interior)]:
        got = p.tcf_get_topology(kind)
        assert np.array_equal(got, np.asarray(ref, dtype=np.int64)), kind
    mult = p.tcf_get_topology(tcf.TCF_TOPO_MULT).reshape(-1, 3)
    assert np.array_equal(mult, topo.mult.reshape(-1, 3))
    N = p.tcf_get_topology(tcf.TCF_TOPO_N).reshape(-1, 3)
    ref = np.concatenate([np.stack([np.full(len(e), s), e, r], axis=1)
                          for s, (e, r) in enumerate(topo.N)] or [np.zeros((0, 3))]).astype(np.int64)
    assert np.array_equal(N, ref)
    return c


@pytest.mark.parametrize("name", sorted(CASES))
def test_tiny_cases(name):
    P, n, p, sig = CASES[name]
    _compare(tiny(P, n, p, sig))


def test_plain_workload():
    c = _compare(W.plain_fp64())
    assert c["n_lambda"] == 352 and c["n_primal"] == 90 and c["n_kept"] == 2106


def test_uneven_workload():
    _compare(W.uneven_fp64())


@pytest.mark.parametrize("seed", [2, 5])
def test_uneven_other_seeds(seed):
    _compare(W.uneven_fp64(seed=seed))


def test_floating_conductor_layout():
    c = _compare(W.floating_mixed())
    assert c["n_floating"] == 1
    assert c["n_kept"] == 229897 and c["n_lambda"] == 22044


def test_serving_requests_sample():
    reqs = W.serving_requests(n_req=24)
    for r in reqs[::3]:
        _compare(r)


def test_checkerboard_reduced():
    _compare(W.largest_multirhs(P=(4, 4, 2), n=4, n_rhs=1, n_steps=1))


@pytest.mark.slow
def test_checkerboard_full():
    c = _compare(W.largest_multirhs(n_rhs=1, n_steps=1))
    assert c["n_primal"] > 100000


def test_invalid_descriptions():
    prob = W.plain_fp64()
    bad = W.plain_fp64()
    bad.sigma = bad.sigma.copy()
    bad.sigma[3] = -1.0
    with pytest.raises(tcf.TcfError) as e:
        tcf.Problem(bad)
    assert e.value.code == tcf.TCF_EINVAL
    bad = W.plain_fp64()
    bad.nu = bad.nu.copy()
    bad.nu[0] = 0.0
    with pytest.raises(tcf.TcfError):
        tcf.Problem(bad)
    bad = W.plain_fp64()
    bad.dt = -1.0
    with pytest.raises(tcf.TcfError):
        tcf.Problem(bad)
    bad = W.plain_fp64()
    bad.breaks = [np.array([0.0, 0.5, 0.4]), prob.breaks[1], prob.breaks[2]]
    with pytest.raises(tcf.TcfError):
        tcf.Problem(bad)


def test_invalid_options():
    prob = W.plain_fp64()
    for kw in ({"pcg_warm": 4}, {"pcg_warm": -1}, {"pcg_rtol": 0.0}, {"precision": 7},
               {"precond_scaling": 2}):
        with pytest.raises(tcf.TcfError) as e:
            tcf.Problem(prob, **kw)
        assert e.value.code == tcf.TCF_EINVAL, kw
    # accepted: batch widths beyond 4 or n_rhs are clamped
    tcf.Problem(prob, rhs_batch=9, pcg_warm=2)
    tcf.Problem(prob, pcg_warm=3, precond_scaling=1)


def test_source_forms_validated():
    """A source mask needs a curl-form potential or a volume field; a volume
    field alone (the homogenised Sec. 4 problem) is accepted, and the host
    plan of the manufactured problem matches the oracle's topology counts."""
    import dataclasses
    prob = W.paper_manufactured(n=3, p=2, n_t=2)
    h = tcf.Problem(prob)
    c = h.counts()
    from oracle.gauge import compute_topology
    from oracle.grid import build_grid
    g = build_grid(prob)
    topo = compute_topology(prob, g)
    assert c["n_edges"] == g.n_edges
    assert c["n_lambda"] == len(topo.dual) and c["n_primal"] == len(topo.primal)
    bad = dataclasses.replace(prob, jvol=None, ainit=None)
    with pytest.raises(tcf.TcfError) as e:
        tcf.Problem(bad)
    assert e.value.code == tcf.TCF_EINVAL


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout


def test_full_size_checkerboard_plan():
    """Host plan of the 256-patch checkerboard at full size (8 x 8 x 4 patches,
    p = 3, n = 12).  The edge count is the control-grid closed form over the
    three edge directions, with N_x = N_y = 8 (12 + 2) + 1 and
    N_z = 4 (12 + 2) + 1 nodes.  The gauged, dual and primal counts are the
    sizes derived from the gauge and split rules (every Gamma-face tree is
    primal)."""
    prob = W.largest_multirhs(n=12, n_steps=1)
    c = tcf.Problem(prob).counts()
    Nx = Ny = 8 * (12 + 3 - 1) + 1
    Nz = 4 * (12 + 3 - 1) + 1
    edges = (Nx - 1) * Ny * Nz + Nx * (Ny - 1) * Nz + Nx * Ny * (Nz - 1)
    assert c["n_edges"] == edges == 2157848
    assert c["n_kept"] == 1776280
    assert c["n_lambda"] == 124800
    assert c["n_primal"] == 115608
