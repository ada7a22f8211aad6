"""Pins of the oracle's gauge and dual-primal split on tiny meshes.

* kernel dimension: dense eigenvalues of the non-Dirichlet system show
  exactly #plain + #floating zero modes (discrete gradients that vanish on
  the root and are constant on each floating conductor), and the tree has
  exactly that many edges;
* the gauged system is SPD;
* gauge validity: the minimum-norm solution of the singular ungauged system
  and the gauged solution have the same fluxes C a and the same values on
  conductor edges, every step; an over-eliminated set fails this;
* every local remainder block W_rr^(s) (r = interior + dual) is SPD,
  floating insulators included, and the assembled coarse matrix is SPD;
* the paper's own two-subdomain setting reduces to: primal = Gamma tree,
  eliminated = Dirichlet + interior insulator tree;
* the dual-primal three-field system, solved densely, has zero interface
  jump and reproduces the global gauged solution;
* implicit Euler against dense numpy solves.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assemble, gauge, grid as G, solve
from tests.feti_ref import DenseFETI


def tiny(P, n, p, sigma, nu=1.0, dt=0.1, src=None, steps=3, phi=None):
    npatch = P[0] * P[1] * P[2]
    sigma = np.asarray(sigma, float)
    return W.Problem(
        name="tiny", np=tuple(P), breaks=[np.linspace(0, 1, P[d] + 1) for d in range(3)],
        nel=[np.full(P[d], n, np.int32) for d in range(3)],
        deg=[np.full(P[d], p, np.int32) for d in range(3)],
        sigma=sigma, nu=np.full(npatch, nu),
        src_mask=(sigma == 0).astype(np.uint8) if src is None else np.asarray(src, np.uint8),
        phi=phi or (lambda x, y, z, k: (np.sin(np.pi * x)[:, None, None] * np.sin(np.pi * y)[None, :, None]
                                        * (1 + z)[None, None, :])),
        amp=np.linspace(1.0, 2.0, steps)[None, :], dt=dt, n_steps=steps)


def _center(P):
    out = np.zeros(P[0] * P[1] * P[2])
    for s in range(len(out)):
        i, j, k = s % P[0], (s // P[0]) % P[1], s // (P[0] * P[1])
        if 0 < i < P[0] - 1 and 0 < j < P[1] - 1 and 0 < k < P[2] - 1:
            out[s] = 2.0
    return out


CASES = {
    "cond_bottom": ((2, 2, 2), 2, 1, [1, 1, 1, 1, 0, 0, 0, 0]),
    "cond_bottom_p2": ((2, 2, 2), 2, 2, [1, 1, 1, 1, 0, 0, 0, 0]),
    "floating": ((3, 3, 3), 1, 1, _center((3, 3, 3))),
    "floating_p2": ((3, 3, 3), 1, 2, _center((3, 3, 3))),
    "checker": ((2, 2, 2), 2, 1, [1, 0, 0, 1, 0, 1, 1, 0]),
    "all_insulator": ((2, 2, 1), 2, 2, [0, 0, 0, 0]),
    "all_conductor": ((2, 1, 2), 2, 2, [3, 3, 3, 3]),
    "single_insulator": ((1, 1, 1), 3, 2, [0]),
    "two_subdomains": ((2, 1, 1), 3, 2, [1, 0]),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    P, n, p, sig = CASES[request.param]
    prob = tiny(P, n, p, sig)
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    return request.param, prob, g, sysm, topo


def test_kernel_dimension_and_tree_size(case):
    name, prob, g, sysm, topo = case
    nonD = np.setdiff1d(np.arange(g.n_edges), topo.dirichlet)
    Wd = sysm.W(prob.dt).toarray()[np.ix_(nonD, nonD)]
    ev = np.linalg.eigvalsh(Wd)
    nzero = int(np.sum(ev < 1e-10 * ev.max()))
    assert nzero == topo.n_plain + topo.n_floating
    assert len(topo.tree_I) == topo.n_plain + topo.n_floating == topo.n_vertices_H - 1
    assert len(topo.kept) == len(nonD) - len(topo.tree_I)
    Wg, _ = solve.gauged_matrix(sysm, topo, prob.dt)
    sla.cholesky(Wg.toarray())  # raises if not SPD


def _ungauged_minnorm(prob, sysm, topo, steps):
    nonD = np.setdiff1d(np.arange(sysm.grid.n_edges), topo.dirichlet)
    Wd = sysm.W(prob.dt).toarray()[np.ix_(nonD, nonD)]
    Wp = np.linalg.pinv(Wd, rcond=1e-11)
    a = np.zeros((sysm.grid.n_edges, 1))
    out = []
    for l in range(steps):
        f = sysm.M @ a + prob.dt * sysm.jhat * prob.amp[:, l][None, :]
        a = np.zeros_like(a)
        a[nonD] = Wp @ f[nonD]
        out.append(a.copy())
    return out


def _gauged_solve(prob, sysm, eliminated, steps):
    keep = np.setdiff1d(np.arange(sysm.grid.n_edges), eliminated)
    Wk = sysm.W(prob.dt).toarray()[np.ix_(keep, keep)]
    a = np.zeros((sysm.grid.n_edges, 1))
    out = []
    for l in range(steps):
        f = sysm.M @ a + prob.dt * sysm.jhat * prob.amp[:, l][None, :]
        a = np.zeros_like(a)
        a[keep] = np.linalg.solve(Wk, f[keep])
        out.append(a.copy())
    return out


def test_gauge_validity(case):
    name, prob, g, sysm, topo = case
    ref = _ungauged_minnorm(prob, sysm, topo, prob.n_steps)
    run = solve.run(prob)
    Cm = G.incidence_C(g).astype(float)
    for a_ref, a in zip(ref, run.fields):
        scale = np.abs(Cm @ a_ref).max() + 1e-300
        assert np.abs(Cm @ (a - a_ref)).max() <= 1e-9 * scale
        cc = topo.cond_closure
        if cc.any():
            assert np.abs(a[cc] - a_ref[cc]).max() <= 1e-9 * (np.abs(a_ref[cc]).max() + 1e-300)
    # the implicit Euler recursion against dense solves of the gauged system
    dense = _gauged_solve(prob, sysm, np.union1d(topo.dirichlet, topo.tree_I), prob.n_steps)
    for a_d, a in zip(dense, run.fields):
        assert np.abs(a - a_d).max() <= 1e-10 * np.abs(a_d).max()


def test_over_elimination_is_detected():
    """Planted mistake: eliminating one more insulator edge than the tree
    closes a cycle and changes the flux, which the validity pin sees."""
    P, n, p, sig = CASES["cond_bottom"]
    prob = tiny(P, n, p, sig)
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    ref = _ungauged_minnorm(prob, sysm, topo, 1)[0]
    cand = np.setdiff1d(np.nonzero(~topo.cond_closure)[0], np.union1d(topo.dirichlet, topo.tree_I))
    Cm = G.incidence_C(g).astype(float)
    worst = 0.0
    for extra in cand[:40]:
        bad = _gauged_solve(prob, sysm, np.union1d(np.union1d(topo.dirichlet, topo.tree_I), [extra]), 1)[0]
        worst = max(worst, np.abs(Cm @ (bad - ref)).max() / np.abs(Cm @ ref).max())
    assert worst > 1e-3


def test_local_blocks_spd(case):
    name, prob, g, sysm, topo = case
    for s, pm in enumerate(sysm.patches):
        loc = topo.local[s]
        pos = {int(e): k for k, e in enumerate(pm.gid)}
        r = [pos[int(e)] for c in "ib" for e in loc[c]]
        # every local edge is in exactly one class
        allc = np.concatenate([loc[c] for c in "ibpe"])
        assert len(allc) == len(pm.gid) and len(np.unique(allc)) == len(pm.gid)
        if not r:
            continue
        Wl = (pm.M + prob.dt * pm.K).toarray()[np.ix_(r, r)]
        sla.cholesky(Wl)
    # the assembled coarse (primal) Schur complement is SPD
    fe = DenseFETI(prob, sysm, topo)
    if fe.nP:
        sla.cholesky(fe.SPi)


def test_two_subdomain_reduction():
    """Conductor x<0.5, insulator x>0.5 as in the paper's experiment: all
    primal edges are Gamma-tree edges, none of the eliminated tree lies on
    Gamma, and the Gamma tree spans every face-interior node of Gamma."""
    prob = tiny((2, 1, 1), 3, 3, [1, 0])
    g = G.build_grid(prob)
    topo = gauge.compute_topology(prob, g)
    assert np.array_equal(topo.primal, topo.tree_gamma)
    ecls = g.edge_class(topo.tree_I)
    assert not np.any(ecls == G.WIREBASKET)
    assert not np.any(topo.cond_closure[topo.tree_I])
    my, mz = 3 + 3, 3 + 3
    assert len(topo.tree_gamma) == (my - 2) * (mz - 2)


@pytest.mark.parametrize("name", ["cond_bottom_p2", "floating_p2", "checker", "all_insulator"])
def test_three_field_dense_solve(name):
    P, n, p, sig = CASES[name]
    prob = tiny(P, n, p, sig)
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    ref = solve.run(prob)
    fe = DenseFETI(prob, sysm, topo)
    dt = prob.dt
    # assemble the full three-field system densely: [a_r^(s) ..., p, lambda]
    sizes = [len(d["i"]) + len(d["b"]) for d in fe.pat]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    nR = offs[-1]
    n = nR + fe.nP + fe.nL
    a = np.zeros(g.n_edges)
    for l in range(prob.n_steps):
        A = np.zeros((n, n))
        rhs = np.zeros(n)
        for s, d in enumerate(fe.pat):
            r = np.concatenate([d["i"], d["b"]])
            o = offs[s]
            nr = len(r)
            Wl = d["W"]
            A[o:o + nr, o:o + nr] = Wl[np.ix_(r, r)]
            Wrp = Wl[np.ix_(r, d["p"])]
            Wpp = Wl[np.ix_(d["p"], d["p"])]
            for k, col in enumerate(d["N"]):
                A[o:o + nr, nR + col] += Wrp[:, k]
                A[nR + col, o:o + nr] += Wrp[:, k]
                for k2, col2 in enumerate(d["N"]):
                    A[nR + col, nR + col2] += Wpp[k, k2]
            Bh = np.zeros((fe.nL, nr))
            Bh[:, len(d["i"]):] = dt * d["B"]
            A[nR + fe.nP:, o:o + nr] = Bh
            A[o:o + nr, nR + fe.nP:] = Bh.T
            f = d["M"] @ a[d["gid"]] + dt * prob.amp[0, l] * d["jhat"][:, 0]
            rhs[o:o + nr] = f[r]
            np.add.at(rhs, nR + d["N"], f[d["p"]])
        x = np.linalg.solve(A, rhs)
        new = np.zeros(g.n_edges)
        seen = np.zeros(g.n_edges, bool)
        for s, d in enumerate(fe.pat):
            r = np.concatenate([d["i"], d["b"]])
            loc = x[offs[s]:offs[s] + len(r)]
            gids = d["gid"][r]
            prev = seen[gids]
            if prev.any():  # interface copies agree (zero jump)
                assert np.abs(new[gids[prev]] - loc[prev]).max() <= 1e-10 * np.abs(loc).max()
            new[gids] = loc
            seen[gids] = True
            new[d["gid"][d["p"]]] = x[nR + d["N"]]
        a = new
        aref = ref.fields[l][:, 0]
        assert np.abs(a - aref).max() <= 1e-10 * np.abs(aref).max()
        # the reduced dual-primal solve (Schur complements + PCG) agrees too
        if l == 0:
            a_fe, it, dvec, lam = fe.step(np.zeros(g.n_edges), prob.amp[0, 0])
            assert np.abs(a_fe - aref).max() <= 1e-9 * np.abs(aref).max()
