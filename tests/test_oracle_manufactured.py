"""Pins of the oracle's volume source, initial value and error norms, and
of the manufactured problem of Sec. 4.

* Closed forms of the homogenised potential U = b F: curl U and curl curl U
  against central differences.
* Volume-form load: for J = curl(0, 0, phi), with phi a polynomial that
  vanishes on the x and y faces, int J . w_e equals the curl-form load
  int phi (curl w_e)_z for every edge.  Both are exact polynomial integrals
  here, so a wrong component, index or sign shows.
* Initial load: for an initial value that is itself a discrete field with
  coefficients c, int sigma A . w_e equals (M c)_e exactly.
* Error norms: a field the space represents exactly, A = (0, 0, x), gives
  curl A_h = (0, -1, 0) with zero error.
* Sec. 4's convergence statement, eps = O(h^p + 1/n_t), with eps the maximum
  over the time levels of the relative L2 errors:
  - the B and E errors of the oracle fall by about 2^p when h halves (p = 1, 2);
  - the E error falls by about 2 when n_t doubles.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, errors, solve, spline
from oracle import grid as G


def _box_problem(P, nel, deg, sigma, breaks, phi=None, jvol=None, ainit=None):
    npatch = P[0] * P[1] * P[2]
    return W.Problem(
        name="custom", np=tuple(P), breaks=[np.asarray(b, float) for b in breaks],
        nel=[np.asarray(v, np.int32) for v in nel], deg=[np.asarray(v, np.int32) for v in deg],
        sigma=np.asarray(sigma, float), nu=np.linspace(1.0, 2.0, npatch),
        src_mask=np.ones(npatch, np.uint8), phi=phi, amp=np.ones((1, 1)), dt=1e-2, n_steps=1,
        jvol=jvol, ainit=ainit)


LAYOUT = dict(P=(2, 1, 2), nel=[[2, 3], [2], [1, 2]], deg=[[2, 3], [2], [3, 1]],
              breaks=[[0.0, 0.4, 1.0], [0.0, 1.0], [0.0, 0.55, 1.0]])


def test_manufactured_closed_forms():
    rng = np.random.default_rng(5)
    x, y, z = rng.random((3, 32))
    U, cU, ccU = W.manufactured_parts(x, y, z)
    h = 1e-4

    def fd_curl(fn):
        def d(i, j):
            e = np.zeros(3)
            e[j] = h
            return (fn(x + e[0], y + e[1], z + e[2])[:, i]
                    - fn(x - e[0], y - e[1], z - e[2])[:, i]) / (2 * h)
        return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)], 1)

    assert np.abs(fd_curl(lambda a, b, c: W.manufactured_parts(a, b, c)[0]) - cU).max() < 1e-6
    assert np.abs(fd_curl(lambda a, b, c: W.manufactured_parts(a, b, c)[1]) - ccU).max() < 1e-5
    # the paper's field is divergence free and the lifting is exact on the boundary
    on_face = np.stack([np.zeros(8), rng.random(8), rng.random(8)])
    assert np.abs(W.manufactured_parts(*on_face)[0]).max() == 0.0


def test_volume_load_equals_curl_form():
    def phi(xs, ys, zs, k):
        fx = xs ** 2 * (1 - xs) ** 2
        fy = ys ** 2 * (1 - ys) ** 2
        return fx[:, None, None] * fy[None, :, None] * (1 + zs)[None, None, :]

    def jvol(s, xs, ys, zs, k):
        # curl (0, 0, phi) = (d_y phi, -d_x phi, 0)
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        fx, dfx = X ** 2 * (1 - X) ** 2, 2 * X * (1 - X) * (1 - 2 * X)
        fy, dfy = Y ** 2 * (1 - Y) ** 2, 2 * Y * (1 - Y) * (1 - 2 * Y)
        return np.stack([fx * dfy * (1 + Z), -dfx * fy * (1 + Z), np.zeros_like(X)], -1)

    sig = [0.0, 2.0, 1.0, 0.0]
    a = assemble.assemble_global(_box_problem(LAYOUT["P"], LAYOUT["nel"], LAYOUT["deg"], sig,
                                              LAYOUT["breaks"], phi=phi))
    b = assemble.assemble_global(_box_problem(LAYOUT["P"], LAYOUT["nel"], LAYOUT["deg"], sig,
                                              LAYOUT["breaks"], jvol=jvol))
    scale = np.abs(a.jhat).max()
    assert scale > 0
    assert np.abs(a.jhat - b.jhat).max() <= 1e-13 * scale


def _discrete_field_eval(prob, grid, c):
    """Point evaluator of the discrete field with global coefficients c, per patch."""
    def ev(s, xs, ys, zs, k):
        rows = assemble.patch_rows(prob, s)
        ax = []
        for (lo_hi, n, p), pts in zip(rows, (xs, ys, zs)):
            t = spline.open_knots(lo_hi[0], lo_hi[1], n, p)
            ax.append((spline.bsplines(t, p, pts), spline.dsplines(t, p, pts)))
        (Nx, Dx), (Ny, Dy), (Nz, Dz) = ax
        mx, my, mz = grid.patch_m(s)
        loc = c[grid.local_edges(s)[0]]
        nX, nY = (mx - 1) * my * mz, mx * (my - 1) * mz
        t3 = lambda f, g, h, cc: np.einsum("ia,jb,kc,cba->ijk", f, g, h, cc)
        return np.stack([t3(Dx, Ny, Nz, loc[:nX].reshape(mz, my, mx - 1)),
                         t3(Nx, Dy, Nz, loc[nX:nX + nY].reshape(mz, my - 1, mx)),
                         t3(Nx, Ny, Dz, loc[nX + nY:].reshape(mz - 1, my, mx))], -1)
    return ev


def test_initial_load_is_mass_times_coefficients():
    sig = [0.0, 2.0, 1.5, 0.0]
    base = _box_problem(LAYOUT["P"], LAYOUT["nel"], LAYOUT["deg"], sig, LAYOUT["breaks"],
                        phi=lambda x, y, z, k: np.zeros((len(x), len(y), len(z))))
    grid = G.build_grid(base)
    c = np.random.default_rng(2).standard_normal(grid.n_edges)
    base.ainit = _discrete_field_eval(base, grid, c)
    sysm = assemble.assemble_global(base, grid)
    want = sysm.M @ c
    assert np.abs(want).max() > 0
    assert np.abs(sysm.m0[:, 0] - want).max() <= 1e-12 * np.abs(want).max()


def test_errors_zero_for_represented_field():
    sig = [1.0, 0.0, 0.0, 2.0]
    prob = _box_problem(LAYOUT["P"], LAYOUT["nel"], LAYOUT["deg"], sig, LAYOUT["breaks"],
                        phi=lambda x, y, z, k: np.zeros((len(x), len(y), len(z))))
    grid = G.build_grid(prob)
    # A = (0, 0, x): z-edge coefficient = Greville abscissa of its x node times
    # the unit-integral D-spline's support length / p along z
    a = np.zeros(grid.n_edges)
    for s in range(prob.n_patches):
        rows = assemble.patch_rows(prob, s)
        (bx, nx, px), _, (bz, nz, pz) = rows
        tx = spline.open_knots(bx[0], bx[1], nx, px)
        tz = spline.open_knots(bz[0], bz[1], nz, pz)
        gx = np.array([tx[i + 1:i + px + 1].mean() for i in range(nx + px)])
        lz = np.array([(tz[c + pz + 1] - tz[c + 1]) / pz for c in range(nz + pz - 1)])
        gid, d, ia, ib, ic = grid.local_edges(s)
        zsel = d == 2
        a[gid[zsel]] = gx[ia[zsel]] * lz[ic[zsel]]
    dt = prob.dt
    e = errors.field_errors(
        prob, a, np.zeros_like(a), 0.0,
        lambda X, Y, Z, t: np.stack([0 * X, -np.ones_like(X), 0 * X], -1),
        lambda X, Y, Z, t: -np.stack([0 * X, 0 * X, X], -1) / dt, grid=grid)
    assert e["eB"] <= 1e-13 and e["eE"] <= 1e-13


def _mms_errors(n, p, n_t):
    """Maximum over the time levels of the relative L2 errors of B and E."""
    prob = W.paper_manufactured(n=n, p=p, n_t=n_t)
    r = solve.run(prob)
    e = errors.step_errors(prob, [f[:, 0] for f in r.fields], prob.extra["B_exact"],
                           prob.extra["E_exact"], grid=r.sys.grid)
    # the last level agrees with the single-level evaluation
    last = errors.field_errors(prob, r.fields[-1][:, 0], r.fields[-2][:, 0], prob.extra["T"],
                               prob.extra["B_exact"], prob.extra["E_exact"], grid=r.sys.grid)
    assert abs(e["eB"][-1] - last["eB"]) <= 1e-12 and abs(e["eE"][-1] - last["eE"]) <= 1e-12
    return {"eB": e["eB_max"], "eE": e["eE_max"]}


@pytest.mark.parametrize("p,ns,lo", [(1, (2, 4, 8), 1.7), (2, (2, 4, 8), 3.5)])
def test_paper_convergence_in_h(p, ns, lo):
    e = [_mms_errors(n, p, 256) for n in ns]
    print(p, e)
    for a, b in zip(e[:-1], e[1:]):
        assert a["eB"] / b["eB"] >= lo and a["eE"] / b["eE"] >= lo, (a, b)


def test_paper_convergence_in_time():
    e = [_mms_errors(4, 3, n_t) for n_t in (4, 8, 16)]
    print(e)
    for a, b in zip(e[:-1], e[1:]):
        assert 1.85 <= a["eE"] / b["eE"] <= 2.3, (a, b)
        assert b["eB"] <= a["eB"]
