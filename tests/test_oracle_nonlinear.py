"""Pins of the nonlinear-reluctivity oracle (oracle/nonlinear.py), each
against something other than the oracle's own formula:
* per-element nu in the assembly: a^T K(nu_e) a equals the sum over
  elements of nu_e times the integral of |curl a|^2, evaluated through the
  field-evaluation route of oracle/errors.py on another quadrature rule;
* the element mean of |B|^2 is exact for a field of constant curl (its L2
  projection onto the spline space is exact);
* a constant curve reduces every step to the linear oracle's;
* the converged iterate is a fixed point: nu re-evaluated from it and the
  step's nonlinear residual vanish to the iteration's tolerance;
* Newton's method: its Jacobian matches central differences of the step
  residual (and fails without the terms of nu's own dependence on a), and
  it reaches the fixed-point iteration's field, superlinearly.
A planted mistake (nu of the wrong element order) fails the energy pin."""
import numpy as np
import pytest

import workloads as W
from oracle import solve
from oracle.assemble import assemble_global, assemble_patch, assemble_patch_vec_load
from oracle.errors import patch_fields
from oracle.grid import build_grid
from oracle.nonlinear import brauer_nu, element_b2, nonlinear_residual, run_picard


def small(n_steps=3, sigma=(1e6, 0.0), n=2, p=2):
    return W.make_uniform((2, 1, 1), n=n, p=p, sigma=np.array(sigma), n_steps=n_steps,
                          name="nl_small")


def _element_energy(prob, grid, s, a):
    """integral of |curl a|^2 per element (nz, ny, nx) through patch_fields."""
    _, _, _, Wq, _, curl = patch_fields(prob, grid, s, a)
    b2 = np.sum(curl * curl, axis=-1) * Wq
    nel = [int(prob.nel[d][prob.patch_ijk(s)[d]]) for d in range(3)]
    q = [b2.shape[d] // nel[d] for d in range(3)]
    e = b2.reshape(nel[0], q[0], nel[1], q[1], nel[2], q[2]).sum(axis=(1, 3, 5))
    return np.transpose(e, (2, 1, 0))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_element_nu_scales_each_element_energy(p):
    prob = small(p=p, n=(3, 2, 2))
    grid = build_grid(prob)
    rng = np.random.default_rng(4 + p)
    a = rng.standard_normal(grid.n_edges)
    for s in range(prob.n_patches):
        nel = [int(prob.nel[d][prob.patch_ijk(s)[d]]) for d in range(3)]
        nu_e = rng.uniform(0.5, 3.0, size=(nel[2], nel[1], nel[0]))
        pm = assemble_patch(prob, grid, s, nu_elem=nu_e)
        al = a[pm.gid]
        lhs = float(al @ (pm.K @ al))
        rhs = float(np.sum(nu_e * _element_energy(prob, grid, s, a)))
        assert abs(lhs - rhs) <= 1e-11 * abs(rhs), (lhs, rhs)
        # a planted mistake: the element values read in (nx, ny, nz) order
        bad = np.ascontiguousarray(np.transpose(nu_e, (2, 1, 0))).reshape(nu_e.shape)
        pmb = assemble_patch(prob, grid, s, nu_elem=bad)
        assert abs(float(al @ (pmb.K @ al)) - rhs) > 1e-6 * abs(rhs)
        # element values equal to the patch's constant give the patch's matrix
        K0 = assemble_patch(prob, grid, s).K
        Kc = assemble_patch(prob, grid, s, nu_elem=np.full(nu_e.shape, prob.nu[s])).K
        assert abs(Kc - K0).max() <= 1e-12 * abs(K0).max()


def test_element_b2_is_exact_for_a_constant_curl():
    """A = (B0/2) (-y, x, 0) has curl (0, 0, B0) and lies in the spline edge
    space (degree 0 along its own direction, 1 across), so its L2 projection
    reproduces it and every element mean of |B|^2 is B0^2."""
    B0 = 0.7
    prob = small(p=2, n=(2, 3, 2), sigma=(1.0, 1.0))
    prob.ainit = None
    grid = build_grid(prob)
    sysm = assemble_global(prob, grid)       # mass with sigma = 1 everywhere
    rhs = np.zeros(grid.n_edges)

    def field(s, xs, ys, zs, k):
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        return np.stack([-0.5 * B0 * Y, 0.5 * B0 * X, 0.0 * Z], axis=-1)

    for s in range(prob.n_patches):
        m = grid.patch_m(s)
        gid = grid.local_edges(s)[0]
        np.add.at(rhs, gid, assemble_patch_vec_load(prob, s, m, field)[:, 0])
    import scipy.sparse.linalg as spla
    c = spla.spsolve(sysm.M.tocsc(), rhs)
    for s in range(prob.n_patches):
        b2 = element_b2(prob, grid, s, c)
        assert np.allclose(b2, B0 * B0, rtol=1e-10, atol=0), (b2.min(), b2.max())


def test_constant_curve_is_the_linear_oracle():
    prob = small(n_steps=3)
    nu0 = float(prob.nu[0])
    ref = solve.run(prob)
    out = run_picard(prob, (0.25 * nu0, 0.0, 0.75 * nu0), [True, True])
    for l in range(prob.n_steps):
        r = ref.fields[l]
        assert np.linalg.norm(out.fields[l] - r) <= 1e-12 * np.linalg.norm(r)
        assert max(out.iterations[l]) <= 2


def test_fixed_point_and_a_real_nonlinearity():
    prob = small(n_steps=3)
    nu0 = float(prob.nu[0])
    lin = solve.run(prob)
    # scale the curve so that k2 |B|^2 reaches about 1 in the conductor
    grid = build_grid(prob)
    b2max = max(float(element_b2(prob, grid, 0, lin.fields[l][:, 0]).max())
                for l in range(prob.n_steps))
    curve = (0.5 * nu0, 1.0 / b2max, 0.5 * nu0)
    out = run_picard(prob, curve, [True, False], tol=1e-13)
    prev = np.zeros_like(out.fields[0])
    for l in range(prob.n_steps):
        a = out.fields[l]
        assert nonlinear_residual(prob, curve, [True, False], a, prev, l) <= 1e-10
        prev = a
    # nu varies over the conductor's elements, and the field moved off the
    # linear one by more than the iteration's tolerance
    nu_last = out.nu[-1][0]
    assert nu_last.max() / nu_last.min() > 1.05
    assert np.linalg.norm(out.fields[-1] - lin.fields[-1]) > 1e-6 * np.linalg.norm(lin.fields[-1])
    assert max(max(it) for it in out.iterations) > 2


def test_brauer_curve_values():
    assert brauer_nu(0.0, 2.0, 3.0, 5.0) == 7.0
    assert np.isclose(brauer_nu(1.0, 2.0, np.log(3.0), 5.0), 11.0)


def _strong_case():
    prob = small(n_steps=3)
    nu0 = float(prob.nu[0])
    lin = solve.run(prob)
    grid = build_grid(prob)
    b2max = max(float(element_b2(prob, grid, 0, lin.fields[l][:, 0]).max())
                for l in range(prob.n_steps))
    return prob, lin, grid, (0.5 * nu0, 3.0 / b2max, 0.5 * nu0), [True, False]


def test_newton_jacobian_matches_central_differences():
    """The step Jacobian (including the rank-one terms of nu's dependence
    on the element mean of |B|^2) against central differences of the step
    residual along a random direction."""
    from oracle.nonlinear import element_data, step_jacobian, step_residual
    prob, lin, grid, curve, nonl = _strong_case()
    sysg = assemble_global(prob, grid)
    ed = [element_data(prob, grid, s) if nonl[s] else None for s in range(prob.n_patches)]
    rng = np.random.default_rng(11)
    x = 1.3 * lin.fields[-1][:, 0]
    f = rng.standard_normal(grid.n_edges)
    v = rng.standard_normal(grid.n_edges)
    Jv = step_jacobian(prob, grid, sysg, x, curve, nonl, ed) @ v
    eps = 1e-6 * np.linalg.norm(x) / np.linalg.norm(v)
    fd = (step_residual(prob, grid, sysg, x + eps * v, f, curve, nonl, ed)
          - step_residual(prob, grid, sysg, x - eps * v, f, curve, nonl, ed)) / (2 * eps)
    assert np.linalg.norm(fd - Jv) <= 1e-5 * np.linalg.norm(Jv)
    # without the rank-one terms (the Picard matrix M + dt K(nu(x))) the
    # check fails: they are not negligible here
    from oracle.nonlinear import _k_nu
    J0 = sysg.M + prob.dt * _k_nu(prob, grid, x, curve, nonl, ed, None)
    assert np.linalg.norm(fd - J0 @ v) > 1e-3 * np.linalg.norm(Jv)


def test_newton_reaches_the_fixed_point_quadratically():
    from oracle.nonlinear import run_newton
    prob, lin, grid, curve, nonl = _strong_case()
    nr = run_newton(prob, curve, nonl, tol=1e-13)
    pr = run_picard(prob, curve, nonl, tol=1e-13)
    for l in range(prob.n_steps):
        ref = pr.fields[l]
        assert np.linalg.norm(nr.fields[l] - ref) <= 1e-10 * np.linalg.norm(ref)
        assert nr.iterations[l][0] <= 8
        # superlinear decrease of the residual once it is small
        r = [x for x in nr.residuals[l] if x > 0]
        for a, b in zip(r, r[1:]):
            if a < 1e-2 and b > 1e-14:
                assert b <= a ** 1.5, (a, b)
    assert sum(max(it) for it in pr.iterations) > sum(max(it) for it in nr.iterations)
