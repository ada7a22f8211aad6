"""Pins of the oracle's 1-D spline spaces against closed forms and SciPy."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import spline


@pytest.mark.parametrize("p,n", [(1, 3), (2, 4), (3, 5), (3, 12), (2, 1)])
def test_partition_of_unity_and_scipy(p, n):
    t = spline.open_knots(0.25, 1.75, n, p)
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(0.25, 1.75, 200), [0.25, 1.75]])
    N = spline.bsplines(t, p, x)
    assert N.shape[1] == n + p
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-14)
    xi = x[x < 1.75]
    for i in range(n + p):
        ref = BSpline.basis_element(t[i:i + p + 2], extrapolate=False)(xi)
        ref = np.nan_to_num(ref)
        assert np.allclose(N[x < 1.75, i], ref, atol=1e-13)


@pytest.mark.parametrize("p,n", [(1, 3), (2, 4), (3, 6)])
def test_derivative_against_finite_differences(p, n):
    t = spline.open_knots(0.0, 1.0, n, p)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.01, 0.99, 100)
    # keep away from knots so the central difference does not straddle a kink
    h = 1e-6
    ok = np.min(np.abs(x[:, None] - t[None, :]), axis=1) > 10 * h
    x = x[ok]
    dN = spline.bspline_derivs(t, p, x)
    fd = (spline.bsplines(t, p, x + h) - spline.bsplines(t, p, x - h)) / (2 * h)
    assert np.allclose(dN, fd, atol=1e-6 * n)


@pytest.mark.parametrize("p,n", [(1, 3), (2, 4), (3, 6), (3, 12)])
def test_dspline_identities(p, n):
    t = spline.open_knots(-1.0, 2.0, n, p)
    m = n + p
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.0, 2.0, 150)
    D = spline.dsplines(t, p, x)
    assert D.shape[1] == m - 1
    dN = spline.bspline_derivs(t, p, x)
    Dpad = np.concatenate([np.zeros((len(x), 1)), D, np.zeros((len(x), 1))], axis=1)
    # d/dx N_e = D_{e-1} - D_e
    assert np.allclose(dN, Dpad[:, :-1] - Dpad[:, 1:], atol=1e-12)
    # unit integral of every D-spline (exact Gauss rule per element)
    xq, wq = spline.element_points(-1.0, 2.0, n, p + 1)
    Dq = spline.dsplines(t, p, xq.ravel())
    assert np.allclose(wq.ravel() @ Dq, 1.0, atol=1e-13)


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 6])
def test_gauss_rule_exactness(nq):
    g, w = spline.gauss_rule(nq)
    for k in range(2 * nq):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * g ** k) - exact) < 1e-14
