"""One-dimensional spline spaces of one patch direction (oracle).

Sec. 2.2 discretises with the spline edge elements of the IGA framework it
cites: per direction an H1 B-spline space of degree p on an open knot vector,
and, along the edge direction, the derivative space of degree p-1.  The edge
basis here is the D-spline (Curry-Schoenberg) normalisation

    D_e = p / (xi_{e+p+1} - xi_{e+1}) * N_{e+1, p-1},   e = 0 .. m-2,

for which d/dx N_e = D_{e-1} - D_e (with D_{-1} = D_{m-1} = 0), so that the
discrete gradient is the signed node-edge incidence of the control grid.
"""
from __future__ import annotations

import numpy as np


def open_knots(a: float, b: float, n: int, p: int) -> np.ndarray:
    """Open uniform knot vector on [a, b] with n elements and degree p."""
    inner = np.linspace(a, b, n + 1)
    return np.concatenate([np.full(p, a), inner, np.full(p, b)])


def bsplines(knots: np.ndarray, p: int, x) -> np.ndarray:
    """All B-splines N_{i,p}(x) by the Cox-de Boor recursion.

    Returns shape (len(x), len(knots) - p - 1).  Degree-0 functions are
    indicators of [t_i, t_{i+1}); the last non-empty span is closed at the
    right end so that the basis sums to one on the whole closed interval.
    Terms with a zero denominator are dropped (the 0/0 = 0 convention).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = np.asarray(knots, dtype=np.float64)
    n0 = len(t) - 1
    N = np.zeros((len(x), n0))
    spans = [i for i in range(n0) if t[i] < t[i + 1]]
    for i in spans:
        N[:, i] = ((x >= t[i]) & (x < t[i + 1])).astype(np.float64)
    last = spans[-1]
    N[x == t[last + 1], last] = 1.0
    for q in range(1, p + 1):
        M = np.zeros((len(x), n0 - q))
        for i in range(n0 - q):
            d1 = t[i + q] - t[i]
            d2 = t[i + q + 1] - t[i + 1]
            acc = np.zeros(len(x))
            if d1 > 0:
                acc += (x - t[i]) / d1 * N[:, i]
            if d2 > 0:
                acc += (t[i + q + 1] - x) / d2 * N[:, i + 1]
            M[:, i] = acc
        N = M
    return N


def bspline_derivs(knots: np.ndarray, p: int, x) -> np.ndarray:
    """First derivatives N'_{i,p}(x) from the textbook formula

    N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}.
    """
    t = np.asarray(knots, dtype=np.float64)
    m = len(t) - p - 1
    Nl = bsplines(t, p - 1, x)  # m + 1 functions of degree p-1
    out = np.zeros((Nl.shape[0], m))
    for i in range(m):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0:
            out[:, i] += p / d1 * Nl[:, i]
        if d2 > 0:
            out[:, i] -= p / d2 * Nl[:, i + 1]
    return out


def dsplines(knots: np.ndarray, p: int, x) -> np.ndarray:
    """Edge-direction basis D_e(x), e = 0 .. m-2 (shape (len(x), m-1))."""
    t = np.asarray(knots, dtype=np.float64)
    m = len(t) - p - 1
    Nl = bsplines(t, p - 1, x)
    out = np.zeros((Nl.shape[0], m - 1))
    for e in range(m - 1):
        out[:, e] = p / (t[e + p + 1] - t[e + 1]) * Nl[:, e + 1]
    return out


def gauss_rule(nq: int):
    """Gauss-Legendre nodes and weights on [-1, 1]."""
    return np.polynomial.legendre.leggauss(nq)


def element_points(a: float, b: float, n: int, nq: int):
    """Physical Gauss points/weights per element of a uniform row on [a, b].

    Returns (x, w), both shape (n, nq): element e spans
    [a + e h, a + (e+1) h] with h = (b - a)/n.
    """
    g, w = gauss_rule(nq)
    h = (b - a) / n
    lo = a + h * np.arange(n)
    x = lo[:, None] + 0.5 * h * (g[None, :] + 1.0)
    ww = np.broadcast_to(0.5 * h * w[None, :], x.shape).copy()
    return x, ww
