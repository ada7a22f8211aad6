"""Pins of the oracle's discrete spaces and assembled matrices.

* the space dimension printed in the paper (Sec. 4);
* discrete de Rham exactness: curl o grad = 0 exactly in integers, the
  stiffness annihilates gradients, the mass does so only off conductors;
* closed-form energies: for linear fields A_i, a_i^T K a_j equals
  sum_s nu_s vol_s curl A_i . curl A_j and a_i^T M a_j equals
  sum_s sigma_s int A_i . A_j (polynomials integrated exactly here);
* the curl-form load: jhat^T a_i = int_src phi (curl A_i)_z, and
  jhat annihilates discrete gradients.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import assemble, grid as G, spline

HERE = os.path.dirname(__file__)


def _custom(P, nel, deg, sigma, src=None, phi=None, ext=(1.0, 1.0, 1.0), breaks=None):
    npatch = P[0] * P[1] * P[2]
    sigma = np.asarray(sigma, float)
    return W.Problem(
        name="custom", np=tuple(P),
        breaks=breaks if breaks is not None else [np.linspace(0, ext[d], P[d] + 1) for d in range(3)],
        nel=[np.asarray(v, np.int32) for v in nel], deg=[np.asarray(v, np.int32) for v in deg],
        sigma=sigma, nu=np.linspace(1.0, 3.0, npatch),
        src_mask=(np.ones(npatch, np.uint8) if src is None else np.asarray(src, np.uint8)),
        phi=phi or (lambda x, y, z, k: np.ones((len(x), len(y), len(z)))),
        amp=np.ones((1, 1)), dt=1e-3, n_steps=1)


def test_paper_space_dimension():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_space_dimension.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        Px, Py, Pz, p, n, dofs = map(int, r)
        prob = _custom((Px, Py, Pz), [[n] * Px, [n] * Py, [n] * Pz], [[p] * Px, [p] * Py, [p] * Pz],
                       np.zeros(Px * Py * Pz), breaks=[np.linspace(0, 1, Px + 1),
                                                        np.linspace(0, 1, Py + 1),
                                                        np.linspace(0, 1, Pz + 1)])
        g = G.build_grid(prob)
        total = sum(len(g.local_edges(s)[0]) for s in range(prob.n_patches))
        assert total == dofs


UNEVEN = dict(P=(2, 3, 2), nel=[[2, 3], [1, 2, 2], [3, 1]], deg=[[1, 2], [2, 3, 1], [2, 2]])


@pytest.fixture(scope="module")
def uneven_sys():
    sig = np.array([0, 2.0, 0, 0, 5.0, 0, 1.5, 0, 0, 0, 3.0, 0])
    phi = lambda x, y, z, k: ((1 + x)[:, None, None] * (y ** 2)[None, :, None]
                              * (2 - z)[None, None, :])
    prob = _custom(UNEVEN["P"], UNEVEN["nel"], UNEVEN["deg"], sig, src=(sig == 0), phi=phi,
                   breaks=[np.array([0.0, 0.4, 1.0]), np.array([-1.0, 0.0, 0.5, 1.5]),
                           np.array([0.0, 0.3, 0.7])])
    g = G.build_grid(prob)
    sys = assemble.assemble_global(prob, g)
    return prob, g, sys


def test_curl_grad_exact_and_stiffness_kernel(uneven_sys):
    prob, g, sys = uneven_sys
    Gm = G.incidence_G(g)
    Cm = G.incidence_C(g)
    CG = (Cm @ Gm).tocoo()
    assert CG.nnz == 0 or np.all(CG.data == 0)
    KG = (sys.K @ Gm.astype(float)).toarray()
    assert np.abs(KG).max() <= 1e-13 * np.abs(sys.K.toarray()).max()
    MG = np.abs((sys.M @ Gm.astype(float)).toarray()).max(axis=1)
    # mass acts only on edges inside conductor closures
    cond = np.zeros(g.n_edges, bool)
    for s in range(prob.n_patches):
        if prob.sigma[s] > 0:
            cond[g.local_edges(s)[0]] = True
    assert np.all(MG[~cond] == 0)
    assert np.all(MG[cond] > 0)


def _greville_nodes(prob, g):
    """Greville abscissae of every global node, per direction."""
    out = []
    for d in range(3):
        xs = []
        for r in range(g.P[d]):
            p = int(prob.deg[d][r])
            t = spline.open_knots(prob.breaks[d][r], prob.breaks[d][r + 1], int(prob.nel[d][r]), p)
            gr = np.array([t[i + 1:i + p + 1].mean() for i in range(len(t) - p - 1)])
            xs.append(gr if r == 0 else gr[1:])
        out.append(np.concatenate(xs))
    return out


# linear fields whose component along e_d does not vary along d, so that the
# edge coefficient A(mid) . (head - tail) between Greville points is exact
FIELDS = [
    (lambda x, y, z: (-y / 2, x / 2, 0 * x), (0, 0, 1)),
    (lambda x, y, z: (0 * x, -z / 2, y / 2), (1, 0, 0)),
    (lambda x, y, z: (z / 2, 0 * x, -x / 2), (0, 1, 0)),
    (lambda x, y, z: (y, 0 * x, 0 * x), (0, 0, -1)),
    (lambda x, y, z: (0 * x, 0 * x, x), (0, -1, 0)),
    (lambda x, y, z: (0 * x, z, 0 * x), (-1, 0, 0)),
    (lambda x, y, z: (1 + 0 * x, 2 + 0 * x, -1 + 0 * x), (0, 0, 0)),
]


def _interp(prob, g, f):
    gx, gy, gz = _greville_nodes(prob, g)
    e = np.arange(g.n_edges)
    d, I, J, K = g.edge_decode(e)
    x0, y0, z0 = gx[I], gy[J], gz[K]
    x1 = np.where(d == 0, gx[np.minimum(I + 1, len(gx) - 1)], x0)
    y1 = np.where(d == 1, gy[np.minimum(J + 1, len(gy) - 1)], y0)
    z1 = np.where(d == 2, gz[np.minimum(K + 1, len(gz) - 1)], z0)
    A = f((x0 + x1) / 2, (y0 + y1) / 2, (z0 + z1) / 2)
    return A[0] * (x1 - x0) + A[1] * (y1 - y0) + A[2] * (z1 - z0)


def _box_integral(fun, box):
    """Exact integral of a polynomial of degree <= 5 per direction over a box."""
    g, w = np.polynomial.legendre.leggauss(3)
    pts = [0.5 * (b[1] - b[0]) * (g + 1) + b[0] for b in box]
    ws = [0.5 * (b[1] - b[0]) * w for b in box]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    Wt = ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]
    return float(np.sum(Wt * fun(X, Y, Z)))


def test_closed_form_energies(uneven_sys):
    prob, g, sys = uneven_sys
    V = np.stack([_interp(prob, g, f) for f, _ in FIELDS], axis=1)
    Kg = V.T @ (sys.K @ V)
    Mg = V.T @ (sys.M @ V)
    nF = len(FIELDS)
    Kex = np.zeros((nF, nF))
    Mex = np.zeros((nF, nF))
    for s in range(prob.n_patches):
        i, j, k = prob.patch_ijk(s)
        box = [(prob.breaks[0][i], prob.breaks[0][i + 1]), (prob.breaks[1][j], prob.breaks[1][j + 1]),
               (prob.breaks[2][k], prob.breaks[2][k + 1])]
        vol = np.prod([b[1] - b[0] for b in box])
        for a in range(nF):
            for b in range(nF):
                Kex[a, b] += prob.nu[s] * vol * np.dot(FIELDS[a][1], FIELDS[b][1])
                if prob.sigma[s] > 0:
                    fa, fb = FIELDS[a][0], FIELDS[b][0]
                    Mex[a, b] += prob.sigma[s] * _box_integral(
                        lambda x, y, z: sum(np.asarray(fa(x, y, z)[c]) * np.asarray(fb(x, y, z)[c])
                                            for c in range(3)), box)
    assert np.allclose(Kg, Kex, rtol=1e-12, atol=1e-12 * np.abs(Kex).max())
    assert np.allclose(Mg, Mex, rtol=1e-12, atol=1e-12 * np.abs(Mex).max())


def test_curl_form_load(uneven_sys):
    prob, g, sys = uneven_sys
    V = np.stack([_interp(prob, g, f) for f, _ in FIELDS], axis=1)
    got = sys.jhat[:, 0] @ V
    exact = np.zeros(len(FIELDS))
    for s in range(prob.n_patches):
        if not prob.src_mask[s]:
            continue
        i, j, k = prob.patch_ijk(s)
        box = [(prob.breaks[0][i], prob.breaks[0][i + 1]), (prob.breaks[1][j], prob.breaks[1][j + 1]),
               (prob.breaks[2][k], prob.breaks[2][k + 1])]
        Iphi = _box_integral(lambda x, y, z: (1 + x) * y ** 2 * (2 - z), box)
        for a, (_, curl) in enumerate(FIELDS):
            exact[a] += Iphi * curl[2]
    assert np.allclose(got, exact, rtol=1e-12, atol=1e-12 * np.abs(exact).max())
    # discrete divergence-free load: jhat^T G = 0
    Gm = G.incidence_G(g).astype(float)
    assert np.abs(Gm.T @ sys.jhat[:, 0]).max() <= 1e-13 * np.abs(sys.jhat).max()


def test_plain_workload_sizes():
    g = G.build_grid(W.plain_fp64())
    assert g.N == (11, 11, 11)
    assert g.n_edges == 3630
