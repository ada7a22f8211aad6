"""Residual of one implicit Euler step against the oracle's own operator,
patch by patch (oracle; test infrastructure).

Where the direct solve of the gauged global system does not fit one CPU, a
field computed elsewhere can still be checked against the oracle's
discretisation: the implicit Euler system of Sec. 2.2,

    W a^(l+1) = M a^(l) + dt g(t_{l+1}) jhat,   W = M + dt K,

restricted to the kept edges K of the split of Sec. 3, is satisfied by the
exact discrete field, so ||f_K - (W a)_K|| / ||f_K|| measures how far a
field is from it.  The global matrices are sums of the patch matrices
through each patch's local-to-global edge map, so W a is the sum over
patches of the local products; nothing global is assembled.

The patch matrices are those of ``assemble.assemble_patch``.  Two patches
whose spline rows have the same element count, degree and length in every
direction, and the same sigma and nu, have identical local matrices: their
bases are translates of each other and the Galerkin integrals do not
change under translation.  Each distinct shape is therefore assembled
once (``tests/test_oracle_residual.py`` pins this against patch-by-patch
assembly).  The loads depend on the position and are computed per patch.

Test infrastructure: only ``tests/``, the smoke check and the CPU baseline
of the benchmark use anything under ``oracle/``.
"""
from __future__ import annotations

import numpy as np

from .assemble import assemble_patch, assemble_patch_load, assemble_patch_vec_load, patch_rows
from .grid import build_grid


def shape_key(prob, s):
    """Identity of patch s's local matrices: per direction (length, n, p), sigma, nu."""
    rows = patch_rows(prob, s)
    geo = tuple((round(b[1] - b[0], 15), n, p) for (b, n, p) in rows)
    return geo, float(prob.sigma[s]), float(prob.nu[s])


class _NoLoad:
    """The problem seen without sources (matrices only)."""

    def __init__(self, prob):
        self._p = prob
        self.src_mask = np.zeros(prob.n_patches, np.uint8)
        self.phi = None
        self.jvol = None
        self.ainit = None

    def __getattr__(self, name):
        return getattr(self._p, name)


def local_operator(prob, s, grid=None):
    """Patch s's local (M, K), without its loads."""
    pm = assemble_patch(_NoLoad(prob), grid or build_grid(prob), s)
    return pm.M.tocsr(), pm.K.tocsr()


def shape_representatives(prob):
    """The key of every patch, and the first patch of each distinct key."""
    keys = [shape_key(prob, s) for s in range(prob.n_patches)]
    reps = {}
    for s, k in enumerate(keys):
        reps.setdefault(k, s)
    return keys, reps


def local_operators(prob, grid=None):
    """{shape key: (M_local, K_local)} and the key of every patch."""
    grid = grid or build_grid(prob)
    keys, reps = shape_representatives(prob)
    return {k: local_operator(prob, s, grid) for k, s in reps.items()}, keys


def patch_load(prob, s, ks):
    """Source load of patch s for the excitations ks, (n_local, len(ks))."""
    rows = patch_rows(prob, s)
    m = tuple(n + p for (_, n, p) in rows)
    nloc = (m[0] - 1) * m[1] * m[2] + m[0] * (m[1] - 1) * m[2] + m[0] * m[1] * (m[2] - 1)
    out = np.zeros((nloc, len(ks)))
    if not prob.src_mask[s]:
        return out

    class _Sub:
        """The problem restricted to the excitations ks (in that order)."""
        n_rhs = len(ks)
        breaks, nel, deg = prob.breaks, prob.nel, prob.deg

        @staticmethod
        def patch_ijk(t):
            return prob.patch_ijk(t)

        @staticmethod
        def phi(x, y, z, k):
            return prob.phi(x, y, z, ks[k])

    if prob.phi is not None:
        out += assemble_patch_load(_Sub, s, m)
    if getattr(prob, "jvol", None) is not None:
        fn = prob.jvol
        out += assemble_patch_vec_load(_Sub, s, m, lambda t, x, y, z, k: fn(t, x, y, z, ks[k]))
    return out


def step_residual(prob, grid, kept, ops, keys, loads, a_prev, a_new, g):
    """||f_K - (W a_new)_K|| / ||f_K|| for one excitation, with
    f = M a_prev + dt g jhat.  loads[s] is patch s's load column (n_local,);
    a_prev, a_new are global edge vectors."""
    nE = grid.n_edges
    Wa = np.zeros(nE)
    f = np.zeros(nE)
    for s in range(prob.n_patches):
        gid = grid.local_edges(s)[0]
        M, K = ops[keys[s]]
        Wa_s = M @ a_new[gid] + prob.dt * (K @ a_new[gid])
        np.add.at(Wa, gid, Wa_s)
        np.add.at(f, gid, M @ a_prev[gid] + prob.dt * g * loads[s])
    r = f[kept] - Wa[kept]
    return float(np.linalg.norm(r) / np.linalg.norm(f[kept]))
