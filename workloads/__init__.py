"""Seeded synthetic problem descriptions (inputs only).

This module builds the problem statements that both the GPU library and the
CPU oracle consume: patch layout, spline rows, materials, source and time
grid.  It holds none of the method's arithmetic -- no basis functions, no
quadrature, no matrices -- only the data a user of the solver would hand in.

Every workload mirrors the paper's experiment structure (Sec. 4: a box split
into axis-aligned hexahedral patches, homogeneous n x A = 0, a smooth
prescribed source, implicit Euler) at the sizes of the benchmark problems.
Random draws use ``numpy.random.default_rng(seed)`` with the seed stated in
each builder.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

MU0 = 4.0e-7 * np.pi
NU0 = 1.0 / MU0
FREQ = 50.0


def _phi_sin2(xs, ys, zs, k):
    """phi(x,y,z) = sin^2(pi x) sin^2(pi y) on a tensor grid, shape (nx,ny,nz)."""
    fx = np.sin(np.pi * np.asarray(xs)) ** 2
    fy = np.sin(np.pi * np.asarray(ys)) ** 2
    return (fx[:, None, None] * fy[None, :, None]) * np.ones(len(zs))[None, None, :]


@dataclass
class Problem:
    """A multi-patch eddy-current problem on an axis-aligned box.

    Patch (i, j, k) spans [bx[i], bx[i+1]] x [by[j], by[j+1]] x [bz[k], bz[k+1]]
    and has id s = i + P0 * (j + P1 * k).  Row r of direction d carries
    ``nel[d][r]`` uniform elements and H1 spline degree ``deg[d][r]``.
    The source is J_k(x, t) = g_k(t) curl(0, 0, phi_k(x)) on patches with
    ``src_mask`` set; ``amp[k, l]`` is g_k(t_{l+1}).  Optionally a volume
    source ``jvol(s, xs, ys, zs, k) -> (nx, ny, nz, 3)`` adds g_k(t) times that
    field on source patches, and ``ainit`` (same signature) gives the initial
    potential A_k(x, 0) (used on conductor patches); ``phi`` may then be None.
    """

    name: str
    np: tuple
    breaks: List[np.ndarray]
    nel: List[np.ndarray]
    deg: List[np.ndarray]
    sigma: np.ndarray
    nu: np.ndarray
    src_mask: np.ndarray
    phi: Callable
    amp: np.ndarray
    dt: float
    n_steps: int
    pcg_rtol: float = 1e-10
    precision: str = "fp64"
    ir_rtol: float = 1e-8
    seed: Optional[int] = None
    note: str = ""
    extra: dict = field(default_factory=dict)
    jvol: Optional[Callable] = None
    ainit: Optional[Callable] = None

    @property
    def n_patches(self) -> int:
        return int(self.np[0] * self.np[1] * self.np[2])

    @property
    def n_rhs(self) -> int:
        return int(self.amp.shape[0])

    def patch_ijk(self, s: int):
        P0, P1, _ = self.np
        return s % P0, (s // P0) % P1, s // (P0 * P1)

    def with_steps(self, n_steps: int) -> "Problem":
        """Same problem, first ``n_steps`` time steps only."""
        q = Problem(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        q.n_steps = int(n_steps)
        q.amp = np.ascontiguousarray(self.amp[:, :n_steps])
        return q


def _sin_amp(dt, n_steps, scale=1.0, n_rhs=1):
    t = dt * np.arange(1, n_steps + 1)
    g = scale * np.sin(2.0 * np.pi * FREQ * t)
    return np.tile(g, (n_rhs, 1)).astype(np.float64)


def _uniform_rows(P, n, p):
    return np.full(P, n, dtype=np.int32), np.full(P, p, dtype=np.int32)


def _box(P, P_lo=0.0, P_hi=1.0):
    return np.linspace(P_lo, P_hi, P + 1)


def make_uniform(np_=(2, 2, 2), n=4, p=2, sigma=None, src_mask=None, dt=1e-4,
                 n_steps=20, name="uniform", extent=(1.0, 1.0, 1.0), phi=None,
                 amp=None, pcg_rtol=1e-10, precision="fp64"):
    P = tuple(int(v) for v in np_)
    nel, deg = [], []
    for d in range(3):
        a, b = _uniform_rows(P[d], n if np.isscalar(n) else n[d], p if np.isscalar(p) else p[d])
        nel.append(a)
        deg.append(b)
    npatch = P[0] * P[1] * P[2]
    if sigma is None:
        sigma = np.zeros(npatch)
    sigma = np.asarray(sigma, dtype=np.float64)
    if src_mask is None:
        src_mask = (sigma == 0).astype(np.uint8)
    return Problem(
        name=name, np=P,
        breaks=[_box(P[d], 0.0, extent[d]) for d in range(3)],
        nel=nel, deg=deg, sigma=sigma, nu=np.full(npatch, NU0),
        src_mask=np.asarray(src_mask, dtype=np.uint8),
        phi=phi if phi is not None else _phi_sin2,
        amp=amp if amp is not None else _sin_amp(dt, n_steps),
        dt=dt, n_steps=n_steps, pcg_rtol=pcg_rtol, precision=precision)


def plain_fp64() -> Problem:
    """Unit cube, 2x2x2 patches, p=2, 4 elements per direction per patch.

    Patches below z=0.5 conduct (sigma=1e6), the others insulate; the source
    sin(2 pi 50 t) curl(0,0,sin^2(pi x) sin^2(pi y)) acts in the insulating
    patches; dt=1e-4, 20 steps, PCG rtol 1e-10.
    """
    P = (2, 2, 2)
    sigma = np.array([1e6 if (s // 4) == 0 else 0.0 for s in range(8)])
    return make_uniform(P, 4, 2, sigma=sigma, dt=1e-4, n_steps=20, name="cube8_p2_n4_fp64")


def uneven_fp64(seed: int = 1, n_steps: int = 50, P=(4, 4, 4)) -> Problem:
    """Unit cube, 4x4x4 patches with seeded per-row element counts and degrees.

    Each row of each direction draws n in {4,6,8,12} and p in {2,3}
    independently (rows keep faces conforming).  Each patch is insulating
    with probability 1/2, else sigma = 10^U(5,7).  Source and dt as the plain
    workload, 50 steps.
    """
    rng = np.random.default_rng(seed)
    nel = [rng.choice([4, 6, 8, 12], size=P[d]).astype(np.int32) for d in range(3)]
    deg = [rng.choice([2, 3], size=P[d]).astype(np.int32) for d in range(3)]
    npatch = P[0] * P[1] * P[2]
    cond = rng.random(npatch) >= 0.5
    sig = np.where(cond, 10.0 ** rng.uniform(5.0, 7.0, size=npatch), 0.0)
    dt = 1e-4
    return Problem(
        name=f"cube64_uneven_seed{seed}_fp64", np=tuple(P),
        breaks=[_box(P[d]) for d in range(3)], nel=nel, deg=deg,
        sigma=sig, nu=np.full(npatch, NU0), src_mask=(sig == 0).astype(np.uint8),
        phi=_phi_sin2, amp=_sin_amp(dt, n_steps), dt=dt, n_steps=n_steps,
        pcg_rtol=1e-10, precision="fp64", seed=seed)


def floating_mixed(n: int = 10, p: int = 3, n_steps: int = 100, precision="fp32_ir") -> Problem:
    """4x4x4 patches, central 2x2x2 block conducting (sigma=5e6, floating).

    p=3 and n=10 elements per direction per patch at full size; dt=5e-5,
    100 steps; local factors in FP32 with FP64 iterative refinement to 1e-8.
    """
    P = (4, 4, 4)
    sig = np.zeros(64)
    for s in range(64):
        i, j, k = s % 4, (s // 4) % 4, s // 16
        if i in (1, 2) and j in (1, 2) and k in (1, 2):
            sig[s] = 5e6
    prob = make_uniform(P, n, p, sigma=sig, dt=5e-5, n_steps=n_steps,
                        name=f"cube64_floating_p{p}_n{n}_{precision}", precision=precision)
    prob.ir_rtol = 1e-8
    return prob


def _phi_modes(coef):
    """phi_k = sum_{a,b=1..3} c[k,a,b] sin(a pi x/2) sin(b pi y/2) (1 + cos(pi z)/2)."""
    def phi(xs, ys, zs, k):
        xs, ys, zs = np.asarray(xs), np.asarray(ys), np.asarray(zs)
        sx = np.stack([np.sin(a * np.pi * xs / 2.0) for a in (1, 2, 3)])  # (3, nx)
        sy = np.stack([np.sin(b * np.pi * ys / 2.0) for b in (1, 2, 3)])
        fxy = np.einsum("ab,ax,by->xy", coef[k], sx, sy)
        fz = 1.0 + 0.5 * np.cos(np.pi * zs)
        return fxy[:, :, None] * fz[None, None, :]
    return phi


def largest_multirhs(P=(8, 8, 4), n: int = 12, p: int = 3, n_rhs: int = 32,
                     n_steps: int = 200, seed: int = 4, precision="fp32_ir") -> Problem:
    """[0,2]x[0,2]x[0,1], 8x8x4 patches of 0.25^3, checkerboard sigma=1e6.

    Conductors where (i+j+k) is even.  32 excitations share the operator:
    phi_k from seeded N(0,1) mode coefficients, g_k(t) = sin(2 pi 50 t),
    source on every patch; dt=1e-4, 200 steps.
    """
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((n_rhs, 3, 3))
    npatch = P[0] * P[1] * P[2]
    sig = np.zeros(npatch)
    for s in range(npatch):
        i, j, k = s % P[0], (s // P[0]) % P[1], s // (P[0] * P[1])
        if (i + j + k) % 2 == 0:
            sig[s] = 1e6
    ext = (P[0] * 0.25, P[1] * 0.25, P[2] * 0.25)
    dt = 1e-4
    prob = make_uniform(P, n, p, sigma=sig, src_mask=np.ones(npatch, np.uint8), dt=dt,
                        n_steps=n_steps, name=f"box{P[0]}x{P[1]}x{P[2]}_p{p}_n{n}_rhs{n_rhs}",
                        extent=ext, phi=_phi_modes(coef), amp=_sin_amp(dt, n_steps, n_rhs=n_rhs),
                        precision=precision)
    prob.seed = seed
    return prob


def serving_requests(n_req: int = 256, seed: int = 3, n_steps: int = 50,
                     ks=(2, 3, 4), nrange=(4, 10)) -> List[Problem]:
    """Independent requests on the unit cube split into k x k x k patches.

    Per request: k in {2,3,4}, per-row n uniform in {4..10}, one p in {2,3},
    per-patch sigma 0 (prob 1/2) or 10^U(5,7), source amplitude U[0.5,2]
    times sin(2 pi 50 t) on every patch, dt=1e-4, 50 steps.
    """
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        k = int(rng.choice(ks))
        p = int(rng.choice([2, 3]))
        P = (k, k, k)
        nel = [rng.integers(nrange[0], nrange[1] + 1, size=k).astype(np.int32) for _ in range(3)]
        deg = [np.full(k, p, dtype=np.int32) for _ in range(3)]
        npatch = k ** 3
        cond = rng.random(npatch) >= 0.5
        sig = np.where(cond, 10.0 ** rng.uniform(5.0, 7.0, size=npatch), 0.0)
        scale = float(rng.uniform(0.5, 2.0))
        dt = 1e-4
        out.append(Problem(
            name=f"req{r}_k{k}_p{p}", np=P, breaks=[_box(k) for _ in range(3)],
            nel=nel, deg=deg, sigma=sig, nu=np.full(npatch, NU0),
            src_mask=np.ones(npatch, np.uint8), phi=_phi_sin2,
            amp=_sin_amp(dt, n_steps, scale=scale), dt=dt, n_steps=n_steps,
            pcg_rtol=1e-10, precision="fp32_ir", seed=seed))
    return out


def poisson_arrivals(n_req: int, rate: float, seed: int = 33) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n_req))


def subproblem(prob: Problem, lo=(0, 0, 0), P=(2, 2, 2)) -> Problem:
    """The same problem restricted to the block of P patch rows starting at
    lo in each direction (same rows, materials, source and time grid)."""
    lo = tuple(int(v) for v in lo)
    P = tuple(min(int(P[d]), int(prob.np[d]) - lo[d]) for d in range(3))
    ids = []
    for k in range(P[2]):
        for j in range(P[1]):
            for i in range(P[0]):
                ids.append((lo[0] + i) + prob.np[0] * ((lo[1] + j) + prob.np[1] * (lo[2] + k)))
    ids = np.array(ids)
    q = Problem(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
    q.name = f"{prob.name}_sub{P[0]}x{P[1]}x{P[2]}"
    q.np = P
    q.breaks = [np.asarray(prob.breaks[d][lo[d]:lo[d] + P[d] + 1]) for d in range(3)]
    q.nel = [np.asarray(prob.nel[d][lo[d]:lo[d] + P[d]]) for d in range(3)]
    q.deg = [np.asarray(prob.deg[d][lo[d]:lo[d] + P[d]]) for d in range(3)]
    q.sigma = np.asarray(prob.sigma)[ids]
    q.nu = np.asarray(prob.nu)[ids]
    q.src_mask = np.asarray(prob.src_mask)[ids]
    return q


# ---------------------------------------------------------------------------
# The paper's manufactured solution (Sec. 4), homogenised by a lifting
# ---------------------------------------------------------------------------
def _trig(x, y, z):
    return np.sin(x), np.cos(x), np.sin(y), np.cos(y), np.sin(z), np.cos(z)


def _paper_field(x, y, z):
    """The spatial factor F(x) of the Sec. 4 solution A = e^{-t} F, and its
    Jacobian dF_i/dx_j; F = (sin x cos y cos z, -2 cos x sin y cos z,
    cos x cos y sin z) is divergence-free and -Laplace(F) = 3 F."""
    sx, cx, sy, cy, sz, cz = _trig(x, y, z)
    F = np.stack([sx * cy * cz, -2.0 * cx * sy * cz, cx * cy * sz], axis=-1)
    J = np.stack([
        np.stack([cx * cy * cz, -sx * sy * cz, -sx * cy * sz], axis=-1),
        np.stack([2.0 * sx * sy * cz, -2.0 * cx * cy * cz, 2.0 * cx * sy * sz], axis=-1),
        np.stack([-sx * cy * sz, -cx * sy * sz, cx * cy * cz], axis=-1)], axis=-2)
    return F, J


def _bubble(x, y, z):
    """b = 64 x(1-x) y(1-y) z(1-z) with its gradient and Hessian."""
    X, Y, Z = 4 * x * (1 - x), 4 * y * (1 - y), 4 * z * (1 - z)
    dX, dY, dZ = 4 * (1 - 2 * x), 4 * (1 - 2 * y), 4 * (1 - 2 * z)
    d2 = -8.0
    b = X * Y * Z
    g = np.stack([dX * Y * Z, X * dY * Z, X * Y * dZ], axis=-1)
    H = np.stack([
        np.stack([d2 * Y * Z, dX * dY * Z, dX * Y * dZ], axis=-1),
        np.stack([dX * dY * Z, X * d2 * Z, X * dY * dZ], axis=-1),
        np.stack([dX * Y * dZ, X * dY * dZ, X * Y * d2], axis=-1)], axis=-2)
    return b, g, H


def manufactured_parts(x, y, z):
    """U = b F (the homogenised potential's spatial factor), curl U and
    curl curl U at points (broadcast arrays); returns three (..., 3) arrays.

    curl(b F) = b curl F + grad b x F with curl F = (-3 cx sy sz, 0, 3 sx sy cz);
    curl curl U = grad div U - Laplace U, div U = grad b . F, and
    Laplace U_i = Laplace(b) F_i + 2 grad b . grad F_i - 3 b F_i.
    """
    x, y, z = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float), np.asarray(z, float))
    F, JF = _paper_field(x, y, z)
    b, g, H = _bubble(x, y, z)
    sx, cx, sy, cy, sz, cz = _trig(x, y, z)
    curlF = np.stack([-3.0 * cx * sy * sz, np.zeros_like(x), 3.0 * sx * sy * cz], axis=-1)
    U = b[..., None] * F
    curlU = b[..., None] * curlF + np.cross(g, F)
    lap_b = H[..., 0, 0] + H[..., 1, 1] + H[..., 2, 2]
    grad_div = np.einsum("...ij,...j->...i", H, F) + np.einsum("...j,...ji->...i", g, JF)
    lap_U = lap_b[..., None] * F + 2.0 * np.einsum("...j,...ij->...i", g, JF) - 3.0 * b[..., None] * F
    return U, curlU, grad_div - lap_U


def paper_manufactured(n: int = 4, p: int = 2, n_t: int = 32, T: float = 1.0,
                       precision: str = "fp64", pcg_rtol: float = 1e-10) -> Problem:
    """The Sec. 4 experiment: (0,1)^3 cut at x = 0.5 into a conductor (x < 0.5,
    sigma = 1) and an insulator (nu = 1 everywhere), exact potential
    A = e^{-t} F(x), t in (0, T), n_t implicit Euler steps.

    A has nonzero tangential trace on the boundary.  It is homogenised with
    the lifting L = e^{-t} (1 - b) F, b = 64 x(1-x) y(1-y) z(1-z), which
    carries the boundary data exactly: the unknown U = A - L = e^{-t} b F has
    n x U = 0, source J = sigma dU/dt + curl nu curl U = e^{-t} (-sigma b F +
    nu curl curl(b F)) in every patch, and initial value b F.  Because L is
    known exactly, A_h - A = U_h - U: errors of U_h are errors of A_h.
    ``n`` elements per direction per patch and H1 degree ``p`` (h = 1/n in
    the patch parameter, as the paper counts it); g(t) = e^{-t}.
    ``extra`` holds the closed forms B = curl U and E = -dU/dt for the errors.
    """
    P = (2, 1, 1)
    sig = np.array([1.0, 0.0])
    nu = np.array([1.0, 1.0])
    dt = T / n_t

    def jvol(s, xs, ys, zs, k):
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        U, _, ccU = manufactured_parts(X, Y, Z)
        return -sig[s] * U + nu[s] * ccU

    def ainit(s, xs, ys, zs, k):
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        return manufactured_parts(X, Y, Z)[0]

    def B_exact(X, Y, Z, t):
        return np.exp(-t) * manufactured_parts(X, Y, Z)[1]

    def E_exact(X, Y, Z, t):
        return np.exp(-t) * manufactured_parts(X, Y, Z)[0]

    amp = np.exp(-dt * np.arange(1, n_t + 1))[None, :].astype(np.float64)
    nel = [np.full(P[d], n, dtype=np.int32) for d in range(3)]
    deg = [np.full(P[d], p, dtype=np.int32) for d in range(3)]
    return Problem(
        name=f"paper_cube2_p{p}_n{n}_nt{n_t}", np=P,
        breaks=[np.array([0.0, 0.5, 1.0]), np.array([0.0, 1.0]), np.array([0.0, 1.0])],
        nel=nel, deg=deg, sigma=sig, nu=nu, src_mask=np.ones(2, np.uint8), phi=None,
        amp=amp, dt=dt, n_steps=n_t, pcg_rtol=pcg_rtol, precision=precision,
        jvol=jvol, ainit=ainit, extra={"B_exact": B_exact, "E_exact": E_exact, "T": T})


WORKLOADS = {
    "plain": plain_fp64,
    "uneven": uneven_fp64,
    "mixed": floating_mixed,
    "largest": largest_multirhs,
}
