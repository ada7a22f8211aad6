"""Small dense NumPy FETI-DP used by the tests (test code, not the oracle).

It rebuilds the dual-primal reduction of Sec. 3 from the oracle's per-patch
matrices and its e / p / b / i split, so that tests can check the reduction
itself (interface jump, primal continuity, agreement with the global gauged
solve) and compare intermediate quantities of the GPU library.

Per patch s, with W = M + dt K restricted to [i | b | p]:
  S_bb = W_bb - W_bi W_ii^-1 W_ib,   S_bp likewise,
  S_pp = W_pp - W_pi W_ii^-1 W_ip - S_bp^T S_bb^-1 S_bp,
  S_Pi = sum_s N_s^T S_pp N_s,
  Bhat_s = dt * (signed Boolean jump on the b rows).
"""
from __future__ import annotations

import numpy as np


class DenseFETI:
    def __init__(self, prob, sysm, topo):
        self.prob = prob
        self.sys = sysm
        self.topo = topo
        dt = prob.dt
        self.dt = dt
        nP = len(topo.primal)
        nL = len(topo.dual)
        self.nP, self.nL = nP, nL
        rankP = {int(e): r for r, e in enumerate(topo.primal)}
        rankL = {int(e): r for r, e in enumerate(topo.dual)}
        self.pat = []
        for s, pm in enumerate(sysm.patches):
            loc = topo.local[s]
            pos = {int(g): k for k, g in enumerate(pm.gid)}
            order = {c: np.array([pos[int(g)] for g in loc[c]], dtype=np.int64) for c in "ibp"}
            Wl = (pm.M + dt * pm.K).toarray()
            Ml = pm.M.toarray()
            ii, bb, pp = order["i"], order["b"], order["p"]
            d = dict(i=ii, b=bb, p=pp, gid=pm.gid, W=Wl, M=Ml, jhat=pm.jhat)
            Wii = Wl[np.ix_(ii, ii)]
            Wib = Wl[np.ix_(ii, bb)]
            Wip = Wl[np.ix_(ii, pp)]
            Sbb = Wl[np.ix_(bb, bb)] - Wib.T @ np.linalg.solve(Wii, Wib)
            Sbp = Wl[np.ix_(bb, pp)] - Wib.T @ np.linalg.solve(Wii, Wip)
            Spp1 = Wl[np.ix_(pp, pp)] - Wip.T @ np.linalg.solve(Wii, Wip)
            Phi = np.linalg.solve(Sbb, Sbp)
            Spp = Spp1 - Sbp.T @ Phi
            Ns = np.array([rankP[int(g)] for g in loc["p"]], dtype=np.int64)
            B = np.zeros((nL, len(bb)))
            for k, g in enumerate(loc["b"]):
                r = rankL[int(g)]
                B[r, k] = 1.0 if topo.mult[r, 1] == s else -1.0
            d.update(Wii=Wii, Wib=Wib, Wip=Wip, Sbb=Sbb, Sbp=Sbp, Spp=Spp, Phi=Phi,
                     Sbbinv=np.linalg.inv(Sbb), N=Ns, B=B)
            self.pat.append(d)
        SPi = np.zeros((nP, nP))
        for d in self.pat:
            SPi[np.ix_(d["N"], d["N"])] += d["Spp"]
        self.SPi = SPi

    # ---- operators -----------------------------------------------------
    def F(self, lam):
        dt = self.dt
        c = np.zeros(self.nP)
        xs = []
        for d in self.pat:
            x = dt * d["B"].T @ lam
            xs.append(x)
            np.add.at(c, d["N"], d["Phi"].T @ x)
        q = np.linalg.solve(self.SPi, c)
        y = np.zeros(self.nL)
        for d, x in zip(self.pat, xs):
            w = d["Sbbinv"] @ x + d["Phi"] @ q[d["N"]]
            y += dt * d["B"] @ w
        return y

    def precond(self, r):
        z = np.zeros(self.nL)
        for d in self.pat:
            z += d["B"] @ (d["Sbb"] @ (d["B"].T @ r))
        return z

    def step(self, a_prev_global, amp, rtol=1e-12, maxit=5000):
        """One implicit Euler step; returns (global field, iterations)."""
        dt = self.dt
        fl = []
        for d in self.pat:
            al = a_prev_global[d["gid"]]
            fl.append(d["M"] @ al + dt * amp * d["jhat"][:, 0])
        h = np.zeros(self.nP)
        us, gbs, ys = [], [], []
        for d, f in zip(self.pat, fl):
            fi, fb, fp = f[d["i"]], f[d["b"]], f[d["p"]]
            y = np.linalg.solve(d["Wii"], fi)
            gb = fb - d["Wib"].T @ y
            gp = fp - d["Wip"].T @ y
            u = np.linalg.solve(d["Sbb"], gb)
            np.add.at(h, d["N"], gp - d["Sbp"].T @ u)
            us.append(u)
            gbs.append(gb)
            ys.append((fi, gb, gp))
        q0 = np.linalg.solve(self.SPi, h)
        dvec = np.zeros(self.nL)
        for d, u in zip(self.pat, us):
            dvec += dt * d["B"] @ (u - d["Phi"] @ q0[d["N"]])
        lam, it = self.pcg(dvec, rtol, maxit)
        # recovery
        c = np.zeros(self.nP)
        for d in self.pat:
            np.add.at(c, d["N"], d["Phi"].T @ (dt * d["B"].T @ lam))
        pglob = np.linalg.solve(self.SPi, h + c)
        out = np.zeros(self.sys.grid.n_edges)
        for d, (fi, gb, gp) in zip(self.pat, ys):
            x = dt * d["B"].T @ lam
            ap = pglob[d["N"]]
            ab = np.linalg.solve(d["Sbb"], gb - x - d["Sbp"] @ ap)
            ai = np.linalg.solve(d["Wii"], fi - d["Wib"] @ ab - d["Wip"] @ ap)
            out[d["gid"][d["i"]]] = ai
            out[d["gid"][d["b"]]] = ab
            out[d["gid"][d["p"]]] = ap
        return out, it, dvec, lam

    def pcg(self, d, rtol, maxit):
        lam = np.zeros_like(d)
        nd = np.linalg.norm(d)
        if nd == 0:
            return lam, 0
        r = d.copy()
        z = self.precond(r)
        p = z.copy()
        rz = r @ z
        for it in range(1, maxit + 1):
            q = self.F(p)
            alpha = rz / (p @ q)
            lam += alpha * p
            r -= alpha * q
            if np.linalg.norm(r) <= rtol * nd:
                return lam, it
            z = self.precond(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return lam, maxit
