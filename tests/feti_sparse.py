"""Sparse FETI-DP on the oracle's per-patch matrices (test code, not the oracle).

The dense prototypes (``feti_ref``, ``feti_loop_ref``) hold dense Schur
complements, which caps them at small layouts.  This one keeps each patch's
remainder block K_rr = W[r, r] (r = interior + dual unknowns) in a sparse LU,
so that the iteration counts of both splits can be measured on full-size
layouts on the CPU.

With W = M + dt K per patch, the primal coupling N_s and jump rows B_s:

  F lam = sum_s B_s K_rr^-1 B_s^T lam + C^T S_Pi^-1 C lam,
  C lam = sum_s N_s^T K_pr K_rr^-1 B_s^T lam,
  S_Pi  = sum_s N_s^T (K_pp - K_pr K_rr^-1 K_rp) N_s,
  d     = sum_s B_s K_rr^-1 f_r - C^T S_Pi^-1 h,
  h     = sum_s N_s^T (f_p - K_pr K_rr^-1 f_r),

and the Dirichlet preconditioner sum_s B_D,s S_bb,s B_D,s^T, with
S_bb = K_bb - K_bi K_ii^-1 K_ib and the weights of ``feti_loop_ref``.  The
PCG stops at ||r|| <= rtol ||d||, the library's test.

``split="tree"`` is the published split (the interface-face trees primal);
``split="loop"`` is the loop split.  The field is mapped back to the oracle's
gauge, so it can be checked against the oracle's gauged global system.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import gauge
from tests.feti_loop_ref import loop_structure


class SparseFETI:
    def __init__(self, prob, sysm, topo, split="tree", weights="none", load_correction=True):
        assert split in ("tree", "loop") and weights in ("none", "stiffness")
        self.prob, self.sys, self.topo = prob, sysm, topo
        dt = prob.dt
        self.dt = dt
        grid = sysm.grid
        nE = grid.n_edges
        cond = np.asarray(prob.sigma) > 0
        self.cond = cond
        if split == "loop":
            L = loop_structure(prob, sysm, topo)
            in_tg, coef, corr = L["in_tg"], L["coef"], L["corr"]
            loop_rows = {e: (cs, is_) for e, cs, is_ in L["cotree"]}
            self.tail, self.head = L["tail"], L["head"]
        else:
            in_tg = np.zeros(nE, dtype=bool)
            coef, corr, loop_rows = {}, None, {}
        self.coef = coef
        primal = np.setdiff1d(topo.primal, np.nonzero(in_tg)[0])
        rankP = np.full(nE, -1, dtype=np.int64)
        rankP[primal] = np.arange(len(primal))
        dual = np.asarray(topo.dual, dtype=np.int64)
        rankL = np.full(nE, -1, dtype=np.int64)
        rankL[dual] = np.arange(len(dual))
        self.nP, self.nL = len(primal), len(dual)
        nL = self.nL
        loop_mask = np.zeros(nL, dtype=bool)
        loop_mask[rankL[np.array(sorted(loop_rows), dtype=np.int64)]] = True
        self.loop_mask = loop_mask

        self.pat = []
        for s, pm in enumerate(sysm.patches):
            loc = topo.local[s]
            pos = {int(x): k for k, x in enumerate(pm.gid)}
            p_ids = np.array([e for e in loc["p"] if not in_tg[e]], dtype=np.int64)
            b_ids = np.asarray(loc["b"], dtype=np.int64)
            if cond[s]:
                b_ids = np.concatenate([b_ids, np.array([e for e in loc["p"] if in_tg[e]],
                                                        dtype=np.int64)])
            ii = np.array([pos[int(x)] for x in loc["i"]], dtype=np.int64)
            bb = np.array([pos[int(x)] for x in b_ids], dtype=np.int64)
            pp = np.array([pos[int(x)] for x in p_ids], dtype=np.int64)
            bpos = {int(x): k for k, x in enumerate(b_ids)}
            rows, cols, vals, own_r, own_c = [], [], [], [], []
            for e in loc["b"]:
                e = int(e)
                r = int(rankL[e])
                own_r.append(r)
                own_c.append(bpos[e])
                if e in loop_rows:
                    cs, is_ = loop_rows[e]
                    if s == is_:
                        rows.append(r); cols.append(bpos[e]); vals.append(-1.0)
                    else:
                        rows.append(r); cols.append(bpos[e]); vals.append(1.0)
                        x, y = int(self.tail[e]), int(self.head[e])
                        for t, w in coef.get(y, {}).items():
                            rows.append(r); cols.append(bpos[t]); vals.append(w)
                        for t, w in coef.get(x, {}).items():
                            rows.append(r); cols.append(bpos[t]); vals.append(-w)
                else:
                    rows.append(r); cols.append(bpos[e])
                    vals.append(1.0 if topo.mult[r, 1] == s else -1.0)
            B = sp.csr_matrix((vals, (rows, cols)), shape=(nL, len(bb)))
            W = (pm.M + dt * pm.K).tocsc()
            rr = np.concatenate([ii, bb])
            Krr = W[rr][:, rr].tocsc()
            Krp = W[rr][:, pp].toarray()
            lu = spla.splu(Krr)
            Z = lu.solve(Krp) if len(pp) else np.zeros((len(rr), 0))
            Spp = W[pp][:, pp].toarray() - Krp.T @ Z
            jh = pm.jhat[:, 0].copy()
            if corr is not None and cond[s] and load_correction:
                jh = jh + corr[pm.gid, 0]
            d = dict(gid=pm.gid, i=ii, b=bb, p=pp, nI=len(ii), B=B, lu=lu, Z=Z, Spp=Spp,
                     Krp=Krp, M=pm.M.tocsr(), m0=pm.m0[:, 0], jhat=jh, W=W,
                     N=rankP[p_ids], own_r=np.array(own_r, dtype=np.int64),
                     own_c=np.array(own_c, dtype=np.int64))
            d["Kii"] = spla.splu(W[ii][:, ii].tocsc()) if len(ii) else None
            d["Kib"] = W[ii][:, bb].tocsc()
            d["Kbb"] = W[bb][:, bb].tocsc()
            self.pat.append(d)
        SPi = np.zeros((self.nP, self.nP))
        for d in self.pat:
            SPi[np.ix_(d["N"], d["N"])] += d["Spp"]
        self.SPi_f = sla.cho_factor(SPi) if self.nP else None
        self._set_weights(weights)
        self.insul_only = np.ones(nE, dtype=bool)
        for s in range(prob.n_patches):
            if cond[s]:
                self.insul_only[gauge._box_edges(grid, s)] = False

    # ---- weights -------------------------------------------------------------
    def _set_weights(self, weights):
        nL, loop = self.nL, self.loop_mask
        if weights == "none":
            for d in self.pat:
                d["BD"] = d["B"]
            return
        k = []
        for d in self.pat:
            kd = d["Kbb"].diagonal()
            kr = np.zeros(nL)
            kr[d["own_r"]] = kd[d["own_c"]]
            k.append(kr)
        tot = sum(k)
        kC = sum(kk for kk, c in zip(k, self.cond) if c)
        kI = sum(kk for kk, c in zip(k, self.cond) if not c)
        w_I = kC / np.where(kI + kC > 0, kI + kC, 1.0)
        for s, d in enumerate(self.pat):
            part = np.zeros(nL, dtype=bool)
            part[d["own_r"]] = True
            w = np.where(part & ~loop, (tot - k[s]) / np.where(tot > 0, tot, 1.0), 0.0)
            if not self.cond[s]:
                w = np.where(part & loop, w_I, w)
            BD = sp.diags(w) @ d["B"]
            mine = np.nonzero(part & loop)[0]
            if self.cond[s] and len(mine):
                Bl = d["B"][mine].toarray()
                P = np.linalg.solve(Bl @ Bl.T, Bl) * (1.0 - w_I[mine])[:, None]
                BD = BD.tolil()
                BD[mine] = P
                BD = BD.tocsr()
            d["BD"] = sp.csr_matrix(BD)

    # ---- operators -------------------------------------------------------------
    def _coarse(self, c):
        return sla.cho_solve(self.SPi_f, c) if self.nP else c

    def F(self, lam):
        c = np.zeros(self.nP)
        us = []
        for d in self.pat:
            rhs = np.zeros(d["nI"] + len(d["b"]))
            rhs[d["nI"]:] = d["B"].T @ lam
            u = d["lu"].solve(rhs)
            us.append(u)
            np.add.at(c, d["N"], d["Krp"].T @ u)
        q = self._coarse(c)
        y = np.zeros(self.nL)
        for d, u in zip(self.pat, us):
            v = u + d["Z"] @ q[d["N"]]
            y += d["B"] @ v[d["nI"]:]
        return y

    def precond(self, r):
        z = np.zeros(self.nL)
        for d in self.pat:
            x = d["BD"].T @ r
            y = d["Kbb"] @ x
            if d["Kii"] is not None:
                y -= d["Kib"].T @ d["Kii"].solve(d["Kib"] @ x)
            z += d["BD"] @ y
        return z

    def pcg(self, dvec, rtol, maxit, lam0=None, r0=None):
        """PCG from lam0 (r0 = d - F lam0 given with it); stops at
        ||r|| <= rtol ||d||.  Returns (lam, iterations)."""
        nd = np.linalg.norm(dvec)
        if nd == 0:
            return np.zeros_like(dvec), 0
        if lam0 is None:
            lam, r = np.zeros_like(dvec), dvec.copy()
        else:
            lam, r = lam0.copy(), r0.copy()
            if np.linalg.norm(r) <= rtol * nd:
                self.last_r = r
                return lam, 0
        z = self.precond(r)
        p = z.copy()
        rz = r @ z
        for it in range(1, maxit + 1):
            q = self.F(p)
            alpha = rz / (p @ q)
            lam += alpha * p
            r -= alpha * q
            if np.linalg.norm(r) <= rtol * nd:
                self.last_r = r
                return lam, it
            z = self.precond(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        self.last_r = r
        return lam, maxit

    # ---- one implicit Euler step ------------------------------------------
    def step(self, a_prev, amp, first=False, rtol=1e-10, maxit=2000, window=0):
        """Returns (field in the oracle's gauge, PCG iterations).

        window > 0 starts the PCG from the Galerkin projection onto the span
        of the newest ``window`` solutions of earlier calls,
        lam0 = L (L^T F L)^-1 L^T d, with F L kept from each solve as d - r.
        """
        dt = self.dt
        h = np.zeros(self.nP)
        dvec = np.zeros(self.nL)
        fr_all, w0 = [], []
        for d in self.pat:
            f = d["M"] @ a_prev[d["gid"]] + dt * amp * d["jhat"]
            if first:
                f = f + d["m0"]
            fr = np.concatenate([f[d["i"]], f[d["b"]]])
            u = d["lu"].solve(fr)
            np.add.at(h, d["N"], f[d["p"]] - d["Krp"].T @ u)
            fr_all.append((fr, f[d["p"]]))
            w0.append(u)
        q0 = self._coarse(h)
        for d, u in zip(self.pat, w0):
            dvec += d["B"] @ (u - d["Z"] @ q0[d["N"]])[d["nI"]:]
        hist = getattr(self, "_hist", [])
        if window and hist:
            Lm = np.stack([h_[0] for h_ in hist], 1)
            FL = np.stack([h_[1] for h_ in hist], 1)
            G = Lm.T @ FL
            G = 0.5 * (G + G.T)
            w_, V = np.linalg.eigh(G)
            keep = w_ > 1e-12 * w_.max()
            coef = V[:, keep] @ ((V[:, keep].T @ (Lm.T @ dvec)) / w_[keep])
            lam0, r0 = Lm @ coef, dvec - FL @ coef
            lam, it = self.pcg(dvec, rtol, maxit, lam0, r0)
        else:
            lam, it = self.pcg(dvec, rtol, maxit)
        if window:
            self._hist = (hist + [(lam.copy(), dvec - self.last_r)])[-window:]
        c = np.zeros(self.nP)
        for d in self.pat:
            rhs = np.zeros(d["nI"] + len(d["b"]))
            rhs[d["nI"]:] = d["B"].T @ lam
            np.add.at(c, d["N"], d["Krp"].T @ d["lu"].solve(rhs))
        up = self._coarse(h + c)
        local = []
        for d, (fr, fp) in zip(self.pat, fr_all):
            ap = up[d["N"]]
            rhs = fr - d["Krp"] @ ap
            rhs[d["nI"]:] -= d["B"].T @ lam
            ur = d["lu"].solve(rhs)
            loc = np.zeros(len(d["gid"]))
            loc[d["i"]] = ur[:d["nI"]]
            loc[d["b"]] = ur[d["nI"]:]
            loc[d["p"]] = ap
            local.append(loc)
        return self._conforming(local), it

    def _conforming(self, local):
        nE = self.sys.grid.n_edges
        a = np.zeros(nE)
        aC = np.zeros(nE)
        for s, (d, loc) in enumerate(zip(self.pat, local)):
            (aC if self.cond[s] else a)[d["gid"]] = loc
        if self.coef:
            psi = np.zeros(self.sys.grid.n_nodes)
            for n, c in self.coef.items():
                psi[n] = sum(w * aC[t] for t, w in c.items())
            gpsi = psi[self.head] - psi[self.tail]
            a[self.insul_only] -= gpsi[self.insul_only]
        for s, (d, loc) in enumerate(zip(self.pat, local)):
            if self.cond[s]:
                a[d["gid"]] = loc
        return a


def main(workload="uneven"):
    """Full-size comparison of the splits: one implicit Euler step from
    zero, then the second step from that field, for each split and
    weighting; the residual is the oracle's gauged global system's.

    * ``uneven``: the benchmark's 64-patch layout (about 7 minutes);
    * ``checkerboard``: the 256-patch checkerboard at n = 4, one excitation
      (the multi-excitation workload's operator).
    """
    import time

    import workloads as W
    from oracle import assemble, grid as G, solve

    if workload == "uneven":
        prob = W.uneven_fp64(seed=1, n_steps=3)
    elif workload == "checkerboard":
        prob = W.largest_multirhs(n=4, n_rhs=1, n_steps=3)
    else:
        raise ValueError(workload)
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    Wg, K = solve.gauged_matrix(sysm, topo, prob.dt)

    def resid(a, a_prev, amp):
        f = sysm.M @ a_prev + prob.dt * amp * sysm.jhat[:, 0]
        return np.linalg.norm(Wg @ a[K] - f[K]) / np.linalg.norm(f[K])

    a1 = None
    for split, w in [("tree", "stiffness"), ("tree", "none"), ("loop", "stiffness")]:
        t0 = time.time()
        sf = SparseFETI(prob, sysm, topo, split=split, weights=w)
        if a1 is None:
            a1, _ = sf.step(np.zeros(g.n_edges), prob.amp[0, 0])
        a2, it = sf.step(a1, prob.amp[0, 1])
        print(f"{split}/{w}: primal {sf.nP}, multipliers {sf.nL}, step-2 PCG iterations {it}, "
              f"residual {resid(a2, a1, prob.amp[0, 1]):.1e}, {time.time() - t0:.0f} s", flush=True)


def main_projection(n_steps=12):
    """Both splits, stiffness-weighted, with the projection start from the
    newest 8 solutions, over the first n_steps steps of the benchmark's
    64-patch layout (about 12 minutes)."""
    import time

    import workloads as W
    from oracle import assemble, grid as G

    prob = W.uneven_fp64(seed=1, n_steps=n_steps)
    g = G.build_grid(prob)
    sysm = assemble.assemble_global(prob, g)
    topo = gauge.compute_topology(prob, g)
    for split in ("tree", "loop"):
        t0 = time.time()
        sf = SparseFETI(prob, sysm, topo, split=split, weights="stiffness")
        a = np.zeros(g.n_edges)
        its = []
        for l in range(n_steps):
            a, it = sf.step(a, prob.amp[0, l], window=8)
            its.append(it)
            print(f"{split}: step {l + 1} PCG iterations {it}", flush=True)
        print(f"{split}/stiffness + projection start: iterations {its}, "
              f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    import sys

    if sys.argv[1:2] == ["projection"]:
        main_projection()
    else:
        main(*sys.argv[1:2])
