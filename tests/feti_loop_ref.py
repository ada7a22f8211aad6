"""Dense NumPy FETI-DP with loop constraints on the conductor-insulator
interface (test code, not the oracle).

Sec. 3 makes the tree edges of every interface face between a conductor and
an insulator primal.  Its outlook (Sec. 5) asks for a split that drops them
from the primal set while every local matrix stays nonsingular.  Dropping
them alone is not enough: on an insulator patch each such edge that moves to
the remainder adds one dimension to the local kernel (the gradients of the
nodal functions of the face's interior nodes).  This module builds a split
that does drop them, and checks it against the oracle.

* Insulator side: the face-tree edges T_G are eliminated (zero), like the
  insulator's own tree.  The local matrices are those of the usual split with
  T_G fixed, hence nonsingular.
* Conductor side: the T_G edges become remainder unknowns with no partner
  (W_C is nonsingular in any case).
* The conductor and insulator fields now differ on the interface by a
  discrete gradient G psi.  psi vanishes on the face boundary (the
  wirebasket), and on the face's interior nodes it is fixed by
  a_C(t) + psi(head t) - psi(tail t) = 0 for t in T_G, i.e. sums of a_C along
  tree paths.  Along the insulator's tree T_I it is extended as a constant
  (G psi = 0 on T_I), so the gauge of the oracle is kept.
* Each cotree edge e of the face keeps one multiplier, and its jump row
  becomes a loop: a_I(e) = a_C(e) + psi(head e) - psi(tail e).
* The insulator energy is invariant under gradients (sigma = 0 there, and
  K G = 0).  The load is not: the functional gains f_I^T G psi(a_C), so the
  conductor's T_G rows get -sum_n (G^T f_I)(n) d psi(n) / d a_C(t).  This
  vanishes for curl-form sources and matters for volume sources that cross
  the interface.

The primal set shrinks by |T_G|.  Mapping the result back,
a_I - G psi(a_C), gives the conforming field in the oracle's gauge, so the
check against the oracle is element by element.

Preconditioner: the Dirichlet preconditioner sum_s B_D,s S_bb,s B_D,s^T
needs weights with sum_s B_D,s B_s^T = I (a partition of unity over the
multipliers); ``_set_weights`` gives three choices.  Unweighted, the long
loop rows dominate, and the iterations grow with 1/h.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from oracle import gauge
from oracle.grid import FACE, incidence_G
from tests.feti_ref import DenseFETI


def _gamma_faces(prob, grid):
    """(s, d, t): patch s, its +d neighbour t, of different conductivity."""
    P = grid.P
    out = []
    for s in range(prob.n_patches):
        ijk = grid.patch_ijk(s)
        for d in range(3):
            if ijk[d] + 1 >= P[d]:
                continue
            nb = list(ijk)
            nb[d] += 1
            t = nb[0] + P[0] * (nb[1] + P[1] * nb[2])
            if (prob.sigma[s] > 0) != (prob.sigma[t] > 0):
                out.append((s, d, t))
    return out


def _face_edges_and_boundary(grid, s, d, ecls):
    """Face edges (class FACE) of the face between s and its +d neighbour,
    and a predicate for nodes on that face's boundary."""
    box = grid.patch_box(s)
    plane = box[d][1]
    u, v = [a for a in range(3) if a != d]
    edges = []
    for dirn in (u, v):
        lo = [box[0][0], box[1][0], box[2][0]]
        hi = [box[0][1], box[1][1], box[2][1]]
        lo[d] = hi[d] = plane
        hi[dirn] -= 1
        rng = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        K, J, I = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        edges.append(grid.edge_id(dirn, I.ravel(), J.ravel(), K.ravel()))
    edges = np.concatenate(edges)
    edges = np.sort(edges[ecls[edges] == FACE])

    def on_boundary(n):
        c = grid.node_ijk(n)
        return any(c[a] in (box[a][0], box[a][1]) for a in (u, v))

    return edges, on_boundary


def loop_structure(prob, sysm, topo):
    """The loop split's data: psi coefficients per node (face trees, then
    constant along T_I), the cotree rows (edge, conductor patch, insulator
    patch), and the load correction on the conductor's T_G rows per
    excitation (corr, indexed by global edge)."""
    grid = sysm.grid
    nE = grid.n_edges
    eids = np.arange(nE)
    tail, head = grid.edge_nodes(eids)
    ecls = grid.edge_class(eids)
    cond = np.asarray(prob.sigma) > 0
    tg = np.asarray(topo.tree_gamma, dtype=np.int64)
    in_tg = np.zeros(nE, dtype=bool)
    in_tg[tg] = True

    # psi(n) = sum_t coef[n][t] a_C(t) on the face interior nodes
    coef = {}
    cotree = []  # (edge, conductor patch, insulator patch)
    is_dual = np.zeros(nE, dtype=bool)
    is_dual[np.asarray(topo.dual, dtype=np.int64)] = True
    for s, d, t in _gamma_faces(prob, grid):
        edges, on_boundary = _face_edges_and_boundary(grid, s, d, ecls)
        tree = [int(e) for e in edges if in_tg[e]]
        adj = {}
        for e in tree:
            a, b = int(tail[e]), int(head[e])
            adj.setdefault(a, []).append(e)
            adj.setdefault(b, []).append(e)
        seeds = [n for n in adj if on_boundary(n)]
        seen = set(seeds)
        q = deque(seeds)
        while q:
            x = q.popleft()
            for e in adj[x]:
                y = int(head[e]) if int(tail[e]) == x else int(tail[e])
                if y in seen:
                    continue
                seen.add(y)
                c = dict(coef.get(x, {}))
                # psi(head) = psi(tail) - a(e)
                c[e] = c.get(e, 0.0) + (-1.0 if int(tail[e]) == x else 1.0)
                coef[y] = c
                q.append(y)
        assert all(on_boundary(n) or n in coef for n in adj)
        c_s, i_s = (s, t) if cond[s] else (t, s)
        for e in edges:
            if not in_tg[e] and is_dual[e]:
                cotree.append((int(e), c_s, i_s))

    # extension along T_I, away from grounded nodes
    grounded = np.asarray(grid.node_on_boundary(np.arange(grid.n_nodes)), dtype=bool).copy()
    for s in range(prob.n_patches):
        if cond[s]:
            grounded[gauge._box_nodes(grid, s)] = True
    adjI = {}
    for e in topo.tree_I:
        a, b = int(tail[e]), int(head[e])
        adjI.setdefault(a, []).append(b)
        adjI.setdefault(b, []).append(a)
    seed = {n: n for n in coef}
    q = deque(n for n in list(coef) if n in adjI)
    while q:
        x = q.popleft()
        for y in adjI.get(x, ()):
            if grounded[y]:
                continue
            if y in seed:
                # T_I is a tree: a subtree hangs from one interface node
                assert seed[y] == seed[x], "subtree reached from two interface nodes"
                continue
            seed[y] = seed[x]
            coef[y] = coef[x]
            q.append(y)

    # load correction from the insulator load, per excitation
    GI = incidence_G(grid).tocsr()
    fI = np.zeros((nE, prob.n_rhs))
    for s, pm in enumerate(sysm.patches):
        if not cond[s]:
            np.add.at(fI, pm.gid, pm.jhat)
    g = GI.T @ fI  # (n_nodes, n_rhs)
    corr = np.zeros((nE, prob.n_rhs))
    for n, c in coef.items():
        for t, w in c.items():
            corr[t] -= g[n] * w

    return dict(grid=grid, nE=nE, tail=tail, head=head, cond=cond, tg=tg, in_tg=in_tg,
                coef=coef, cotree=cotree, corr=corr)


def loop_structure_from_host_plan(prob, sysm, topo, loop_terms, psi_terms):
    """The same data as loop_structure, built only from the library's host
    plan: loop_terms (multiplier row, edge, +-1) are the conductor-side terms
    of every loop row, psi_terms (node, edge, +-1) the coefficients of psi.
    The cotree rows come from the multiplier table, the load correction from
    psi and G^T of the insulator load.  Also returns the rows' terms
    (row_terms: multiplier row -> [(edge, +-1)])."""
    grid = sysm.grid
    nE = grid.n_edges
    tail, head = grid.edge_nodes(np.arange(nE))
    cond = np.asarray(prob.sigma) > 0
    tg = np.asarray(topo.tree_gamma, dtype=np.int64)
    in_tg = np.zeros(nE, dtype=bool)
    in_tg[tg] = True
    coef = {}
    for n, t, w in np.asarray(psi_terms, dtype=np.int64).reshape(-1, 3):
        coef.setdefault(int(n), {})[int(t)] = float(w)
    row_terms = {}
    for r, t, w in np.asarray(loop_terms, dtype=np.int64).reshape(-1, 3):
        row_terms.setdefault(int(r), []).append((int(t), float(w)))
    cotree = []
    for r in sorted(row_terms):
        e, sp, sm = (int(v) for v in topo.mult[r])
        cotree.append((e, sp, sm) if cond[sp] else (e, sm, sp))
    GI = incidence_G(grid).tocsr()
    fI = np.zeros((nE, prob.n_rhs))
    for s, pm in enumerate(sysm.patches):
        if not cond[s]:
            np.add.at(fI, pm.gid, pm.jhat)
    g = GI.T @ fI
    corr = np.zeros((nE, prob.n_rhs))
    for n, c in coef.items():
        for t, w in c.items():
            corr[t] -= g[n] * w
    return dict(grid=grid, nE=nE, tail=tail, head=head, cond=cond, tg=tg, in_tg=in_tg,
                coef=coef, cotree=cotree, corr=corr, row_terms=row_terms)


class LoopFETI(DenseFETI):
    """FETI-DP on the loop split; same operators and PCG as DenseFETI.

    With host_plan = (loop_terms, psi_terms), the library's arrays of the
    loop rows and of psi replace this file's own construction: the conductor
    side of each loop row takes the row's terms as given."""

    def __init__(self, prob, sysm, topo, load_correction=True, weights="stiffness",
                 host_plan=None):
        if host_plan is None:
            L = loop_structure(prob, sysm, topo)
        else:
            L = loop_structure_from_host_plan(prob, sysm, topo, *host_plan)
        row_terms = L.get("row_terms")
        grid, nE, tail, head, cond = L["grid"], L["nE"], L["tail"], L["head"], L["cond"]
        tg, in_tg, coef, cotree, corr = L["tg"], L["in_tg"], L["coef"], L["cotree"], L["corr"]
        self.coef = coef

        # the split
        primal = np.setdiff1d(topo.primal, tg)
        rankP = {int(e): r for r, e in enumerate(primal)}
        dual = np.asarray(topo.dual, dtype=np.int64)
        rankL = {int(e): r for r, e in enumerate(dual)}
        loop_rows = {e: (cs, is_) for e, cs, is_ in cotree}
        self.prob, self.sys, self.topo = prob, sysm, topo
        dt = prob.dt
        self.dt = dt
        self.nP, self.nL = len(primal), len(dual)
        self.primal = primal
        self.pat = []
        for s, pm in enumerate(sysm.patches):
            loc = topo.local[s]
            pos = {int(x): k for k, x in enumerate(pm.gid)}
            p_ids = np.array([e for e in loc["p"] if not in_tg[e]], dtype=np.int64)
            b_ids = np.asarray(loc["b"], dtype=np.int64)
            if cond[s]:
                b_ids = np.concatenate([b_ids, np.array([e for e in loc["p"] if in_tg[e]],
                                                        dtype=np.int64)])
            order = {"i": np.array([pos[int(x)] for x in loc["i"]], dtype=np.int64),
                     "b": np.array([pos[int(x)] for x in b_ids], dtype=np.int64),
                     "p": np.array([pos[int(x)] for x in p_ids], dtype=np.int64)}
            bpos = {int(x): k for k, x in enumerate(b_ids)}
            B = np.zeros((self.nL, len(b_ids)))
            own = np.full(self.nL, -1, dtype=np.int64)  # column of the row's own edge
            for e in loc["b"]:
                r = rankL[int(e)]
                own[r] = bpos[int(e)]
                if int(e) in loop_rows:
                    cs, is_ = loop_rows[int(e)]
                    if s == is_:
                        B[r, bpos[int(e)]] = -1.0
                    elif row_terms is not None:
                        for t, w in row_terms[r]:
                            B[r, bpos[t]] += w
                    else:
                        B[r, bpos[int(e)]] += 1.0
                        x, y = int(tail[e]), int(head[e])
                        for t, w in coef.get(y, {}).items():
                            B[r, bpos[t]] += w
                        for t, w in coef.get(x, {}).items():
                            B[r, bpos[t]] -= w
                else:
                    B[r, bpos[int(e)]] = 1.0 if topo.mult[r, 1] == s else -1.0
            jh = pm.jhat.copy()
            if cond[s] and load_correction:
                jh = jh + corr[pm.gid]
            self._add_patch(pm, order, B, np.array([rankP[int(x)] for x in p_ids],
                                                   dtype=np.int64), jh)
            self.pat[-1]["own"] = own
        SPi = np.zeros((self.nP, self.nP))
        for d in self.pat:
            SPi[np.ix_(d["N"], d["N"])] += d["Spp"]
        self.SPi = SPi
        self.cond = cond
        loop_mask = np.zeros(self.nL, dtype=bool)
        loop_mask[[rankL[e] for e in loop_rows]] = True
        self.loop_mask = loop_mask
        self._set_weights(weights)
        self.tail, self.head = tail, head
        self.insul_only = ~np.zeros(nE, dtype=bool)
        for s in range(prob.n_patches):
            if cond[s]:
                self.insul_only[gauge._box_edges(grid, s)] = False

    def _set_weights(self, weights):
        """B_D per patch for the Dirichlet preconditioner
        sum_s B_D,s S_bb,s B_D,s^T, with sum_s B_D,s B_s^T = I.

        * "none": B_D = B (unweighted).
        * "insulator": 1/2 per side on Boolean rows; a loop row weight 1 on
          the insulator's single entry, 0 on the conductor's loop.
        * "stiffness": with k_s the diagonal of patch s's W at the row's own
          edge, the side s of a Boolean row gets k_o / (k_s + k_o) (the
          other side's share).  A loop row gives its insulator entry
          w_I = k_C / (k_I + k_C), and the conductor the rest,
          (1 - w_I) (B_C B_C^T)^-1 B_C over that patch's loop rows (B_C B_C^T
          is SPD: each loop row holds its own edge, which no other row does).
        """
        nL, cond, loop = self.nL, self.cond, self.loop_mask
        if weights == "none":
            for d in self.pat:
                d["BD"] = d["B"]
            return
        k = []
        for d in self.pat:
            kd = np.diag(d["W"])[d["b"]]
            k.append(np.where(d["own"] >= 0, kd[np.maximum(d["own"], 0)], 0.0))
        tot = sum(k)
        kC = sum(kk for kk, c in zip(k, cond) if c)
        kI = sum(kk for kk, c in zip(k, cond) if not c)
        for s, d in enumerate(self.pat):
            part = d["own"] >= 0
            if weights == "insulator":
                w_bool = np.where(part, 0.5, 0.0)
                w_I = np.ones(nL)
            elif weights == "stiffness":
                w_bool = np.where(part, (tot - k[s]) / np.where(tot > 0, tot, 1.0), 0.0)
                w_I = kC / np.where(kI + kC > 0, kI + kC, 1.0)
            else:
                raise ValueError(weights)
            BD = np.where(loop, 0.0, w_bool)[:, None] * d["B"]
            mine = loop & part
            if mine.any():
                if cond[s]:
                    if weights == "stiffness":
                        Bl = d["B"][mine]
                        BD[mine] = (1.0 - w_I[mine])[:, None] * np.linalg.solve(Bl @ Bl.T, Bl)
                else:
                    BD[mine] = w_I[mine][:, None] * d["B"][mine]
            d["BD"] = BD

    def precond(self, r):
        z = np.zeros(self.nL)
        for d in self.pat:
            z += d["BD"] @ (d["Sbb"] @ (d["BD"].T @ r))
        return z


    def _add_patch(self, pm, order, B, Ns, jhat):
        dt = self.dt
        Wl = (pm.M + dt * pm.K).toarray()
        ii, bb, pp = order["i"], order["b"], order["p"]
        Wii = Wl[np.ix_(ii, ii)]
        Wib = Wl[np.ix_(ii, bb)]
        Wip = Wl[np.ix_(ii, pp)]
        Sbb = Wl[np.ix_(bb, bb)] - Wib.T @ np.linalg.solve(Wii, Wib)
        Sbp = Wl[np.ix_(bb, pp)] - Wib.T @ np.linalg.solve(Wii, Wip)
        Spp1 = Wl[np.ix_(pp, pp)] - Wip.T @ np.linalg.solve(Wii, Wip)
        Phi = np.linalg.solve(Sbb, Sbp)
        self.pat.append(dict(i=ii, b=bb, p=pp, gid=pm.gid, W=Wl, M=pm.M.toarray(), jhat=jhat,
                             Wii=Wii, Wib=Wib, Wip=Wip, Sbb=Sbb, Sbp=Sbp,
                             Spp=Spp1 - Sbp.T @ Phi, Phi=Phi, Sbbinv=np.linalg.inv(Sbb),
                             N=Ns, B=B))

    def conforming(self, out_patch_fields):
        """Global edge vector in the oracle's gauge from the per-patch local
        fields: insulator values minus G psi(a_C), conductor values as they are."""
        nE = self.sys.grid.n_edges
        a = np.zeros(nE)
        for s, loc in enumerate(out_patch_fields):
            if not self.cond[s]:
                a[self.sys.patches[s].gid] = loc
        aC = np.zeros(nE)
        for s, loc in enumerate(out_patch_fields):
            if self.cond[s]:
                aC[self.sys.patches[s].gid] = loc
        psi = np.zeros(self.sys.grid.n_nodes)
        for n, c in self.coef.items():
            psi[n] = sum(w * aC[t] for t, w in c.items())
        gpsi = psi[self.head] - psi[self.tail]
        a[self.insul_only] -= gpsi[self.insul_only]
        for s, loc in enumerate(out_patch_fields):
            if self.cond[s]:
                a[self.sys.patches[s].gid] = loc
        return a

    def step_local(self, a_prev_global, amp, first=False, rtol=1e-12, maxit=5000):
        """One implicit Euler step; returns (per-patch local fields, iterations).
        The first step adds the initial load int sigma A0 . w (conductors only,
        so the gradient shift of the insulator leaves it unchanged)."""
        dt = self.dt
        h = np.zeros(self.nP)
        us, ys = [], []
        for d, pm in zip(self.pat, self.sys.patches):
            f = d["M"] @ a_prev_global[d["gid"]] + dt * amp * d["jhat"][:, 0]
            if first and pm.m0 is not None:
                f = f + pm.m0[:, 0]
            fi, fb, fp = f[d["i"]], f[d["b"]], f[d["p"]]
            y = np.linalg.solve(d["Wii"], fi)
            gb = fb - d["Wib"].T @ y
            gp = fp - d["Wip"].T @ y
            u = np.linalg.solve(d["Sbb"], gb)
            np.add.at(h, d["N"], gp - d["Sbp"].T @ u)
            us.append(u)
            ys.append((fi, gb))
        q0 = np.linalg.solve(self.SPi, h)
        dvec = np.zeros(self.nL)
        for d, u in zip(self.pat, us):
            dvec += dt * d["B"] @ (u - d["Phi"] @ q0[d["N"]])
        lam, it = self.pcg(dvec, rtol, maxit)
        c = np.zeros(self.nP)
        for d in self.pat:
            np.add.at(c, d["N"], d["Phi"].T @ (dt * d["B"].T @ lam))
        pglob = np.linalg.solve(self.SPi, h + c)
        fields = []
        for d, (fi, gb) in zip(self.pat, ys):
            x = dt * d["B"].T @ lam
            ap = pglob[d["N"]]
            ab = np.linalg.solve(d["Sbb"], gb - x - d["Sbp"] @ ap)
            ai = np.linalg.solve(d["Wii"], fi - d["Wib"] @ ab - d["Wip"] @ ap)
            loc = np.zeros(len(d["gid"]))
            loc[d["i"]] = ai
            loc[d["b"]] = ab
            loc[d["p"]] = ap
            fields.append(loc)
        return fields, it


def stiffness_weighted(fe):
    """The stiffness-scaled Dirichlet preconditioner on the published (tree)
    split of a DenseFETI: side s of a multiplier gets k_o / (k_s + k_o)."""
    nL = fe.nL
    k = []
    for d in fe.pat:
        kd = np.diag(d["W"])[d["b"]]
        kr = np.zeros(nL)
        rows, cols = np.nonzero(d["B"])
        kr[rows] = kd[cols]
        k.append(kr)
    tot = sum(k)
    BD = [np.where(kk > 0, (tot - kk) / np.where(tot > 0, tot, 1.0), 0.0)[:, None] * d["B"]
          for kk, d in zip(k, fe.pat)]

    def precond(r):
        z = np.zeros(nL)
        for bd, d in zip(BD, fe.pat):
            z += bd @ (d["Sbb"] @ (bd.T @ r))
        return z
    fe.precond = precond
    return fe
