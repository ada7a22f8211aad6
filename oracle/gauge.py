"""Dirichlet set, tree-cotree gauge and the e / p / b / i split (oracle).

Sec. 3 gauges the insulating region by a spanning tree on the control mesh,
built globally over the wirebasket first, then the subdomain faces, then the
subdomain interiors; tree edges inside the insulator are eliminated, tree
edges on the conductor-insulator interface become primal, and everything
else is kept.  The paper states this for one conductor and one insulator
subdomain.  For many patches and floating conductors it is read here as:

Gauge tree T_I.  Build the graph H whose vertices are
  * the root R: every node on the outer boundary together with every node of
    a conductor component (closures of sigma>0 patches, joined when they
    share a node) that touches the outer boundary,
  * one super-vertex per floating conductor component,
  * every other ("plain") node,
and whose edges are the insulator-only edges (not Dirichlet and not inside
the closure of any conductor patch), self-loops dropped.  Breadth-first
search from R in three phases -- wirebasket edges, then face-interior edges,
then patch-interior edges -- with each later phase seeded by all vertices
visited so far in canonical order (R, floating components by smallest
member node, plain nodes by id), scanning a vertex's eligible edges in
increasing global edge id.  T_I is a spanning tree of H, so the discrete
gradients left in the kernel of the insulator system are removed exactly.

Primal set.  For every face shared by a conducting and an insulating patch,
a BFS tree of that face's face-interior edges rooted at the merged face
boundary; plus every non-Dirichlet wirebasket edge outside T_I.

Dual set.  Face-interior edges of faces between two patches that are neither
eliminated nor primal; each gives one multiplier row, ordered by global edge
id, with sign +1 in the lower patch id and -1 in the higher.

Interior set.  Patch-interior edges outside T_I.  Eliminated = D u T_I.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

from .grid import FACE, INTERIOR, WIREBASKET, Grid

# Sec. 3: the tree grows over the wirebasket first, then the subdomain faces,
# then the subdomain interiors.
PHASES = (WIREBASKET, FACE, INTERIOR)


@dataclass
class Topology:
    dirichlet: np.ndarray        # sorted global edge ids
    tree_I: np.ndarray           # sorted
    tree_gamma: np.ndarray       # sorted (primal Gamma-face tree edges)
    primal: np.ndarray           # sorted
    dual: np.ndarray             # sorted == multiplier order
    interior: np.ndarray         # sorted
    mult: np.ndarray             # (n_lambda, 3): edge id, patch +, patch -
    n_vertices_H: int
    n_plain: int
    n_floating: int
    cond_closure: np.ndarray     # bool per edge
    local: list                  # per patch dict: i, b, p, e (global ids, sorted)
    N: list                      # per patch: (p-edge gid sorted, global primal rank)

    @property
    def kept(self) -> np.ndarray:
        return np.setdiff1d(np.arange(len(self.cond_closure)),
                            np.union1d(self.dirichlet, self.tree_I))


def _patch_adjacency_components(prob, grid):
    """Conductor components: conducting patches joined when they share a node."""
    P = grid.P
    cond = [s for s in range(prob.n_patches) if prob.sigma[s] > 0]
    parent = {s: s for s in cond}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for s in cond:
        i, j, k = grid.patch_ijk(s)
        for t in cond:
            if t <= s:
                continue
            a, b, c = grid.patch_ijk(t)
            if abs(a - i) <= 1 and abs(b - j) <= 1 and abs(c - k) <= 1:
                ra, rb = find(s), find(t)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    comps = {}
    for s in cond:
        comps.setdefault(find(s), []).append(s)
    out = []
    for root, members in comps.items():
        touches = any(
            grid.patch_ijk(s)[d] in (0, P[d] - 1) for s in members for d in range(3))
        out.append((sorted(members), touches))
    return out


def _box_nodes(grid, s):
    (I0, I1), (J0, J1), (K0, K1) = grid.patch_box(s)
    K, J, I = np.meshgrid(np.arange(K0, K1 + 1), np.arange(J0, J1 + 1), np.arange(I0, I1 + 1),
                          indexing="ij")
    Nx, Ny, _ = grid.N
    return (I + Nx * (J + Ny * K)).ravel()


def _box_edges(grid, s):
    return grid.local_edges(s)[0]


def _bfs(adj, visited, seeds, tree):
    q = deque(seeds)
    while q:
        v = q.popleft()
        for (e, u) in adj.get(v, ()):
            if not visited[u]:
                visited[u] = True
                tree.append(e)
                q.append(u)


def compute_topology(prob, grid: Grid) -> Topology:
    nE, nN = grid.n_edges, grid.n_nodes
    eids = np.arange(nE)
    tail, head = grid.edge_nodes(eids)
    bnode = grid.node_on_boundary(np.arange(nN))
    dirichlet = bnode[tail] & bnode[head]
    ecls = grid.edge_class(eids)

    # conductor closures
    cond_closure = np.zeros(nE, dtype=bool)
    for s in range(prob.n_patches):
        if prob.sigma[s] > 0:
            cond_closure[_box_edges(grid, s)] = True
    insul_only = (~dirichlet) & (~cond_closure)

    # vertices of H
    comps = _patch_adjacency_components(prob, grid)
    node_vertex = np.full(nN, -1, dtype=np.int64)
    root_nodes = bnode.copy()
    floating = []
    for members, touches in comps:
        nodes = np.unique(np.concatenate([_box_nodes(grid, s) for s in members]))
        if touches:
            root_nodes[nodes] = True
        else:
            floating.append(nodes)
    node_vertex[root_nodes] = 0
    floating.sort(key=lambda nodes: int(nodes.min()))
    for j, nodes in enumerate(floating):
        assert np.all(node_vertex[nodes] == -1), "floating component overlaps root"
        node_vertex[nodes] = 1 + j
    plain = np.nonzero(node_vertex == -1)[0]
    node_vertex[plain] = 1 + len(floating) + np.arange(len(plain))
    nV = 1 + len(floating) + len(plain)

    # phased BFS
    visited = np.zeros(nV, dtype=bool)
    visited[0] = True
    tree = []
    for phase, cls in enumerate(PHASES):
        elig = np.nonzero(insul_only & (ecls == cls))[0]
        adj = {}
        for e in elig:  # increasing edge id
            a, b = int(node_vertex[tail[e]]), int(node_vertex[head[e]])
            if a == b:
                continue
            adj.setdefault(a, []).append((int(e), b))
            adj.setdefault(b, []).append((int(e), a))
        if phase == 0:
            seeds = [0]
        else:
            seeds = [int(v) for v in np.nonzero(visited)[0]]
        _bfs(adj, visited, seeds, tree)
    if not visited.all():
        raise RuntimeError("gauge tree does not span the insulator graph")
    tree_I = np.array(sorted(tree), dtype=np.int64)
    assert len(tree_I) == nV - 1

    in_tree = np.zeros(nE, dtype=bool)
    in_tree[tree_I] = True

    # Gamma-face trees
    gamma = []
    P = grid.P
    Nx, Ny, _ = grid.N
    for s in range(prob.n_patches):
        ijk = grid.patch_ijk(s)
        for d in range(3):
            if ijk[d] + 1 >= P[d]:
                continue
            nb = list(ijk)
            nb[d] += 1
            t = nb[0] + P[0] * (nb[1] + P[1] * nb[2])
            if (prob.sigma[s] > 0) == (prob.sigma[t] > 0):
                continue
            gamma.extend(_face_tree(grid, s, d, tail, head, ecls))
    tree_gamma = np.array(sorted(gamma), dtype=np.int64)

    primal_mask = np.zeros(nE, dtype=bool)
    primal_mask[tree_gamma] = True
    primal_mask |= (ecls == WIREBASKET) & (~dirichlet) & (~in_tree)
    interior_mask = (ecls == INTERIOR) & (~in_tree)
    dual_mask = (ecls == FACE) & (~dirichlet) & (~in_tree) & (~primal_mask)

    primal = np.nonzero(primal_mask)[0]
    dual = np.nonzero(dual_mask)[0]
    interior = np.nonzero(interior_mask)[0]

    # which patches own each edge
    owners = [[] for _ in range(nE)]
    local = []
    for s in range(prob.n_patches):
        g = _box_edges(grid, s)
        for e in g[dual_mask[g]]:
            owners[int(e)].append(s)
        loc = {
            "i": np.sort(g[interior_mask[g]]),
            "b": np.sort(g[dual_mask[g]]),
            "p": np.sort(g[primal_mask[g]]),
            "e": np.sort(g[dirichlet[g] | in_tree[g]]),
        }
        local.append(loc)
    mult = np.zeros((len(dual), 3), dtype=np.int64)
    for r, e in enumerate(dual):
        o = sorted(owners[int(e)])
        assert len(o) == 2, f"dual edge {e} owned by {o}"
        mult[r] = (e, o[0], o[1])
    rank = np.full(nE, -1, dtype=np.int64)
    rank[primal] = np.arange(len(primal))
    Ns = [(loc["p"], rank[loc["p"]]) for loc in local]
    return Topology(dirichlet=np.nonzero(dirichlet)[0], tree_I=tree_I, tree_gamma=tree_gamma,
                    primal=primal, dual=dual, interior=interior, mult=mult, n_vertices_H=nV,
                    n_plain=len(plain), n_floating=len(floating), cond_closure=cond_closure,
                    local=local, N=Ns)


def _face_tree(grid, s, d, tail, head, ecls):
    """BFS tree over the face-interior edges of the face between patch s and
    its +d neighbour, rooted at the merged boundary of that face."""
    box = grid.patch_box(s)
    plane = box[d][1]
    u, v = [a for a in range(3) if a != d]
    Nx, Ny, _ = grid.N
    # face-interior edges on this face: direction u or v, lying in the plane,
    # with both nodes inside the face rectangle and the edge not wirebasket
    edges = []
    for dirn in (u, v):
        lo = [box[0][0], box[1][0], box[2][0]]
        hi = [box[0][1], box[1][1], box[2][1]]
        lo[d] = hi[d] = plane
        hi[dirn] -= 1
        rng = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        K, J, I = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        ids = grid.edge_id(dirn, I.ravel(), J.ravel(), K.ravel())
        edges.append(ids)
    edges = np.concatenate(edges)
    edges = np.sort(edges[ecls[edges] == FACE])

    def on_face_boundary(n):
        I, J, K = grid.node_ijk(n)
        c = (I, J, K)
        return any(c[a] in (box[a][0], box[a][1]) for a in (u, v))

    ROOT = -1
    adj = {}
    for e in edges:
        a, b = int(tail[e]), int(head[e])
        va = ROOT if on_face_boundary(a) else a
        vb = ROOT if on_face_boundary(b) else b
        if va == vb:
            continue
        adj.setdefault(va, []).append((int(e), vb))
        adj.setdefault(vb, []).append((int(e), va))
    visited = {ROOT}
    tree = []
    q = deque([ROOT])
    while q:
        x = q.popleft()
        for (e, y) in adj.get(x, ()):
            if y not in visited:
                visited.add(y)
                tree.append(e)
                q.append(y)
    return tree
