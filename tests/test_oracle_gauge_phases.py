"""Pin of the gauge tree's phase order (Sec. 3: wirebasket, then faces, then
interiors) that does not reuse the oracle's own construction.

Any spanning tree of the contracted insulator graph H is a valid gauge, so
the validity and kernel-dimension pins cannot see the order in which the
tree was grown.  The order leaves a trace that is independent of tie
breaking: the tree's wirebasket edges alone must span exactly the vertices
that wirebasket edges reach from the root; its wirebasket and face edges
together must span exactly the vertices that face edges then reach from
those; the interior edges must add every vertex left.  The graph is rebuilt
here from the grid alone (conductor components by connected components of
the conductor-closure edges, not by the oracle's patch adjacency), and a
planted swap of two phases in the oracle makes the pin fail.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle import gauge, grid as G
from tests.test_oracle_gauge import CASES, tiny


def _contracted_graph(prob, g):
    """Vertex of every node, edge classes and the insulator-only mask."""
    nE, nN = g.n_edges, g.n_nodes
    eids = np.arange(nE)
    tail, head = g.edge_nodes(eids)
    bnode = g.node_on_boundary(np.arange(nN))
    dirichlet = bnode[tail] & bnode[head]
    cond = np.zeros(nE, dtype=bool)
    for s in range(prob.n_patches):
        if prob.sigma[s] > 0:
            cond[g.local_edges(s)[0]] = True
    # conductor components: connected components of the closure edges
    ce = np.nonzero(cond)[0]
    A = sp.coo_matrix((np.ones(len(ce)), (tail[ce], head[ce])), shape=(nN, nN))
    _, lab = connected_components(A, directed=False)
    in_cond = np.zeros(nN, dtype=bool)
    in_cond[tail[ce]] = True
    in_cond[head[ce]] = True
    grounded = set(lab[in_cond & bnode].tolist())
    vert = np.full(nN, -1, dtype=np.int64)
    vert[bnode] = 0
    for c in grounded:
        vert[(lab == c) & in_cond] = 0
    nxt = 1
    for c in sorted(set(lab[in_cond].tolist()) - grounded):
        vert[(lab == c) & in_cond] = nxt
        nxt += 1
    free = vert < 0
    vert[free] = nxt + np.arange(int(free.sum()))
    nV = int(vert.max()) + 1
    elig = (~dirichlet) & (~cond)
    return vert, nV, g.edge_class(eids), elig, tail, head


def _component_of_root(nV, a, b, extra_root=None):
    """Vertices connected to vertex 0 through edges (a, b); extra_root
    (a vertex mask) is joined to the root first."""
    ra, rb = list(a), list(b)
    if extra_root is not None:
        v = np.nonzero(extra_root)[0]
        ra += [0] * len(v)
        rb += list(v)
    A = sp.coo_matrix((np.ones(len(ra)), (ra, rb)), shape=(nV, nV))
    _, lab = connected_components(A, directed=False)
    return lab == lab[0]


def _spans(nV, mask, a, b):
    """Edges (a, b) form a spanning tree of the vertices in mask."""
    if len(a) != int(mask.sum()) - 1:
        return False
    if not (mask[a].all() and mask[b].all()):
        return False
    sub = np.nonzero(mask)[0]
    idx = np.full(nV, -1)
    idx[sub] = np.arange(len(sub))
    A = sp.coo_matrix((np.ones(len(a)), (idx[a], idx[b])), shape=(len(sub), len(sub)))
    return connected_components(A, directed=False)[0] == 1


def phase_order_holds(prob, g, tree_I):
    vert, nV, ecls, elig, tail, head = _contracted_graph(prob, g)

    def ends(edges):
        a, b = vert[tail[edges]], vert[head[edges]]
        keep = a != b
        return a[keep], b[keep]

    cls_edges = {c: np.nonzero(elig & (ecls == c))[0] for c in (G.WIREBASKET, G.FACE, G.INTERIOR)}
    t_cls = ecls[tree_I]
    # wirebasket phase: the root's component over wirebasket edges
    VW = _component_of_root(nV, *ends(cls_edges[G.WIREBASKET]))
    tW = tree_I[t_cls == G.WIREBASKET]
    if not _spans(nV, VW, *ends(tW)):
        return False
    # face phase: what face edges reach from the visited set
    VF = _component_of_root(nV, *ends(cls_edges[G.FACE]), extra_root=VW)
    tWF = tree_I[(t_cls == G.WIREBASKET) | (t_cls == G.FACE)]
    if not _spans(nV, VF, *ends(tWF)):
        return False
    # interior phase: everything
    return _spans(nV, np.ones(nV, dtype=bool), *ends(tree_I))


@pytest.mark.parametrize("name", sorted(CASES))
def test_tree_follows_the_phase_order(name):
    P, n, p, sig = CASES[name]
    prob = tiny(P, n, p, sig)
    g = G.build_grid(prob)
    topo = gauge.compute_topology(prob, g)
    assert phase_order_holds(prob, g, topo.tree_I)


def test_tree_follows_the_phase_order_uneven():
    """An uneven layout with mixed degrees and a floating conductor."""
    import workloads as W
    prob = W.subproblem(W.uneven_fp64(), P=(3, 3, 2))
    prob = W.Problem(**{**prob.__dict__, "nel": [np.minimum(x, 3) for x in prob.nel]})
    g = G.build_grid(prob)
    topo = gauge.compute_topology(prob, g)
    assert phase_order_holds(prob, g, topo.tree_I)


@pytest.mark.parametrize("swapped", [(G.FACE, G.WIREBASKET, G.INTERIOR),
                                     (G.WIREBASKET, G.INTERIOR, G.FACE),
                                     (G.INTERIOR, G.FACE, G.WIREBASKET)])
def test_planted_phase_swap_fails(monkeypatch, swapped):
    """Planted mistake in the oracle: two phases swapped.  The tree is still
    a valid gauge, but the phase-order pin rejects it on some layout."""
    monkeypatch.setattr(gauge, "PHASES", swapped)
    failed = []
    for name in ("cond_bottom_p2", "floating_p2", "checker", "all_insulator"):
        P, n, p, sig = CASES[name]
        prob = tiny(P, n, p, sig)
        g = G.build_grid(prob)
        topo = gauge.compute_topology(prob, g)
        assert len(topo.tree_I) == topo.n_vertices_H - 1  # still a spanning tree
        if not phase_order_holds(prob, g, topo.tree_I):
            failed.append(name)
    assert failed, "a swapped phase order went unnoticed"


def test_gamma_face_trees_span_their_faces():
    """The conductor/insulator face trees together touch every interior node
    of every such face, with one edge per interior node, and connect each to
    the face boundaries (a spanning tree of the faces with their boundaries
    contracted to one vertex)."""
    for name in ("cond_bottom_p2", "checker", "two_subdomains", "floating_p2"):
        P, n, p, sig = CASES[name]
        prob = tiny(P, n, p, sig)
        g = G.build_grid(prob)
        topo = gauge.compute_topology(prob, g)
        inner = set()
        for s in range(prob.n_patches):
            ijk = g.patch_ijk(s)
            box = g.patch_box(s)
            for d in range(3):
                if ijk[d] + 1 >= P[d]:
                    continue
                nb = list(ijk)
                nb[d] += 1
                t = nb[0] + P[0] * (nb[1] + P[1] * nb[2])
                if (prob.sigma[s] > 0) == (prob.sigma[t] > 0):
                    continue
                rng = [np.arange(box[a][0] + 1, box[a][1]) for a in range(3)]
                rng[d] = np.array([box[d][1]])
                K, J, I = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
                inner |= set((I + g.N[0] * (J + g.N[1] * K)).ravel().tolist())
        assert len(topo.tree_gamma) == len(inner)
        tail, head = g.edge_nodes(topo.tree_gamma)
        touched = set(tail.tolist()) | set(head.tolist())
        assert inner <= touched
        nodes = sorted(touched)
        pos = {x: i + 1 for i, x in enumerate(nodes)}
        vid = lambda x: pos[int(x)] if int(x) in inner else 0  # noqa: E731
        a = [vid(x) for x in tail]
        b = [vid(x) for x in head]
        A = sp.coo_matrix((np.ones(len(a)), (a, b)), shape=(len(nodes) + 1,) * 2)
        lab = connected_components(A, directed=False)[1]
        assert len({lab[pos[x]] for x in inner} | {lab[0]}) == 1
