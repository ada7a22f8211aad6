"""Oracle side of the full-size residual checks (test helper).

At full size the oracle's direct solve does not fit one CPU, so a GPU field
is checked by the oracle's patch-by-patch residual of the implicit Euler
system (oracle/residual.py).  The oracle's work (the local matrices of each
distinct patch shape and the per-patch loads of the checked excitations)
runs in worker processes started fresh, which use no GPU; the problem is
rebuilt in each worker from its seeded maker.
"""
import multiprocessing as mp
import os

import workloads as W
from oracle import residual
from oracle.gauge import compute_topology
from oracle.grid import build_grid

MAKERS = {
    "largest": lambda steps: W.largest_multirhs(n_steps=steps),
    "mixed": lambda steps: W.floating_mixed(n_steps=steps),
}


def _op(args):
    name, steps, s = args
    return residual.local_operator(MAKERS[name](steps), s)


def _loads(args):
    name, steps, ks, chunk = args
    prob = MAKERS[name](steps)
    return [(s, residual.patch_load(prob, s, list(ks))) for s in chunk]


def oracle_side(name, steps, ks):
    """(prob, grid, kept edges, local operators, shape keys, per-patch loads)."""
    prob = MAKERS[name](steps)
    grid = build_grid(prob)
    topo = compute_topology(prob, grid)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    chunks = [list(range(s, prob.n_patches, workers)) for s in range(workers)]
    keys, reps = residual.shape_representatives(prob)
    print(f"[oracle side] {name}: {workers} workers, {len(reps)} patch shapes", flush=True)
    with ctx.Pool(workers) as pool:
        ops_async = {k: pool.apply_async(_op, ((name, steps, s),)) for k, s in reps.items()}
        loads = [None] * prob.n_patches
        for part in pool.imap_unordered(_loads, [(name, steps, ks, c) for c in chunks]):
            for s, L in part:
                loads[s] = L
        ops = {k: a.get() for k, a in ops_async.items()}
    return prob, grid, topo.kept, ops, keys, loads
