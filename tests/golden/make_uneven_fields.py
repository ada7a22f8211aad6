"""Writes the oracle's fields of the 64-patch uneven workload at full size.

The fixture ``uneven_seed1_fields.npz`` holds the first three implicit-Euler
steps of ``workloads.uneven_fp64(seed=1)`` (4x4x4 patches, per-row elements
in {4,6,8,12} and degrees in {2,3}, 185,689 edges, 144,914 gauged unknowns),
computed by ``oracle.solve.run`` alone: global FP64 assembly, the gauge of
Sec. 3 and one sparse direct factorisation of the gauged system (nested
dissection order), then one solve per step.  Nothing from the GPU path is
read or called.  Stored: the kept edge ids and the field values on them
(every other edge is zero), per step, plus the oracle's timings.

Run from the repository root:  python -m tests.golden.make_uneven_fields
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import solve  # noqa: E402

OUT = os.path.join(HERE, "uneven_seed1_fields.npz")
STEPS = 3


def main():
    prob = W.uneven_fp64(seed=1).with_steps(STEPS)
    t0 = time.perf_counter()
    run = solve.run(prob)
    wall = time.perf_counter() - t0
    K = run.topo.kept
    fields = np.stack([f[K, 0] for f in run.fields])  # (steps, n_kept)
    meta = dict(workload=prob.name, steps=STEPS, n_edges=int(run.sys.M.shape[0]),
                n_kept=int(len(K)), timings=run.timings, wall_s=wall)
    np.savez_compressed(OUT, kept=K.astype(np.int64), fields=fields,
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
