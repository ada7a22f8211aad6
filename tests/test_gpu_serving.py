"""Serving: requests admitted by device memory, overlapping on the GPU.

Each request's final field in the mix must equal its field when run alone
(within the solver tolerance: the tile products accumulate with atomics, so
runs agree to rounding, not bitwise), and match the CPU oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import solve
from paper_2510_23446_amd import tcf

pytestmark = pytest.mark.gpu


def _requests(n=6, steps=4):
    reqs = W.serving_requests(n_req=n, seed=3, n_steps=steps, ks=(2, 3), nrange=(3, 5))
    return reqs


def _alone(prob, precision):
    p = tcf.Problem(prob, precision=precision)
    p.tcf_setup()
    p.tcf_step(prob.n_steps)
    return p.tcf_get_field(0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_alone_equals_mix(precision):
    reqs = _requests()
    srv = tcf.Server(max_bytes=64 << 30, max_slots=3)
    ids = [srv.tcf_server_submit(r, precision=precision) for r in reqs]
    for i in ids:
        assert srv.tcf_server_wait(i) == tcf.TCF_OK
    st = srv.tcf_server_stats()
    print(f"[serving] {precision} stats {st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["steps"] == sum(r.n_steps for r in reqs)
    tol = 1e-9 if precision == "fp64" else 1e-8
    for i, r in zip(ids, reqs):
        mix, s = srv.tcf_server_fetch(i)
        alone = _alone(r, precision)
        d = np.linalg.norm(mix - alone) / np.linalg.norm(alone)
        print(f"[serving] {r.name} alone-vs-mix {d:.2e} steps {s['steps_done']}", flush=True)
        assert d <= tol
    # two of them against the oracle
    for i, r in list(zip(ids, reqs))[:2]:
        mix, _ = srv.tcf_server_fetch(i)
        ref = solve.run(r).fields[-1][:, 0]
        d = np.linalg.norm(mix - ref) / np.linalg.norm(ref)
        print(f"[serving] {r.name} vs oracle {d:.2e}", flush=True)
        assert d <= tol
    srv.tcf_server_destroy()


def test_admission_by_memory():
    reqs = _requests(n=4)
    fps = []
    for r in reqs:
        fps.append(tcf.Problem(r).tcf_footprint()[0])
    budget = max(fps) + min(fps) // 2  # never room for two of the largest
    srv = tcf.Server(max_bytes=budget, max_slots=4)
    ids = [srv.tcf_server_submit(r, precision="fp64") for r in reqs]
    for i in ids:
        assert srv.tcf_server_wait(i) == tcf.TCF_OK
    st = srv.tcf_server_stats()
    assert st["completed"] == len(reqs)
    assert st["peak_bytes"] <= budget
    srv.tcf_server_destroy()


def test_oversize_request_rejected():
    r = _requests(n=1)[0]
    fp = tcf.Problem(r).tcf_footprint()[0]
    srv = tcf.Server(max_bytes=fp // 2, max_slots=2)
    with pytest.raises(tcf.TcfError) as e:
        srv.tcf_server_submit(r, precision="fp64")
    assert e.value.code == tcf.TCF_ENOMEM
    srv.tcf_server_destroy()
