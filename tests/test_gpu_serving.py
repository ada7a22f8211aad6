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


def test_alone_equals_mix_on_the_served_draws():
    """The served workload's own draws (256 seeded requests, k in {2, 3, 4},
    per-row n in {4..10}): the first three 4 x 4 x 4 requests and two
    smaller ones, 3 steps each, in one mix of 3 slots, each against its run
    alone."""
    draws = W.serving_requests(n_req=256, seed=3, n_steps=50)
    big = [r for r in draws if r.np[0] == 4][:3]
    small = [r for r in draws if r.np[0] < 4][:2]
    reqs = [r.with_steps(3) for r in big + small]
    assert max(int(max(n.max() for n in r.nel)) for r in big) >= 8
    srv = tcf.Server(max_bytes=128 << 30, max_slots=3)
    ids = [srv.tcf_server_submit(r, precision="fp32_ir") for r in reqs]
    for i in ids:
        assert srv.tcf_server_wait(i) == tcf.TCF_OK
    for i, r in zip(ids, reqs):
        mix, _ = srv.tcf_server_fetch(i)
        alone = _alone(r, "fp32_ir")
        d = np.linalg.norm(mix - alone) / np.linalg.norm(alone)
        print(f"[serving] {r.name} nel {[[int(v) for v in n] for n in r.nel]} alone-vs-mix {d:.2e}", flush=True)
        assert d <= 1e-8
    srv.tcf_server_destroy()


def test_alone_equals_mix_bitwise_with_deterministic_sums():
    """Requests served three at a time give the same bits as each run alone
    when the library sums deterministically."""
    reqs = _requests(n=5, steps=3)
    srv = tcf.Server(max_bytes=64 << 30, max_slots=3)
    ids = [srv.tcf_server_submit(r, precision="fp32_ir", deterministic=1) for r in reqs]
    for i in ids:
        assert srv.tcf_server_wait(i) == tcf.TCF_OK
    for i, r in zip(ids, reqs):
        mix, _ = srv.tcf_server_fetch(i)
        p = tcf.Problem(r, precision="fp32_ir", deterministic=1)
        p.tcf_setup()
        p.tcf_step(r.n_steps)
        alone = p.tcf_get_field(0)
        print(f"[serving] {r.name} deterministic alone-vs-mix bitwise {np.array_equal(mix, alone)}",
              flush=True)
        assert np.array_equal(mix, alone)
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
