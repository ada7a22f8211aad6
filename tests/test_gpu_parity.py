"""GPU parity: the library's field against the oracle, element by element.

Fields are global edge vectors (zeros on Dirichlet and gauge-tree edges).
Bar: max over steps of ||a_gpu - a_oracle||_2 / ||a_oracle||_2 <= 1e-9 on the
FP64 path.  The PCG stops at ||r|| <= rtol ||d||, so the field error is about
cond(F) * rtol; the workloads run at their own rtol (1e-10).
"""
import numpy as np
import pytest

import workloads as W
from oracle import solve
from paper_2510_23446_amd import tcf
from tests.test_oracle_gauge import CASES, tiny

pytestmark = pytest.mark.gpu


def _run_and_compare(prob, tol, rtol=None, steps=None, every=1):
    steps = prob.n_steps if steps is None else steps
    ref = solve.run(prob, n_steps=steps)
    p = tcf.Problem(prob, pcg_rtol=rtol)
    print(f"[parity] {prob.name} steps={steps} counts={p.counts()}", flush=True)
    p.tcf_setup()
    worst = 0.0
    for l in range(steps):
        p.tcf_step(1)
        if l % every == 0 or l == steps - 1:
            for k in range(prob.n_rhs):
                a = p.tcf_get_field(k)
                r = ref.fields[l][:, k]
                assert np.linalg.norm(r) > 0, "reference field is zero: the case has no source"
                err = np.linalg.norm(a - r) / np.linalg.norm(r)
                worst = max(worst, err)
    st = p.tcf_get_stats()
    print(f"[parity] {prob.name} {prob.precision} worst rel err {worst:.3e} last iters {st['last_pcg_iters']} ir {st['last_ir_sweeps']} ir_res {st['last_ir_residual']:.2e}", flush=True)
    assert worst <= tol, worst
    return worst, st


@pytest.mark.parametrize("name", ["cond_bottom_p2", "floating_p2", "checker", "all_insulator",
                                  "all_conductor", "single_insulator", "two_subdomains"])
def test_tiny(name):
    P, n, p, sig = CASES[name]
    npatch = P[0] * P[1] * P[2]
    src = np.ones(npatch, np.uint8) if name == "all_conductor" else None
    prob = tiny(P, n, p, sig, src=src)
    _run_and_compare(prob, 1e-9, rtol=1e-12)


def test_plain_fp64_all_steps():
    worst, st = _run_and_compare(W.plain_fp64(), 1e-9)
    assert st["nonconverged_steps"] == 0


def test_uneven_reduced_seeded():
    prob = W.uneven_fp64(seed=1, n_steps=3, P=(3, 3, 3))
    _run_and_compare(prob, 1e-9)


# ---- FP32 factors + FP64 refinement ------------------------------------------
@pytest.mark.parametrize("mode", ["fp32_ir", "fp32_full_ir"])
@pytest.mark.parametrize("name", ["cond_bottom_p2", "floating_p2", "checker", "all_insulator"])
def test_tiny_fp32_ir(name, mode):
    P, n, p, sig = CASES[name]
    prob = tiny(P, n, p, sig)
    prob.precision = mode
    worst, st = _run_and_compare(prob, 1e-8)
    assert st["nonconverged_steps"] == 0


def test_plain_fp32_ir():
    prob = W.plain_fp64()
    prob.precision = "fp32_ir"
    worst, st = _run_and_compare(prob, 1e-8)
    assert st["last_ir_sweeps"] >= 1 and st["nonconverged_steps"] == 0


@pytest.mark.parametrize("mode", ["fp32_ir", "fp32_full_ir"])
def test_floating_reduced_fp32_ir(mode):
    """The floating-conductor layout (central 2x2x2 block) at n=4."""
    prob = W.floating_mixed(n=4, p=3, n_steps=3, precision=mode)
    _run_and_compare(prob, 1e-8)


def test_floating_reduced_fp64():
    prob = W.floating_mixed(n=4, p=3, n_steps=3, precision="fp64")
    _run_and_compare(prob, 1e-9)
