"""GPU parity of the coarse solve through the nested-dissection factor, and
of the setup in patch groups.

The coarse matrix S_Pi (Sec. 3, the second Schur complement) is solved
either through one dense inverse or through a Cholesky factor in a nested
dissection of the patch grid (dense blocks per separator, the top
separator's Schur complement inverted densely).  Both are S_Pi^-1 to
rounding, so the field matches the oracle to the same bar either way; these
cases force the factor (coarse_mode=2) on layouts where the automatic
choice would take the dense inverse, and split the setup into groups of
one patch (setup_group_mb=1) so that every group boundary is crossed.
"""
import numpy as np
import pytest

import workloads as W
from paper_2510_23446_amd import tcf
from tests.test_gpu_parity import _run_and_compare
from tests.test_oracle_gauge import CASES, tiny

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "plain":
        return W.plain_fp64().with_steps(4), 1e-9, {}
    if name == "uneven_3x3x3":
        return W.uneven_fp64(seed=1, n_steps=3, P=(3, 3, 3)), 1e-9, {}
    if name == "floating_fp32_ir":
        return W.floating_mixed(n=4, p=3, n_steps=3, precision="fp32_ir"), 1e-8, {}
    if name == "checkerboard_4x4x2_batched":
        prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=4, n_steps=3, precision="fp64")
        return prob, 1e-9, {"rhs_batch": 4}
    if name == "checkerboard_4x4x2_fp32_ir":
        prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=3, n_steps=3, precision="fp32_ir")
        return prob, 1e-8, {"rhs_batch": 3}
    if name == "floating_fp32_full_ir":
        return W.floating_mixed(n=4, p=3, n_steps=3, precision="fp32_full_ir"), 1e-8, {}
    raise KeyError(name)


@pytest.mark.parametrize("name", ["plain", "uneven_3x3x3", "floating_fp32_ir",
                                  "checkerboard_4x4x2_batched", "checkerboard_4x4x2_fp32_ir"])
def test_nested_dissection_coarse_matches_oracle(name):
    prob, tol, kw = _case(name)
    worst, st = _run_and_compare(prob, tol, coarse_mode=2, **kw)
    print(f"[coarse] {name}: nodes {st['coarse_nodes']} launches {st['coarse_launches']} "
          f"top block {st['coarse_root']} of {st['n_primal']}", flush=True)
    assert st["coarse_nodes"] > 1
    assert st["coarse_root"] < st["n_primal"]
    assert st["nonconverged_steps"] == 0


@pytest.mark.parametrize("name", ["checker", "floating_p2"])
def test_nested_dissection_coarse_tiny(name):
    P, n, p, sig = CASES[name]
    prob = tiny(P, n, p, sig)
    worst, st = _run_and_compare(prob, 1e-9, rtol=1e-12, coarse_mode=2)
    assert st["coarse_nodes"] >= 1


def test_dense_and_factored_coarse_agree():
    """The two coarse solvers give the same field to the PCG tolerance."""
    prob = W.uneven_fp64(seed=1, n_steps=3, P=(3, 3, 3))
    out = []
    for mode in (1, 2):
        p = tcf.Problem(prob, coarse_mode=mode, pcg_rtol=1e-12)
        p.tcf_setup()
        p.tcf_step(prob.n_steps)
        out.append(p.tcf_get_field(0))
        st = p.tcf_get_stats()
        assert (st["coarse_nodes"] == 1) == (mode == 1)
    a, b = out
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)


@pytest.mark.parametrize("name", ["uneven_3x3x3", "floating_fp32_ir", "floating_fp32_full_ir"])
def test_setup_in_single_patch_groups(name):
    """Setup with one patch per group (and the coarse factor) gives the same
    field as the oracle; the handle's device high-water mark stays within
    the footprint it reports for its precision."""
    prob, tol, kw = _case(name)
    worst, st = _run_and_compare(prob, tol, setup_group_mb=1, coarse_mode=2, **kw)
    assert st["setup_chunks"] == st["n_patches"]


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp32_full_ir"])
def test_device_peak_within_footprint(prec):
    """Admission by footprint is safe: the high-water mark of the handle's
    device allocations, setup included, never exceeds tcf_footprint for its
    precision (FP32_IR factorises in FP64 and keeps FP32 operators)."""
    prob = W.floating_mixed(n=4, p=3, n_steps=2, precision=prec)
    for kw in ({}, {"coarse_mode": 2, "setup_group_mb": 64}):
        p = tcf.Problem(prob, **kw)
        b64, b32 = p.tcf_footprint()
        p.tcf_setup()
        p.tcf_step(prob.n_steps)
        st = p.tcf_get_stats()
        bound = b64 if prec == "fp64" else b32
        print(f"[memory] {prec} {kw}: peak {st['device_bytes_peak'] / 2**20:.1f} MiB, "
              f"resident {st['device_bytes'] / 2**20:.1f} MiB, footprint {bound / 2**20:.1f} MiB",
              flush=True)
        assert st["device_bytes_peak"] <= bound
