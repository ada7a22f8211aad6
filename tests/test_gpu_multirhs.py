"""Many excitations in one PCG on the matrix cores.

Batches wider than 4 columns run every tile product as v_mfma_f64_16x16x4
(FP64 accumulation) in widths of 8, 16 or 32, each operator tile read once
per iteration for all columns; each column keeps its own step lengths and
stopping test, and idle columns carry zero right-hand sides.  The fields
match the oracle, and the same solves in batches of 4 on the vector path.
"""
import numpy as np
import pytest

import workloads as W
from paper_2510_23446_amd import tcf
from tests.test_gpu_parity import _run_and_compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_rhs,batch", [(8, 0), (12, 0), (32, 0), (32, 16)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_wide_batches_match_the_oracle(n_rhs, batch, prec):
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=n_rhs, n_steps=3, precision=prec)
    tol = 1e-9 if prec == "fp64" else 1e-8
    worst, st = _run_and_compare(prob, tol, rhs_batch=batch)
    assert st["nonconverged_steps"] == 0


def test_wide_and_narrow_batches_agree():
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=32, n_steps=2, precision="fp64")
    out = {}
    for batch in (4, 32):
        p = tcf.Problem(prob, rhs_batch=batch, pcg_rtol=1e-12)
        p.tcf_setup()
        p.tcf_step(prob.n_steps)
        out[batch] = np.stack([p.tcf_get_field(k) for k in range(prob.n_rhs)])
    a, b = out[4], out[32]
    err = np.linalg.norm(a - b, axis=1) / np.linalg.norm(a, axis=1)
    assert err.max() <= 1e-10, err.max()


@pytest.mark.parametrize("coarse_mode", [1, 2])
def test_wide_batch_with_each_coarse_solver(coarse_mode):
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=16, n_steps=2, precision="fp64")
    worst, st = _run_and_compare(prob, 1e-9, coarse_mode=coarse_mode)
    assert st["nonconverged_steps"] == 0


@pytest.mark.parametrize("chunk", [1, 3, 1000])
def test_panel_split_lengths_keep_the_solution(chunk):
    """Row panels split into jobs of 1 tile (every output row added by many
    jobs), 3, or not at all: the same solution as the oracle."""
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=8, n_steps=2, precision="fp64")
    worst, st = _run_and_compare(prob, 1e-9, panel_chunk=chunk, coarse_mode=2)
    assert st["panel_chunk"] == [chunk] * 4 and st["panel_chunk_src"] == 0


def test_autotuned_split_and_tune_table(tmp_path):
    """Timing the split lengths at setup keeps the solution; the result goes
    to the tune table, and a second handle of the same shape takes it from
    there without timing."""
    table = str(tmp_path / "panels.txt")
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=16, n_steps=2, precision="fp64")
    worst, st = _run_and_compare(prob, 1e-9, autotune=1, tune_table=table, coarse_mode=2)
    assert st["panel_chunk_src"] == 2
    cands = (4, 8, 16, 32, 1 << 20)
    assert all(c in cands for c in st["panel_chunk"])
    assert all(t > 0 for t in st["panel_tune_us"])
    lines = open(table).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(" ".join(map(str, st["panel_chunk"])))
    q = tcf.Problem(prob, autotune=1, tune_table=table, coarse_mode=2)
    q.tcf_setup()
    s2 = q.tcf_get_stats()
    assert s2["panel_chunk_src"] == 1 and s2["panel_chunk"] == st["panel_chunk"]
    assert open(table).read().splitlines() == lines


@pytest.mark.parametrize("batch,prec", [(1, "fp64"), (4, "fp64"), (32, "fp64"), (8, "fp32_ir")])
def test_deterministic_sums_match_the_oracle_and_rerun_bitwise(batch, prec):
    """deterministic = 1 (row panels at every batch width, staged shared rows,
    per-job quadratic forms): the oracle's fields, and a second handle gives
    the same bits."""
    n_rhs = max(batch, 2)
    prob = W.largest_multirhs(P=(4, 4, 2), n=4, p=3, n_rhs=n_rhs, n_steps=2, precision=prec)
    tol = 1e-9 if prec == "fp64" else 1e-8
    worst, st = _run_and_compare(prob, tol, rhs_batch=batch, deterministic=1, coarse_mode=2)
    assert st["rhs_batch"] == batch and st["panel_jobs"] > 0
    fields = []
    for _ in range(2):
        p = tcf.Problem(prob, rhs_batch=batch, deterministic=1, coarse_mode=2)
        p.tcf_setup()
        p.tcf_step(prob.n_steps)
        fields.append(np.stack([p.tcf_get_field(k) for k in range(prob.n_rhs)]))
    assert np.array_equal(fields[0], fields[1])
