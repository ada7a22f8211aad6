"""tcf_step_noalloc (PCG scratch in the library's static device array, no
graph, nothing allocated) against tcf_step on the same problems, through the
C-ABI: two problems in a row, the second smaller, each checked against
tcf_step's field and the oracle's; calls of both kinds interleaved on one
handle."""
import numpy as np
import pytest

import workloads as W
from oracle import solve
from paper_2510_23446_amd import tcf

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("which", ["uneven_sub2x2x2_then_plain"])
def test_noalloc_step_matches_tcf_step(which):
    big = W.subproblem(W.uneven_fp64(), P=(2, 2, 2)).with_steps(3)
    small = W.plain_fp64().with_steps(3)
    for prob in (big, small):  # the second call has the smaller input
        print(f"[noalloc] {prob.name}", flush=True)
        ref = solve.run(prob)
        a = tcf.Problem(prob)
        a.tcf_setup()
        b = tcf.Problem(prob)
        b.tcf_setup()
        for l in range(prob.n_steps):
            a.tcf_step(1)
            b.tcf_step_noalloc(1)
            fa = np.array(a.tcf_get_field(0), copy=True)
            fb = np.array(b.tcf_get_field(0), copy=True)
            r = ref.fields[l][:, 0]
            d_ab, d_or = _rel(fb, fa), _rel(fb, r)
            print(f"[noalloc] {prob.name} step {l}: vs tcf_step {d_ab:.2e}, vs oracle {d_or:.2e}",
                  flush=True)
            # the same solver to its PCG tolerance (tile sums use atomics, so
            # the rounding order differs between runs)
            assert d_ab <= 1e-9
            assert d_or <= 1e-9
        sa, sb = a.tcf_get_stats(), b.tcf_get_stats()
        assert abs(sa["total_pcg_iters"] - sb["total_pcg_iters"]) <= prob.n_steps


def test_noalloc_interleaved_with_tcf_step():
    """One handle: noalloc, regular (captures its graph), noalloc again."""
    prob = W.plain_fp64().with_steps(3)
    ref = solve.run(prob)
    p = tcf.Problem(prob)
    p.tcf_setup()
    for l, fn in enumerate((p.tcf_step_noalloc, p.tcf_step, p.tcf_step_noalloc)):
        fn(1)
        f = np.array(p.tcf_get_field(0), copy=True)
        e = _rel(f, ref.fields[l][:, 0])
        print(f"[noalloc] interleaved step {l}: vs oracle {e:.2e}", flush=True)
        assert e <= 1e-9
    with pytest.raises(tcf.TcfError) as err:
        tcf.Problem(prob).tcf_step_noalloc(1)
    assert err.value.code == tcf.TCF_ESTATE
