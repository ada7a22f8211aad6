"""The two configurations beyond the oracle's direct solve, at full size on
one GPU, checked against the oracle's discretisation.

* Largest single problem: box [0,2]x[0,2]x[0,1], 8x8x4 patches of 0.25^3,
  p = 3, 12 elements per direction, conductor/insulator checkerboard, 32
  excitations: 2,157,848 edges, 1,776,280 gauged unknowns, 124,800
  multipliers, 115,608 primal unknowns.
* Mixed precision: 4x4x4 patches, p = 3, n = 10, floating central
  conductor: 229,897 gauged unknowns, in both FP32 operator modes.

The fields of the checked excitations after each of the first two steps
satisfy the oracle's patch-by-patch residual of the implicit Euler system
(oracle/residual.py, computed on the host in worker processes):
||f_K - (W a)_K|| / ||f_K|| <= 1e-8, the bar of the full-size residual
checks (at reduced sizes, where the oracle's field exists, this residual
level goes with field errors below 1e-9).
"""
import numpy as np
import pytest

from oracle import residual
from paper_2510_23446_amd import tcf
from tests.fullsize_residual import oracle_side

pytestmark = pytest.mark.gpu

STEPS = 2
CASES = {
    "largest": dict(ks=(0, 17), counts=(2157848, 1776280, 124800, 115608)),
    "mixed": dict(ks=(0,), counts=(None, 229897, 22044, None)),
}
_SIDE = {}


def _side(name):
    if name not in _SIDE:
        _SIDE[name] = oracle_side(name, STEPS, CASES[name]["ks"])
    return _SIDE[name]


def _check(name, prec):
    prob, grid, kept, ops, keys, loads = _side(name)
    ks = CASES[name]["ks"]
    p = tcf.Problem(prob, precision=prec)
    c = p.counts()
    for want, got in zip(CASES[name]["counts"],
                         (c["n_edges"], c["n_kept"], c["n_lambda"], c["n_primal"])):
        assert want is None or want == got
    p.tcf_setup()
    st = p.tcf_get_stats()
    print(f"[full size] {name} {prec}: setup {st['setup_ms'] / 1e3:.1f} s, "
          f"{st['setup_chunks']} patch groups, coarse factor {st['coarse_nodes']} nodes, "
          f"device peak {st['device_bytes_peak'] / 2**30:.1f} GiB", flush=True)
    prev = {k: np.zeros(grid.n_edges) for k in ks}
    for l in range(STEPS):
        p.tcf_step(1)
        for j, k in enumerate(ks):
            a = p.tcf_get_field(k)
            r = residual.step_residual(prob, grid, kept, ops, keys,
                                       [L[:, j] for L in loads], prev[k], a, prob.amp[k, l])
            print(f"[full size] {name} {prec} step {l} excitation {k}: residual {r:.3e}",
                  flush=True)
            assert r <= 1e-8, r
            prev[k] = a
    assert p.tcf_get_stats()["nonconverged_steps"] == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_largest_full_size_residual(prec):
    _check("largest", prec)


@pytest.mark.parametrize("prec", ["fp32_ir", "fp32_full_ir"])
def test_mixed_full_size_residual(prec):
    _check("mixed", prec)
