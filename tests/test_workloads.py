"""Input generators: seeded, reproducible, and the reduced instances are true
restrictions of the full ones (no method arithmetic is involved here)."""
import numpy as np

import workloads as W


def test_largest_reduced_takes_the_first_excitations():
    full = W.largest_multirhs(n_steps=3)
    red = W.largest_multirhs(P=(4, 4, 2), n=4, n_rhs=4, n_steps=3)
    xs = np.linspace(0.05, 0.95, 5)
    for k in range(4):
        a = full.phi(xs, xs, xs, k)
        b = red.phi(xs, xs, xs, k)
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(full.amp[:4], red.amp)


def test_generators_are_seeded():
    a = W.uneven_fp64(seed=1, n_steps=2)
    b = W.uneven_fp64(seed=1, n_steps=2)
    assert a.name == b.name
    for d in range(3):
        np.testing.assert_array_equal(a.nel[d], b.nel[d])
        np.testing.assert_array_equal(a.deg[d], b.deg[d])
    np.testing.assert_array_equal(a.sigma, b.sigma)
    c = W.uneven_fp64(seed=2, n_steps=2)
    assert not all(np.array_equal(a.nel[d], c.nel[d]) for d in range(3)) or \
        not np.array_equal(a.sigma, c.sigma)


def test_subproblem_restricts_rows_and_materials():
    prob = W.uneven_fp64(seed=1, n_steps=2)
    sub = W.subproblem(prob, (0, 0, 0), (2, 2, 2))
    for d in range(3):
        np.testing.assert_array_equal(sub.nel[d], prob.nel[d][:2])
        np.testing.assert_array_equal(sub.deg[d], prob.deg[d][:2])
    for k in range(2):
        for j in range(2):
            for i in range(2):
                s_sub = i + 2 * (j + 2 * k)
                s_full = i + prob.np[0] * (j + prob.np[1] * k)
                assert sub.sigma[s_sub] == prob.sigma[s_full]
