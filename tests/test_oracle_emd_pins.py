"""Pins for the oracle's EMD (Sec. 4.2) and its Sinkhorn approximation.

Sources of truth: SciPy's independent assignment solver (for equal set sizes
the uniform transport problem has an optimal permutation plan, so EMD is the
minimum-cost matching divided by m), closed forms (one point each, identical
sets), the metric axioms the paper relies on, the paper's bound CH <= EMD, and
the convergence of entropic transport to the exact optimum as eps shrinks.
"""
import numpy as np
from scipy.optimize import linear_sum_assignment

from oracle import emd as oe


def _unit(rng, n, d=16):
    x = rng.standard_normal((n, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def test_equal_sizes_match_the_assignment_solver():
    rng = np.random.default_rng(0)
    for m in (1, 3, 7, 12):
        A, B = _unit(rng, m), _unit(rng, m)
        C = oe.cost_matrix(A, B)
        r, c = linear_sum_assignment(C)
        assert abs(oe.emd_exact(A, B) - C[r, c].sum() / m) <= 1e-9


def test_closed_forms():
    rng = np.random.default_rng(1)
    a, b = _unit(rng, 1), _unit(rng, 1)
    d = float(np.linalg.norm(a - b))
    assert abs(oe.emd_exact(a, b) - d) <= 1e-12
    assert abs(oe.sinkhorn(a, b, 0.1, 3) - d) <= 1e-12           # a single entry carries all the mass
    A = _unit(rng, 9)
    assert oe.emd_exact(A, A) <= 1e-9
    # one point against m: every unit of mass travels from it
    B = _unit(rng, 5)
    assert abs(oe.emd_exact(a, B) - np.linalg.norm(B - a, axis=1).mean()) <= 1e-9


def test_metric_axioms_and_the_chamfer_bound():
    rng = np.random.default_rng(2)
    for _ in range(6):
        A, B, C = _unit(rng, rng.integers(1, 8)), _unit(rng, rng.integers(1, 8)), _unit(rng, rng.integers(1, 8))
        ab, ba = oe.emd_exact(A, B), oe.emd_exact(B, A)
        assert abs(ab - ba) <= 1e-9                                      # symmetry
        assert ab <= oe.emd_exact(A, C) + oe.emd_exact(C, B) + 1e-9     # triangle inequality
        assert oe.chamfer_distance(A, B) <= ab + 1e-12                  # CH <= EMD (Sec. 4.2)


def test_sinkhorn_converges_to_the_exact_transport():
    rng = np.random.default_rng(3)
    A, B = _unit(rng, 6), _unit(rng, 9)
    exact = oe.emd_exact(A, B)
    prev = None
    for eps in (0.5, 0.1, 0.02):
        s, T = oe.sinkhorn(A, B, eps, 3000, return_plan=True)
        np.testing.assert_allclose(T.sum(axis=0), 1 / 9, atol=1e-12)   # the last update fixes the columns
        np.testing.assert_allclose(T.sum(axis=1), 1 / 6, atol=1e-6)
        assert s >= exact - 1e-9                                        # a feasible plan costs at least the optimum
        if prev is not None:
            assert s - exact <= prev - exact + 1e-12
        prev = s
    assert prev - exact <= 0.02 * np.log(6 * 9)
