"""Pins of the MaxVol active-set oracle: determinant identity, dominance at exit, local
optimality by brute force on tiny matrices, the one-column closed form, row conservation."""
import itertools

import numpy as np

from oracle.maxvol import maxvol_update


def _random(rng, n, m):
    a = np.eye(n) + 0.3 * rng.normal(size=(n, n))
    c = rng.normal(size=(m, n))
    return a, c


def test_each_swap_multiplies_the_volume_by_its_grade():
    rng = np.random.default_rng(1)
    a, c = _random(rng, 6, 40)
    a1, c1, swaps = maxvol_update(a, c, tol=1e-3)
    assert swaps
    # replay the swaps on copies and compare determinants computed from scratch
    A, C = a.copy(), c.copy()
    for i, k, g in swaps:
        d0 = np.linalg.slogdet(A)[1]
        row = A[k].copy()
        A[k], C[i] = C[i], row
        d1 = np.linalg.slogdet(A)[1]
        assert abs((d1 - d0) - np.log(abs(g))) < 1e-10
        assert abs(g) > 1.0
    np.testing.assert_array_equal(A, a1)
    np.testing.assert_array_equal(C, c1)


def test_dominance_at_exit():
    rng = np.random.default_rng(2)
    for n, m, tol in ((4, 30, 1e-3), (10, 200, 1e-2), (3, 5, 0.0)):
        a, c = _random(rng, n, m)
        a1, c1, _ = maxvol_update(a, c, tol=tol)
        assert np.max(np.abs(c1 @ np.linalg.inv(a1))) <= 1.0 + tol + 1e-12


def test_no_single_swap_grows_the_volume_at_exit_brute_force():
    rng = np.random.default_rng(3)
    for trial in range(20):
        n, m = int(rng.integers(1, 4)), int(rng.integers(2, 7))
        a, c = _random(rng, n, m)
        tol = 1e-6
        a1, c1, _ = maxvol_update(a, c, tol=tol)
        base = abs(np.linalg.det(a1))
        for i, k in itertools.product(range(m), range(n)):
            t = a1.copy()
            t[k] = c1[i]
            assert abs(np.linalg.det(t)) <= base * (1.0 + tol) + 1e-12


def test_one_column_keeps_the_largest_magnitude():
    rng = np.random.default_rng(4)
    vals = rng.permutation(np.linspace(-3.0, 2.0, 23))
    a, c = vals[:1].reshape(1, 1), vals[1:].reshape(-1, 1)
    a1, c1, _ = maxvol_update(a, c, tol=1e-6)
    assert a1[0, 0] == vals[np.argmax(np.abs(vals))]


def test_rows_are_conserved_and_grades_below_one_swap_nothing():
    rng = np.random.default_rng(5)
    a, c = _random(rng, 5, 25)
    a1, c1, swaps = maxvol_update(a, c)
    before = sorted(map(tuple, np.vstack([a, c]).round(15)))
    after = sorted(map(tuple, np.vstack([a1, c1]).round(15)))
    assert before == after
    # candidates that are combinations of active rows with coefficients below one in magnitude
    u = rng.uniform(-0.5, 0.5, size=(25, 5))
    a2, c2, swaps2 = maxvol_update(a, u @ a)
    assert swaps2 == [] and np.array_equal(a2, a)


def test_swap_limit():
    rng = np.random.default_rng(6)
    a, c = _random(rng, 8, 100)
    _, _, swaps = maxvol_update(a, c, max_swaps=2)
    assert len(swaps) == 2
