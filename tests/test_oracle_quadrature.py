"""Pins for the oracle's Grundmann-Moeller rule: exactness on barycentric
monomials, whose integral over the reference n-simplex is the textbook closed
form a_0! ... a_n! / (|a| + n)!."""
from itertools import product
from math import factorial

import numpy as np
import pytest

from oracle.quadrature import gm_rule


@pytest.mark.parametrize("n", [1, 2, 3])
def test_weights_sum_to_volume(n):
    _, w = gm_rule(n, 2)
    assert abs(w.sum() - 1.0 / factorial(n)) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3])
def test_points_are_barycentric(n):
    x, _ = gm_rule(n, 2)
    assert np.allclose(x.sum(1), 1.0, atol=1e-15) and np.all(x > 0)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_exact_to_degree_5(n):
    x, w = gm_rule(n, 2)
    for a in product(range(6), repeat=n + 1):
        if sum(a) > 5:
            continue
        exact = np.prod([factorial(k) for k in a]) / factorial(sum(a) + n)
        val = np.sum(w * np.prod(x ** np.array(a)[None, :], 1))
        assert abs(val - exact) < 1e-14 * max(1.0, exact), (n, a)


def test_not_exact_at_degree_6():
    x, w = gm_rule(3, 2)
    a = (6, 0, 0, 0)
    exact = factorial(6) / factorial(9)
    assert abs(np.sum(w * x[:, 0] ** 6) - exact) > 1e-8
