"""Oracle Gauss-Lobatto grid (App. C.1, Lobatto: poles plus the zeros of
P'_{n-1}), pinned by textbook rules and by its exactness degree 2n - 3."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _node(expr):
    if expr.startswith("-sqrt("):
        return -math.sqrt(float(Fraction(expr[6:-1])))
    if expr.startswith("sqrt("):
        return math.sqrt(float(Fraction(expr[5:-1])))
    return float(Fraction(expr))


def test_golden_rules():
    rows = {}
    with open(os.path.join(HERE, "golden", "lobatto_rules.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, x, w = line.split()
                rows.setdefault(int(n), []).append((_node(x), float(Fraction(w))))
    assert sorted(rows) == [3, 4, 5]
    for n, pts in rows.items():
        x, w = O.gauss_lobatto(n)
        np.testing.assert_allclose(x, [p[0] for p in pts], atol=1e-15)
        np.testing.assert_allclose(w, [p[1] for p in pts], rtol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 7, 16, 33, 90, 181])
def test_exactness_degree(n):
    x, w = O.gauss_lobatto(n)
    assert x[0] == 1.0 and x[-1] == -1.0 and np.all(np.diff(x) < 0)
    # interior nodes are the zeros of P'_{n-1}
    dP = npleg.legder(np.eye(n)[n - 1])
    assert np.abs(npleg.legval(x[1:-1], dP)).max() < 1e-10 * n * n
    # exact for x^k, k <= 2n - 3
    for k in range(0, 2 * n - 2, 2):
        assert (w * x ** k).sum() == pytest.approx(2.0 / (k + 1), rel=1e-12, abs=1e-14), k
    # not at degree 2n - 2: P_{n-1}^2 integrates to 2/(2n-1), the rule gives
    # 2/(n-1) (w_j P_{n-1}(x_j)^2 = 2/(n(n-1)) at every node)
    P = npleg.legval(x, np.eye(n)[n - 1])
    assert (w * P * P).sum() == pytest.approx(2.0 / (n - 1), rel=1e-11)
    assert abs((w * P * P).sum() - 2.0 / (2 * n - 1)) > 0.5 / n


def test_lobatto_grid_heat_operator_is_the_dense_kernel():
    g = O.make_grid("lob", 17, 34, 16)
    rng = np.random.default_rng(2)
    v = rng.standard_normal((2, g.nlat, g.nlon))
    t = 3e-3
    np.testing.assert_allclose(O.heat_apply(v, g, t), O.dense_heat_apply(v, g, t), rtol=0,
                               atol=1e-13 * np.abs(v).max())
