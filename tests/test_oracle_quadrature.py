"""Pins for the oracle's quadratures (App. C.1 grids, App. C.2 area weights).

Pinned against: textbook closed forms (tests/golden), numpy's leggauss (a
library routine), exact polynomial moments, and a linear solve of the
Chebyshev moment equations (an independent characterisation of Clenshaw-Curtis).
"""

import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quadrature_closed_forms.txt")


def _golden():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rule, n, x, w = line.split()
            rows.setdefault((rule, int(n)), []).append((float(x), float(w)))
    return rows


def test_closed_form_rules():
    for (rule, n), pts in _golden().items():
        x, w = O.gauss_legendre(n) if rule == "gl" else O.clenshaw_curtis(n)
        np.testing.assert_allclose(x, [p[0] for p in pts], atol=1e-15)
        np.testing.assert_allclose(w, [p[1] for p in pts], rtol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 7, 32, 90, 181, 360])
def test_gauss_legendre_matches_numpy(n):
    x, w = O.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr[::-1], atol=2e-15)
    np.testing.assert_allclose(w, wr[::-1], rtol=1e-10, atol=1e-16)  # numpy loses ~n*1e-14 on the smallest weights
    assert np.all(np.diff(x) < 0)  # north to south


@pytest.mark.parametrize("n", [8, 33])
def test_gauss_legendre_exact_degree(n):
    x, w = O.gauss_legendre(n)
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13
    # and not exact at degree 2n: the nodes are the roots of P_n, so the rule
    # gives 0 for P_n^2 whose integral is 2/(2n+1)
    Pn = np.polynomial.legendre.legval(x, [0] * n + [1])
    assert np.abs(Pn).max() < 1e-13


@pytest.mark.parametrize("n", [3, 4, 9, 16, 33, 65])
def test_clenshaw_curtis_moments(n):
    x, w = O.clenshaw_curtis(n)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_allclose(x[0], 1.0)
    np.testing.assert_allclose(x[-1], -1.0)
    for k in range(n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("n", [5, 12, 31, 64])
def test_clenshaw_curtis_against_moment_solve(n):
    # CC weights are the unique weights on the nodes cos(j pi/(n-1)) that
    # integrate T_0..T_{n-1} exactly; solve that system directly.
    th = np.pi * np.arange(n) / (n - 1)
    V = np.array([np.cos(k * th) for k in range(n)])
    mom = np.array([2.0 / (1.0 - k * k) if k % 2 == 0 else 0.0 for k in range(n)])
    wref = np.linalg.solve(V, mom)
    _, w = O.clenshaw_curtis(n)
    np.testing.assert_allclose(w, wref, rtol=1e-11, atol=1e-14)


def test_area_weights_sum():
    for kind, nlat, nlon, L in [("gl", 32, 64, 32), ("cc", 33, 64, 32), ("gl", 17, 35, 18)]:
        g = O.make_grid(kind, nlat, nlon, L)
        assert abs(g.area.sum() - 4 * np.pi) < 1e-12
        # symmetric about the equator (used by the folded HIP kernels)
        np.testing.assert_allclose(g.w, g.w[::-1], rtol=1e-13)
        np.testing.assert_allclose(g.x, -g.x[::-1], atol=1e-15)


def test_bandlimit_rule():
    with pytest.raises(ValueError):
        O.make_grid("gl", 8, 14, 8)
