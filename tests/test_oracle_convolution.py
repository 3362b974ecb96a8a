"""Pins of the heat-versus-matrix convolution oracle (appendix on convolution on S^2).

Each pin reaches the oracle's result by a route other than its own code:
C(eps) through the error function of a complex argument and through its
small- and large-eps expansions; the matrix convolution through a constant
field (whose image is C(eps) wherever the quadrature is exact enough), through
a discrete delta (whose image is the kernel at the haversine distance), and
through its symmetry in the area-weighted inner product; the comparison
through its limits (Varadhan's formula
makes the rescaled heat output approach the matrix output as eps shrinks on a
fine grid).
"""

import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from oracle import convolution as C
from paper_2605_18389_amd import synth

EPS8 = np.logspace(-3, 1, 8)   # eight log-spaced values in [1e-3, 10]


def _vmf(g, seed=4):
    X = g.points()
    z, phi = X[..., 2], np.arctan2(X[..., 1], X[..., 0])
    return synth.vmf_at(seed, z, phi, 10.0)[0]


def _c_erf(eps):
    # int_0^pi e^{-g^2/eps} e^{i g} dg = e^{-eps/4} sqrt(pi eps)/2 [erf((pi - i eps/2)/sqrt(eps)) - erf(-i sqrt(eps)/2)]
    z1 = (math.pi - 0.5j * eps) / math.sqrt(eps)
    z0 = -0.5j * math.sqrt(eps)
    v = math.exp(-eps / 4) * math.sqrt(math.pi * eps) / 2 * (sp.erf(z1) - sp.erf(z0))
    return 2 * math.pi * v.imag


@pytest.mark.parametrize("eps", list(EPS8) + [3e-4, 0.05, 30.0])
def test_kernel_integral_matches_complex_erf(eps):
    assert C.geodesic_kernel_integral(eps) == pytest.approx(_c_erf(eps), rel=1e-12)


def test_kernel_integral_expansions():
    # small eps: sin g = g - g^3/6 + g^5/120, int_0^inf e^{-g^2/eps} g^{2k+1} dg = k! eps^{k+1} / 2
    e = 1e-3
    small = 2 * math.pi * (e / 2 - e ** 2 / 12 + e ** 3 / 120)
    assert C.geodesic_kernel_integral(e) == pytest.approx(small, rel=1e-10)
    # large eps: e^{-g^2/eps} = sum_k (-g^2/eps)^k / k!, with I_n = int_0^pi g^n sin g dg
    # = pi^n - n (n - 1) I_{n-2} (parts twice), I_0 = 2
    E = 1e4
    I = {0: 2.0}
    for n in (2, 4, 6):
        I[n] = math.pi ** n - n * (n - 1) * I[n - 2]
    large = 2 * math.pi * (I[0] - I[2] / E + I[4] / (2 * E ** 2) - I[6] / (6 * E ** 3))
    assert C.geodesic_kernel_integral(E) == pytest.approx(large, rel=1e-12)
    # whole sphere as eps grows
    assert C.geodesic_kernel_integral(1e9) == pytest.approx(4 * math.pi, rel=1e-8)


@pytest.mark.parametrize("eps", [0.05, 0.1, 0.5])
def test_matrix_convolution_of_constant_is_kernel_integral(eps):
    g = O.make_grid("gl", 64, 128, 64)
    k = C.matrix_convolution(np.ones(g.area.shape), g, eps)
    np.testing.assert_allclose(k, C.geodesic_kernel_integral(eps), rtol=1e-11)


@pytest.mark.parametrize("grid", [("cc", 9, 16, 8), ("gl", 8, 15, 8), ("hp", 2, 4)])
def test_matrix_convolution_of_delta_is_kernel_at_haversine_distance(grid):
    g = O.HealpixGrid(grid[1], grid[2]) if grid[0] == "hp" else O.make_grid(*grid)
    a = g.area.reshape(-1)
    j0 = a.size // 3
    f = np.zeros(a.size)
    f[j0] = 1.0 / a[j0]
    eps = 0.7
    k = C.matrix_convolution(f.reshape(g.area.shape), g, eps).reshape(-1)
    X = g.points().reshape(-1, 3)
    lat = np.arcsin(np.clip(X[:, 2], -1, 1))
    lon = np.arctan2(X[:, 1], X[:, 0])
    dlat, dlon = lat - lat[j0], lon - lon[j0]
    hav = np.sin(dlat / 2) ** 2 + np.cos(lat) * np.cos(lat[j0]) * np.sin(dlon / 2) ** 2
    d = 2 * np.arcsin(np.sqrt(np.clip(hav, 0, 1)))
    np.testing.assert_allclose(k, np.exp(-d * d / eps), rtol=1e-12, atol=1e-12)


def test_matrix_convolution_is_self_adjoint_in_area_product():
    g = O.make_grid("cc", 11, 20, 10)   # unequal row weights
    rng = np.random.default_rng(3)
    f, h = rng.standard_normal((2,) + g.area.shape)
    for eps in (0.01, 0.3, 3.0):
        lhs = (g.area * h * C.matrix_convolution(f, g, eps)).sum()
        rhs = (g.area * f * C.matrix_convolution(h, g, eps)).sum()
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_heat_convolution_keeps_constants():
    # exact-quadrature grids only: HEALPix's pseudo-spectral analysis leaks a
    # constant into l > 0
    for g in (O.make_grid("cc", 17, 32, 16), O.make_grid("gl", 8, 16, 8)):
        out = C.heat_convolution(np.full(g.area.shape, 2.5), g, 0.3)
        np.testing.assert_allclose(out, 2.5, rtol=1e-12)


def test_rescaled_heat_approaches_matrix_convolution():
    """Error falls with the band limit at small eps and is larger at large eps;
    on a fine grid and small eps the two outputs agree to a small fraction of their size."""
    errs = []
    for L in (8, 16, 32):
        g = O.make_grid("cc", L + 1, 2 * L, L)
        f = _vmf(g)
        errs.append(C.heat_vs_matrix(f, g, EPS8))
    errs = np.array(errs)
    for e in range(3):               # eps = 1e-3 .. 1.4e-2: resolution-limited
        assert errs[0, e] > errs[1, e] > errs[2, e]
    assert np.all(errs[:, -1] > 10 * errs[:, 3])   # eps = 10 far worse than eps = 5e-2
    g = O.make_grid("cc", 33, 64, 32)
    km = C.matrix_convolution(_vmf(g), g, EPS8[2])
    assert errs[2, 2] < 1e-3 * np.abs(km).mean()
