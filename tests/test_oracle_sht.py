"""Pins for the oracle's Legendre functions, SHT and HeatConv (Sec. 3.2, App. B, Prop. 3.4).

Closed forms and library routines that fix the operator without re-typing it:
scipy's spherical harmonics, orthonormality, the Y_lm eigen-relation
HeatConv(Y_lm) = exp(-t l(l+1)) Y_lm, preservation of constants and mass,
self-adjointness, the semigroup law, and the dense radial-kernel identity
built from numpy's Legendre series evaluation.
"""

import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle as O


def test_legendre_against_scipy():
    L = 61
    x = np.linspace(-0.999, 0.999, 23)
    tab = O.legendre_table(L, x)
    th = np.arccos(x)
    for m in range(L):
        for l in range(m, L):
            ref = sph_harm_y(l, m, th, 0.0).real * (-1) ** m  # drop Condon-Shortley phase
            np.testing.assert_allclose(tab[m][l - m], ref, atol=1e-12, rtol=1e-11)


@pytest.mark.parametrize("L", [8, 40])
def test_legendre_orthonormal(L):
    x, w = O.gauss_legendre(L)
    tab = O.legendre_table(L, x)
    for m in range(L):
        G = 2 * np.pi * (tab[m] * w) @ tab[m].T
        np.testing.assert_allclose(G, np.eye(L - m), atol=1e-13)


def _real_Y(l, m, g):
    th = g.theta[:, None]
    ph = g.phi[None, :]
    Y = sph_harm_y(l, m, th, ph)
    return Y.real, Y.imag


@pytest.mark.parametrize("t", [1e-3, 3e-2])
def test_eigen_relation_gauss_legendre(t):
    g = O.make_grid("gl", 20, 40, 20)
    for l in range(20):
        for m in range(0, l + 1, 3 if l > 6 else 1):
            for Y in _real_Y(l, m, g):
                if np.abs(Y).max() < 1e-12:
                    continue
                out = O.heat_apply(Y, g, t)
                np.testing.assert_allclose(out, math.exp(-t * l * (l + 1)) * Y, atol=2e-13)


def test_eigen_relation_clenshaw_curtis_low_degrees():
    # With nlat CC rows the quadrature is exact for latitude polynomials of
    # degree <= nlat-1, so Y_lm is an eigenfunction for l + (L-1) <= nlat - 1.
    nlat, L = 25, 16
    g = O.make_grid("cc", nlat, 32, L)
    t = 0.01
    for l in range(nlat - L + 1):
        for m in range(l + 1):
            for Y in _real_Y(l, m, g):
                if np.abs(Y).max() < 1e-12:
                    continue
                np.testing.assert_allclose(O.heat_apply(Y, g, t), math.exp(-t * l * (l + 1)) * Y,
                                           atol=1e-13)
    # and at the band limit it is not (the CC forward transform is inexact there)
    Y, _ = _real_Y(L - 1, 0, g)
    assert np.abs(O.heat_apply(Y, g, t) - math.exp(-t * (L - 1) * L) * Y).max() > 1e-6


@pytest.mark.parametrize("kind,nlat,nlon,L", [("gl", 16, 32, 16), ("cc", 21, 40, 20),
                                              ("gl", 13, 25, 13), ("cc", 8, 16, 6)])
def test_constants_mass_selfadjoint(kind, nlat, nlon, L):
    g = O.make_grid(kind, nlat, nlon, L)
    rng = np.random.default_rng(1)
    t = 2e-3
    one = np.ones((nlat, nlon))
    np.testing.assert_allclose(O.heat_apply(one, g, t), one, atol=1e-13)
    x = rng.random((nlat, nlon))
    y = rng.random((nlat, nlon))
    a = g.area
    Kx = O.heat_apply(x, g, t)
    Ky = O.heat_apply(y, g, t)
    assert abs((a * Kx).sum() - (a * x).sum()) < 1e-13
    assert abs((a * x * Ky).sum() - (a * Kx * y).sum()) < 1e-13
    # plain transpose: <x, K y> = <K^T x, y>
    KTx = O.heat_apply(x, g, t, transpose=True)
    assert abs((x * Ky).sum() - (KTx * y).sum()) < 1e-12


def test_semigroup_gauss_legendre():
    g = O.make_grid("gl", 24, 48, 24)
    v = np.random.default_rng(2).random((24, 48))
    a = O.heat_apply(O.heat_apply(v, g, 1e-3), g, 4e-3)
    b = O.heat_apply(v, g, 5e-3)
    np.testing.assert_allclose(a, b, atol=1e-13)


@pytest.mark.parametrize("kind,nlat,nlon,L,t", [("gl", 16, 32, 16, 1e-2), ("gl", 32, 64, 32, 1e-2),
                                                ("cc", 33, 64, 32, 1e-3), ("cc", 17, 31, 16, 5e-2),
                                                ("gl", 15, 36, 12, 1e-1)])
def test_dense_kernel_identity(kind, nlat, nlon, L, t):
    g = O.make_grid(kind, nlat, nlon, L)
    v = np.random.default_rng(3).standard_normal((2, nlat, nlon))
    d = O.dense_heat_apply(v, g, t)
    s = O.heat_apply(v, g, t)
    assert np.abs(d - s).max() <= 1e-13 * np.abs(d).max()


def test_heat_multipliers():
    h = O.heat_multipliers(5, 0.1)
    np.testing.assert_allclose(h, np.exp(-0.1 * np.array([0, 2, 6, 12, 20])), rtol=1e-15)


def test_analysis_synthesis_roundtrip_bandlimited():
    # a band-limited field is reproduced exactly on a Gauss-Legendre grid
    g = O.make_grid("gl", 12, 24, 12)
    rng = np.random.default_rng(4)
    c = [rng.standard_normal(12 - m) + 1j * rng.standard_normal(12 - m) for m in range(12)]
    c[0] = c[0].real + 0j
    f = O.synthesis(c, g)
    c2 = O.analysis(f, g)
    for m in range(12):
        np.testing.assert_allclose(c2[m], c[m], atol=1e-13)
