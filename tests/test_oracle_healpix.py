"""Oracle HEALPix grid and pseudo-spectral heat operator, pinned without the GPU.

* ring geometry: the published base pixels and the Nside = 2 rings
  (tests/golden/healpix_rings.txt); the equal-area identity that fixes every
  ring's z from the pixel counts; mirror symmetry;
* heat operator: the ring SHT's S diag(h) S^T diag(a) equals the dense
  radial kernel of the addition theorem on the pixel centres (numpy legval,
  independent of the oracle's associated-Legendre code), for band limits
  below and above the shortest rings' Nyquist limits;
* self-adjointness in <.,.>_a; Sinkhorn through the SHT equals Sinkhorn
  through the dense kernel.
"""

import math
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "healpix_rings.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, i, zn, zd, npix, p0 = line.split()
                rows.append((int(n), int(i), int(zn) / int(zd), int(npix), float(p0)))
    return rows


def test_golden_rings():
    rows = _golden()
    assert len(rows) == 10
    for n, i, z, npix, p0 in rows:
        zz, nn, pp = O.ring_geometry(n)
        assert zz[i - 1] == pytest.approx(z, abs=1e-15)
        assert nn[i - 1] == npix
        assert pp[i - 1] == pytest.approx(p0 * math.pi, abs=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 3, 5, 8, 16, 64])
def test_equal_area_rings(nside):
    z, npix, phi0 = O.ring_geometry(nside)
    N = 12 * nside * nside
    assert z.size == 4 * nside - 1 and npix.sum() == N
    assert np.all(np.diff(z) < 0)
    # mirror symmetry about the equator: z, pixel count and longitude offset
    np.testing.assert_allclose(z, -z[::-1], atol=1e-15)
    assert np.array_equal(npix, npix[::-1]) and np.allclose(phi0, phi0[::-1])
    # equal-area pixels: the cap above ring i's centres holds the rings above
    # it and half of ring i, so 2 pi (1 - z_i) = (pixels above + N_i / 2) 4 pi / N
    above = np.concatenate([[0], np.cumsum(npix)[:-1]])
    np.testing.assert_allclose(2 * np.pi * (1 - z), (above + npix / 2) * 4 * np.pi / N, rtol=0, atol=1e-13)
    # phi0 lies in [0, 2 pi / N_i): RING order starts at the smallest longitude >= 0
    assert np.all(phi0 >= 0) and np.all(phi0 < 2 * np.pi / npix)


@pytest.mark.parametrize("nside,L,t", [(2, 4, 1e-2), (4, 8, 1e-2), (4, 12, 3e-3), (6, 16, 1e-3)])
def test_heat_apply_matches_dense_kernel(nside, L, t):
    g = O.HealpixGrid(nside, L)
    rng = np.random.default_rng(nside * 100 + L)
    v = rng.standard_normal((3, 1, g.npix))
    K = O.dense_heat_matrix(g, t)
    got = O.heat_apply(v, g, t)
    want = O.dense_heat_apply(v, g, t, K=K)
    assert got.shape == v.shape
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_self_adjoint_and_transpose():
    g = O.HealpixGrid(5, 10)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal((2, 1, g.npix))
    t = 5e-3
    a = g.area
    lhs = (a * O.heat_apply(u, g, t) * v).sum()
    rhs = (a * u * O.heat_apply(v, g, t)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-13)
    K = O.dense_heat_matrix(g, t)
    np.testing.assert_allclose(O.heat_apply(v, g, t, transpose=True).ravel(), K.T @ v.ravel(),
                               rtol=0, atol=1e-13 * np.abs(K.T @ v.ravel()).max())


def test_sinkhorn_sht_equals_dense():
    g = O.HealpixGrid(4, 8)
    rng = np.random.default_rng(7)
    p = rng.uniform(0.5, 1.5, (1, g.npix))
    q = rng.uniform(0.5, 1.5, (1, g.npix))
    p /= (g.area * p).sum()
    q /= (g.area * q).sum()
    eps = 0.1
    Kd = O.dense_heat_matrix(g, eps / 4)
    r1 = O.sinkhorn(p, q, g, eps, T=50)
    r2 = O.sinkhorn(p, q, g, eps, T=50, K=lambda x: O.dense_heat_apply(x, g, eps / 4, K=Kd))
    assert r1["breakdown"] == 0 and r2["breakdown"] == 0
    assert r1["cost"] == pytest.approx(r2["cost"], rel=1e-11)
    np.testing.assert_allclose(r1["phi"], r2["phi"], rtol=0, atol=1e-10)
