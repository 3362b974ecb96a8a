"""Oracle regional attribution (Sec. 4.2.2), pinned by closed forms and invariances."""

import math

import numpy as np
import pytest

import oracle as O


def test_whole_sphere_rms_of_z_is_sqrt_one_third():
    # g = z = sin(latitude): mean 0 over the sphere and mean square 1/3
    # (integral of z^2 over S^2 is 4 pi / 3); exact on a Gauss-Legendre grid
    g = O.make_grid("gl", 12, 24, 12)
    z = np.repeat(g.x[:, None], g.nlon, axis=1)
    rms = O.regional_rms(z * g.area, g, [(-91.0, 91.0)])
    assert rms[0] == pytest.approx(math.sqrt(1.0 / 3.0), rel=1e-14)


@pytest.mark.parametrize("grid", [("gl", 16, 32, 16), ("cc", 21, 40, 20), ("hp", 4, 8)])
def test_invariances(grid):
    g = O.HealpixGrid(grid[1], grid[2]) if grid[0] == "hp" else O.make_grid(*grid)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(g.area.shape)
    bands = [(-23.5, 23.5), (-10.0, 10.0), (30.0, 60.0), (-60.0, -30.0), (66.5, 90.5)]
    base = O.regional_rms(f * g.area, g, bands)
    # constants do not matter (the field is centred); scaling scales the RMS
    np.testing.assert_allclose(O.regional_rms((f + 3.0) * g.area, g, bands), base, rtol=1e-12)
    np.testing.assert_allclose(O.regional_rms(-2.5 * f * g.area, g, bands), 2.5 * base, rtol=1e-12)
    # a constant field has zero RMS everywhere
    np.testing.assert_allclose(O.regional_rms(7.0 * g.area, g, bands), 0.0, atol=1e-12)
    # an empty band
    assert np.isnan(O.regional_rms(f * g.area, g, [(89.99, 89.995)])[0])


def test_rows_on_a_bound_are_outside_the_band():
    # 7 equiangular rows at latitudes 90, 60, 30, 0, -30, -60, -90 (exactly, up to
    # the arcsine's rounding): (30, 60) holds none of them, (29.9, 60.1) two
    g = O.make_grid("cc", 7, 12, 6)
    rng = np.random.default_rng(2)
    f = rng.standard_normal(g.area.shape)
    assert np.isnan(O.regional_rms(f * g.area, g, [(30.0, 60.0)])[0])
    assert np.isnan(O.regional_rms(f * g.area, g, [(-60.0, -30.0)])[0])
    got = O.regional_rms(f * g.area, g, [(29.9, 60.1)])[0]
    a = g.area
    mean = (a * f).sum() / a.sum()
    rows = [1, 2]
    want = math.sqrt(sum((a[j] * (f[j] - mean) ** 2).sum() for j in rows) / sum(a[j].sum() for j in rows))
    assert got == pytest.approx(want, rel=1e-13)
