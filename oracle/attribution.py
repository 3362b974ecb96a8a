"""Regional attribution of a divergence gradient (oracle; test infrastructure only).

Sec. 4.2.2: the gradient of the divergence with respect to a measure is a
signed field g on the sphere, defined by the potentials up to an additive
constant, so it is centred by subtracting its area-weighted mean; the
area-weighted RMS of the centred field over a latitude band is that band's
bias index.  Here g = dS_dp / a, dS_dp being the derivative with respect to
the density array (it carries the point areas a).  A point belongs to the band
(lat_lo, lat_hi) when its latitude lies strictly between the bounds; a
latitude within EDGE degrees of a bound counts as lying on it (equiangular
rows sit exactly on bounds such as 30 degrees, where the last bit of the
arcsine would otherwise decide membership).
"""

import numpy as np

EDGE = 1e-9   # degrees


def latitudes(grid):
    """Latitude in degrees of every point, shaped like a field."""
    lat_row = np.degrees(np.arcsin(np.clip(grid.x, -1.0, 1.0)))
    if grid.kind == "hp":
        return np.repeat(lat_row, grid.ring_npix)[None]
    return np.repeat(lat_row[:, None], grid.nlon, axis=1)


def regional_rms(dS_dp, grid, bands):
    """bands: list of (lat_lo, lat_hi); returns the RMS per band (NaN for an empty band)."""
    a = grid.area
    d = np.asarray(dS_dp, dtype=np.float64).reshape(a.shape)
    g = d / a
    gc = g - (a * g).sum() / a.sum()
    lat = latitudes(grid)
    out = []
    for lo, hi in bands:
        m = (lat > lo + EDGE) & (lat < hi - EDGE)
        w = a[m]
        out.append(np.sqrt((w * gc[m] ** 2).sum() / w.sum()) if w.size else np.nan)
    return np.array(out)
