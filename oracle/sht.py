"""Semi-naive spherical harmonic transform and HeatConv (oracle; test infrastructure only).

Sec. 3.2 ("Algorithm" paragraph) defines
    HeatConv(v; {h_l}) = F^{-1}( {h_l} (.) F(v) ),   h_l = exp(-t l (l+1)),
with the SHT F taken as in App. B (f_lm = <f, Y_lm>) and evaluated on a grid by
the semi-naive algorithm of App. C.1: an FFT along each latitude row, then, per
order m, a projection onto P̄_l^m(x_j) weighted by the quadrature.  Only
degrees l < L and orders |m| < L are kept (Alg. 1 uses l = 0..L-1).

For real fields only m >= 0 is stored (f_{l,-m} is fixed by conjugate symmetry):
    F_m(j)   = sum_k f_{jk} e^{-2 pi i m k / nlon}            (numpy rfft)
    f_lm     = (2 pi / nlon) sum_j w_j P̄_l^m(x_j) F_m(j)
    G_m(j)   = sum_l c_lm P̄_l^m(x_j)
    g_{jk}   = G_0(j) + 2 Re sum_{m>=1} G_m(j) e^{2 pi i m k / nlon}
Arrays carry any leading batch dimensions: f has shape (..., nlat, nlon).
HEALPix grids (pseudo-spectral, per-ring longitude sums) are handled in
``healpix``; their fields have shape (..., 1, Npix).
"""

import numpy as np

from . import healpix
from .legendre import legendre_table


def _table(grid):
    tab = getattr(grid, "_oracle_plm", None)
    if tab is None:
        tab = legendre_table(grid.L, grid.x)
        grid._oracle_plm = tab
    return tab


def heat_multipliers(L, t):
    """h_l = exp(-t l (l+1)) for l = 0..L-1 (Alg. 1, second step)."""
    l = np.arange(L, dtype=np.float64)
    return np.exp(-t * l * (l + 1.0))


def analysis(f, grid):
    """Forward SHT.  Returns a list over m of complex arrays (..., L-m) holding f_lm, l = m..L-1."""
    if grid.kind == "hp":
        return healpix.analysis(f, grid)
    f = np.asarray(f, dtype=np.float64)
    F = np.fft.rfft(f, axis=-1)
    wq = grid.w * (2.0 * np.pi / grid.nlon)
    tab = _table(grid)
    out = []
    for m in range(grid.L):
        y = F[..., :, m] * wq                      # (..., nlat)
        out.append((y.real @ tab[m].T) + 1j * (y.imag @ tab[m].T))   # (..., L-m)
    return out


def synthesis(coeffs, grid):
    """Inverse SHT of a list over m of (..., L-m) coefficient arrays; returns (..., nlat, nlon)."""
    if grid.kind == "hp":
        return healpix.synthesis(coeffs, grid)
    tab = _table(grid)
    lead = coeffs[0].shape[:-1]
    G = np.zeros(lead + (grid.nlat, grid.nlon // 2 + 1), dtype=np.complex128)
    for m in range(grid.L):
        c = np.asarray(coeffs[m])
        G[..., :, m] = (c.real @ tab[m]) + 1j * (c.imag @ tab[m])
    return np.fft.irfft(G, n=grid.nlon, axis=-1) * grid.nlon


def heat_apply(v, grid, t, transpose=False):
    """HeatConv(v) = F^{-1}(h (.) F(v)) on the grid; h_l = exp(-t l(l+1)).

    transpose=True applies the transpose of the matrix of this linear map,
    x -> a (.) HeatConv(x / a), where a are the area weights (the map is
    self-adjoint in the a-weighted inner product, so its plain transpose is this).
    """
    v = np.asarray(v, dtype=np.float64)
    a = grid.area
    if transpose:
        v = v / a
    h = heat_multipliers(grid.L, t)
    c = analysis(v, grid)
    c = [cm * h[m:] for m, cm in enumerate(c)]
    out = synthesis(c, grid)
    if transpose:
        out = out * a
    return out
