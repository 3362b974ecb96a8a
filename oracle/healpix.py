"""HEALPix grid and its pseudo-spectral SHT (oracle; test infrastructure only).

Sec. 3.3 and App. C.1 name the HEALPix grid (Gorski et al. 2005): 12 Nside^2
equal-area pixels whose centres lie on 4 Nside - 1 iso-latitude rings, with no
exact quadrature, so the transform is pseudo-spectral: the analysis is the
area-weighted sum over pixels (every pixel has area 4 pi / Npix).

Ring geometry (rings numbered i = 1 .. 4 Nside - 1 from the north, RING pixel
order, pixel k of a ring at longitude phi0_i + 2 pi k / N_i):
  north polar cap, i < Nside:   z = 1 - i^2 / (3 Nside^2),  N_i = 4 i,
                                phi0 = pi / (4 i);
  equatorial belt, Nside <= i <= 3 Nside:
                                z = 4/3 - 2 i / (3 Nside),  N_i = 4 Nside,
                                phi0 = s pi / (4 Nside), s = (i - Nside + 1) mod 2
                                (rings alternate between a pixel at phi = 0 and a
                                half-pixel shift; RING order starts each ring at
                                its smallest longitude >= 0);
  south polar cap, i > 3 Nside: the mirror of ring 4 Nside - i (z -> -z,
                                same N and phi0).

The SHT is written from its definition, f_lm = sum_pixels a f(x) conj(Y_lm(x))
and f(x) = sum_lm f_lm Y_lm(x) (App. B), with Y_lm(theta, phi) = P̄_l^m(cos
theta) e^{i m phi}: per ring the longitude sum is taken directly over the ring's
pixels (no FFT), then projected on P̄_l^m(z_i).  Fields have shape
(..., 1, Npix): one "row" holding every pixel in RING order, so that the
Sinkhorn code's sums over the last two axes cover the whole sphere.
"""

import numpy as np

from .legendre import legendre_table


def ring_geometry(nside):
    """Per ring (north to south): z, number of pixels, longitude of pixel 0."""
    n = int(nside)
    z, npix, phi0 = [], [], []
    for i in range(1, 4 * n):
        ii = i if i <= 2 * n else 4 * n - i     # mirror index into the northern half
        if ii < n:
            zi = 1.0 - ii * ii / (3.0 * n * n)
            ni = 4 * ii
            p0 = np.pi / (4.0 * ii)
        else:
            zi = 4.0 / 3.0 - 2.0 * ii / (3.0 * n)
            ni = 4 * n
            s = (ii - n + 1) % 2
            p0 = s * np.pi / (4.0 * n)
        z.append(zi if i <= 2 * n else -zi)
        npix.append(ni)
        phi0.append(p0)
    return np.array(z), np.array(npix, dtype=np.int64), np.array(phi0)


class HealpixGrid:
    """HEALPix grid with band limit L (degrees and orders l, m < L)."""

    kind = "hp"

    def __init__(self, nside, L):
        self.nside = int(nside)
        self.L = int(L)
        self.x, self.ring_npix, self.ring_phi0 = ring_geometry(self.nside)
        self.nring = self.x.size
        self.npix = 12 * self.nside * self.nside
        self.ring_start = np.concatenate([[0], np.cumsum(self.ring_npix)[:-1]])

    @property
    def n(self):
        return self.npix

    @property
    def field_shape(self):
        return (1, self.npix)

    @property
    def pixel_phi(self):
        return np.concatenate([self.ring_phi0[i] + 2.0 * np.pi * np.arange(self.ring_npix[i]) / self.ring_npix[i]
                               for i in range(self.nring)])

    @property
    def pixel_z(self):
        return np.repeat(self.x, self.ring_npix)

    @property
    def area(self):
        """Equal pixel areas 4 pi / Npix, shape (1, Npix)."""
        return np.full((1, self.npix), 4.0 * np.pi / self.npix)

    def points(self):
        """Cartesian unit vectors of the pixel centres, shape (1, Npix, 3)."""
        z = self.pixel_z
        s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        ph = self.pixel_phi
        return np.stack([np.cos(ph) * s, np.sin(ph) * s, z], axis=-1)[None]


def _table(grid):
    tab = getattr(grid, "_oracle_plm", None)
    if tab is None:
        tab = legendre_table(grid.L, grid.x)
        grid._oracle_plm = tab
    return tab


def _ring_phases(grid, i):
    """e^{i m phi} for the pixels of ring i and m = 0..L-1, shape (N_i, L)."""
    ph = grid.ring_phi0[i] + 2.0 * np.pi * np.arange(grid.ring_npix[i]) / grid.ring_npix[i]
    return np.exp(1j * np.outer(ph, np.arange(grid.L)))


def analysis(f, grid):
    """f_lm = sum_pixels a f conj(Y_lm); list over m of (..., L-m) complex arrays."""
    f = np.asarray(f, dtype=np.float64)
    lead = f.shape[:-2]
    f = f.reshape(lead + (grid.npix,))
    a = 4.0 * np.pi / grid.npix
    tab = _table(grid)
    # F[..., i, m] = sum_k a f_ik e^{-i m phi_ik}
    F = np.empty(lead + (grid.nring, grid.L), dtype=np.complex128)
    for i in range(grid.nring):
        s0, ni = grid.ring_start[i], grid.ring_npix[i]
        F[..., i, :] = a * (f[..., s0:s0 + ni] @ np.conj(_ring_phases(grid, i)))
    out = []
    for m in range(grid.L):
        y = F[..., :, m]
        out.append((y.real @ tab[m].T) + 1j * (y.imag @ tab[m].T))
    return out


def synthesis(coeffs, grid):
    """f(x) = sum_{l, |m| < L} f_lm Y_lm(x) for a real field (f_{l,-m} = conj f_lm); (..., 1, Npix)."""
    tab = _table(grid)
    lead = coeffs[0].shape[:-1]
    G = np.zeros(lead + (grid.nring, grid.L), dtype=np.complex128)
    for m in range(grid.L):
        c = np.asarray(coeffs[m])
        G[..., :, m] = (c.real @ tab[m]) + 1j * (c.imag @ tab[m])
    out = np.empty(lead + (grid.npix,))
    wm = np.where(np.arange(grid.L) == 0, 1.0, 2.0)      # m = 0 once, m > 0 with its conjugate
    for i in range(grid.nring):
        s0, ni = grid.ring_start[i], grid.ring_npix[i]
        out[..., s0:s0 + ni] = ((G[..., i, :] * wm) @ _ring_phases(grid, i).T).real
    return out.reshape(lead + (1, grid.npix))
