"""ctypes binding of libshot (include/shot.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of libshot.so.  PyTorch provides device memory and the current stream.  If
the shared library has not been built, loading fails loudly -- there is no
CPU fallback.
"""

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshot.so")

GRID_GAUSS_LEGENDRE = 0
GRID_CLENSHAW_CURTIS = 1
GRID_HEALPIX = 2
GRID_LOBATTO = 3
FP64, FP32, BF16_MFMA, BF16X3_MFMA = 0, 1, 2, 3
LEG_AUTO, LEG_TABLE, LEG_RECURRENCE = 0, 1, 2

OK = 0
E_INVALID = 1
E_NOMEM = 2
E_HIP = 3
E_UNSUPPORTED = 4
W_NOT_CONVERGED = 16
E_BREAKDOWN = 17

_PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16_MFMA, "bf16_mfma": BF16_MFMA, "bf16x3": BF16X3_MFMA}
_LEG = {"auto": LEG_AUTO, "table": LEG_TABLE, "recurrence": LEG_RECURRENCE}
_KIND = {"gl": GRID_GAUSS_LEGENDRE, "gauss_legendre": GRID_GAUSS_LEGENDRE,
         "cc": GRID_CLENSHAW_CURTIS, "clenshaw_curtis": GRID_CLENSHAW_CURTIS,
         "equiangular": GRID_CLENSHAW_CURTIS, "hp": GRID_HEALPIX, "healpix": GRID_HEALPIX,
         "lob": GRID_LOBATTO, "lobatto": GRID_LOBATTO}

# Every entry point declared in include/shot.h.
EXPORTS = [
    "shot_sht_plan", "shot_plan_destroy", "shot_plan_grid", "shot_sht_analysis",
    "shot_sht_synthesis", "shot_heat_apply", "shot_sinkhorn_solve", "shot_sinkhorn_divergence",
    "shot_sinkhorn_divergence_grad", "shot_profile_enable", "shot_profile_read",
    "shot_status_string", "shot_last_error", "shot_plan_set_tuning", "shot_plan_get_tuning",
    "shot_autotune", "shot_plan_set_graphs", "shot_plan_ring", "shot_gradient_regional_rms",
    "shot_plan_area_weights", "shot_build_id", "shot_heat_apply_noalloc",
]

# The five latitude bands of the regional attribution (Sec. 4.2.2), degrees,
# bounds exclusive: Tropics |lat| < 23.5, ITCZ |lat| < 10, NH and SH
# midlatitudes 30-60, Arctic > 66.5 N (the upper bound admits a pole row).
PAPER_REGIONS = {"tropics": (-23.5, 23.5), "itcz": (-10.0, 10.0), "nh_midlatitudes": (30.0, 60.0),
                 "sh_midlatitudes": (-60.0, -30.0), "arctic": (66.5, 90.5)}


class GridDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nlat", ctypes.c_int32), ("nlon", ctypes.c_int32),
                ("L", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("tau", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("err", ctypes.c_double), ("iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("breakdown_iter", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kratio", ctypes.c_double)]


class ShotError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        detail = ""
        if code == E_HIP or code == E_NOMEM:
            try:
                detail = " -- " + load_library().shot_last_error().decode()
            except Exception:
                pass
        super().__init__(f"{fn} failed: {status_string(code)} ({code}){detail}")


_lib = None


def load_library(path=None):
    """Load libshot.so (once).  Raises if it is missing: no fallback exists."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libshot.so is not built ({path}); run `python -m paper_2605_18389_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname; load it first so
    # that libshot binds to that one runtime and shares torch's device memory
    # and streams (a second runtime loaded ahead of torch does not see the GPU).
    _torch()
    lib = ctypes.CDLL(path)
    lib.shot_build_id.argtypes = []
    lib.shot_build_id.restype = ctypes.c_char_p
    if path == LIB_PATH:
        from .build import source_hash
        built, want = lib.shot_build_id().decode(), source_hash()
        if built != want:
            raise RuntimeError(f"libshot.so was built from other sources (build id {built}, sources {want}); "
                               f"rebuild with `python -m paper_2605_18389_amd.build`")
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "shot_sht_plan": [ctypes.POINTER(vp), ctypes.POINTER(GridDesc), i32, i32, i32, vp],
        "shot_plan_destroy": [vp],
        "shot_plan_grid": [vp, i32, dp, dp],
        "shot_plan_ring": [vp, i32, ip, dp],
        "shot_plan_area_weights": [vp, i32, dp],
        "shot_gradient_regional_rms": [vp, ip, i32, vp, dp, i32, dp, vp],
        "shot_sht_analysis": [vp, ip, i32, vp, vp, vp],
        "shot_sht_synthesis": [vp, ip, i32, vp, vp, vp],
        "shot_heat_apply": [vp, ip, i32, dp, vp, vp, i32, vp],
        "shot_heat_apply_noalloc": [vp, ip, i32, dp, vp, vp, i32, vp],
        "shot_sinkhorn_solve": [vp, ip, i32, ctypes.POINTER(Params), vp, vp, vp, vp,
                                ctypes.POINTER(SolveInfo), vp],
        "shot_sinkhorn_divergence": [vp, ip, i32, ctypes.POINTER(Params), vp, vp, dp,
                                     ctypes.POINTER(SolveInfo), vp],
        "shot_sinkhorn_divergence_grad": [vp, ip, i32, ctypes.POINTER(Params), vp, vp, dp, vp, i32,
                                          i32, ctypes.POINTER(SolveInfo), vp],
        "shot_profile_enable": [vp, i32],
        "shot_plan_set_tuning": [vp, i32, i32, i32],
        "shot_plan_get_tuning": [vp, i32, ip, ip],
        "shot_autotune": [vp, i32, i32, vp],
        "shot_plan_set_graphs": [vp, i32],
        "shot_profile_read": [vp, i32, ctypes.POINTER(ctypes.c_int64), dp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.shot_status_string.argtypes = [i32]
    lib.shot_status_string.restype = ctypes.c_char_p
    lib.shot_last_error.argtypes = []
    lib.shot_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(code):
    try:
        return load_library().shot_status_string(int(code)).decode()
    except Exception:
        return str(code)


def _check(fn, code, allow=(OK,)):
    if code not in allow:
        raise ShotError(fn, code)
    return code


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _i32_array(vals):
    a = (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])
    return a


def _grid_tuple(g):
    """(kind, nlat, nlon, L); ("hp", nside, L) expands to ("hp", 4 nside - 1, 4 nside, L)."""
    kind = g[0]
    code = _KIND[kind] if isinstance(kind, str) else int(kind)
    if code == GRID_HEALPIX and len(g) == 3:
        nside = int(g[1])
        return (kind, 4 * nside - 1, 4 * nside, int(g[2]))
    return (kind, int(g[1]), int(g[2]), int(g[3]))


class Plan:
    """A libshot plan for one or more grids.

    grids: list of (kind, nlat, nlon, L) with kind "gl", "cc" or "lob", or ("hp", nside, L) for a
    HEALPix grid (stored as ("hp", 4 nside - 1, 4 nside, L): rings, longest ring, L).
    precision: "fp64", "fp32", "bf16" (bfloat16 Legendre operands, float32 accumulation) or
    "bf16x3" (split bfloat16 operands, three products per term; recurrence Legendre only).
    legendre: "auto", "table" (P̄ streamed from HBM) or "recurrence" (generated in float64).
    """

    def __init__(self, grids, precision="fp32", legendre="auto"):
        self.lib = load_library()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libshot needs a ROCm GPU")
        self.grids = [_grid_tuple(g) for g in grids]
        self.precision = precision
        self.prec_code = _PREC[precision]
        self.dtype = torch.float64 if self.prec_code == FP64 else torch.float32
        arr = (GridDesc * len(self.grids))(*[GridDesc(_KIND[k] if isinstance(k, str) else int(k), a, b, c)
                                              for k, a, b, c in self.grids])
        h = ctypes.c_void_p()
        _check("shot_sht_plan", self.lib.shot_sht_plan(ctypes.byref(h), arr, len(self.grids), self.prec_code,
                                                       _LEG[legendre], _stream_ptr()))
        self.handle = h
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.shot_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ grid
    def grid_nodes(self, grid=0):
        nlat = self.grids[grid][1]
        x = np.zeros(nlat)
        w = np.zeros(nlat)
        _check("shot_plan_grid", self.lib.shot_plan_grid(
            self.handle, grid, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return x, w

    def is_healpix(self, grid=0):
        k = self.grids[grid][0]
        return (_KIND[k] if isinstance(k, str) else int(k)) == GRID_HEALPIX

    def ring_layout(self, grid=0):
        """Points per row (ring) and the longitude of each row's first point."""
        nlat = self.grids[grid][1]
        npix = np.zeros(nlat, dtype=np.int32)
        phi0 = np.zeros(nlat)
        _check("shot_plan_ring", self.lib.shot_plan_ring(
            self.handle, grid, npix.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            phi0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return npix, phi0

    def pixel_coords(self, grid=0):
        """(z, phi) of every point in field order (rows, or rings in RING order)."""
        x, _ = self.grid_nodes(grid)
        npix, phi0 = self.ring_layout(grid)
        z = np.repeat(x, npix)
        phi = np.concatenate([phi0[r] + 2 * np.pi * np.arange(npix[r]) / npix[r] for r in range(len(npix))])
        return z, phi

    def area(self, grid=0):
        """Area weights of the grid's points, shaped like one field ((nlat, nlon), or (Npix,))."""
        _, nlat, nlon, _ = self.grids[grid]
        n = self.field_size(grid)
        a = np.zeros(n)
        _check("shot_plan_area_weights", self.lib.shot_plan_area_weights(
            self.handle, grid, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return a if self.is_healpix(grid) else a.reshape(nlat, nlon)

    def field_size(self, grid):
        if self.is_healpix(grid):
            nside = self.grids[grid][2] // 4
            return 12 * nside * nside
        return self.grids[grid][1] * self.grids[grid][2]

    def ncoeff(self, grid):
        L = self.grids[grid][3]
        return L * (L + 1) // 2

    # --------------------------------------------------------------- helpers
    def _items(self, x, grid_of_item, per_item):
        """Resolve (tensor, grid_of_item) -> (flat tensor, int32 array)."""
        torch = _torch()
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("expected a CUDA (ROCm) tensor")
        if x.dtype != (self.dtype if per_item != "coeff" else self.dtype):
            raise TypeError(f"expected dtype {self.dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if grid_of_item is None:
            if len(self.grids) != 1:
                raise ValueError("grid_of_item is required for multi-grid plans")
            unit = self.field_size(0) if per_item == "field" else 2 * self.ncoeff(0)
            if x.numel() % unit:
                raise ValueError("tensor size is not a multiple of the item size")
            grid_of_item = [0] * (x.numel() // unit)
        grid_of_item = [int(g) for g in grid_of_item]
        unit = [self.field_size(g) if per_item == "field" else 2 * self.ncoeff(g) for g in grid_of_item]
        if sum(unit) != x.numel():
            raise ValueError(f"tensor has {x.numel()} elements, items need {sum(unit)}")
        return grid_of_item

    # ------------------------------------------------------------ operators
    def heat_apply(self, v, t, grid_of_item=None, transpose=False, out=None):
        torch = _torch()
        goi = self._items(v, grid_of_item, "field")
        n = len(goi)
        tv = np.broadcast_to(np.asarray(t, dtype=np.float64), (n,)).copy()
        if out is None:
            out = torch.empty_like(v)
        _check("shot_heat_apply", self.lib.shot_heat_apply(
            self.handle, _i32_array(goi), n, tv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(bool(transpose)),
            _stream_ptr()))
        return out

    def analysis(self, f, grid_of_item=None):
        """Forward SHT; returns complex coefficients packed by (m, l) per item."""
        torch = _torch()
        goi = self._items(f, grid_of_item, "field")
        total = sum(self.ncoeff(g) for g in goi)
        c = torch.empty(2 * total, dtype=self.dtype, device=f.device)
        _check("shot_sht_analysis", self.lib.shot_sht_analysis(
            self.handle, _i32_array(goi), len(goi), ctypes.c_void_p(f.data_ptr()),
            ctypes.c_void_p(c.data_ptr()), _stream_ptr()))
        return torch.view_as_complex(c.view(-1, 2))

    def synthesis(self, coeffs, grid_of_item=None):
        torch = _torch()
        c = torch.view_as_real(coeffs).contiguous().view(-1) if coeffs.is_complex() else coeffs
        goi = self._items(c, grid_of_item, "coeff")
        total = sum(self.field_size(g) for g in goi)
        f = torch.empty(total, dtype=self.dtype, device=c.device)
        _check("shot_sht_synthesis", self.lib.shot_sht_synthesis(
            self.handle, _i32_array(goi), len(goi), ctypes.c_void_p(c.data_ptr()),
            ctypes.c_void_p(f.data_ptr()), _stream_ptr()))
        return f

    # ---------------------------------------------------------------- solver
    @staticmethod
    def _params(n, eps, tau, T, C, tol):
        eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,))
        tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (n,))
        arr = (Params * n)()
        for i in range(n):
            arr[i] = Params(float(eps[i]), float(tau[i]), int(T), int(C), float(tol))
        return arr

    @staticmethod
    def _info_dicts(info, n):
        return [dict(cost=info[i].cost, err=info[i].err, iters=info[i].iters, status=info[i].status,
                     breakdown_iter=info[i].breakdown_iter, kratio=info[i].kratio) for i in range(n)]

    def sinkhorn(self, p, q, eps, tau=math.inf, T=100, C=10, tol=0.0, grid_of_item=None,
                 potentials=True):
        """Alg. 1 per item.  Returns (phi, psi, [info dict per item])."""
        torch = _torch()
        goi = self._items(p, grid_of_item, "field")
        if q.shape != p.shape or q.dtype != p.dtype or not q.is_contiguous():
            raise ValueError("p and q must have the same shape, dtype and be contiguous")
        n = len(goi)
        prm = self._params(n, eps, tau, T, C, tol)
        info = (SolveInfo * n)()
        phi = torch.empty_like(p) if potentials else None
        psi = torch.empty_like(p) if potentials else None
        code = self.lib.shot_sinkhorn_solve(
            self.handle, _i32_array(goi), n, prm, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr()),
            ctypes.c_void_p(phi.data_ptr() if phi is not None else 0),
            ctypes.c_void_p(psi.data_ptr() if psi is not None else 0), info, _stream_ptr())
        _check("shot_sinkhorn_solve", code, allow=(OK, W_NOT_CONVERGED, E_BREAKDOWN))
        return phi, psi, self._info_dicts(info, n)

    def divergence(self, p, q, eps, tau=math.inf, T=100, C=10, tol=0.0, grid_of_pair=None):
        """Def. 2.3 per pair.  Returns (S numpy array, [info dicts, 3 per pair])."""
        goi = self._items(p, grid_of_pair, "field")
        n = len(goi)
        prm = self._params(n, eps, tau, T, C, tol)
        S = np.zeros(n)
        info = (SolveInfo * (3 * n))()
        code = self.lib.shot_sinkhorn_divergence(
            self.handle, _i32_array(goi), n, prm, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr()),
            S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), info, _stream_ptr())
        _check("shot_sinkhorn_divergence", code, allow=(OK, W_NOT_CONVERGED, E_BREAKDOWN))
        return S, self._info_dicts(info, 3 * n)

    def regional_rms(self, dS_dp, bands=None, grid_of_pair=None):
        """Area-weighted RMS of the centred gradient field dS_dp / a per latitude band.
        bands: dict name -> (lat_lo, lat_hi) in degrees (default: the paper's five regions).
        Returns a dict name -> numpy array over pairs."""
        bands = PAPER_REGIONS if bands is None else bands
        names = list(bands)
        goi = self._items(dS_dp, grid_of_pair, "field")
        n = len(goi)
        b = np.array([bands[k] for k in names], dtype=np.float64).reshape(-1)
        out = np.zeros(n * len(names))
        _check("shot_gradient_regional_rms", self.lib.shot_gradient_regional_rms(
            self.handle, _i32_array(goi), n, ctypes.c_void_p(dS_dp.data_ptr()),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(names),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr()))
        out = out.reshape(n, len(names))
        return {k: out[:, i] for i, k in enumerate(names)}

    def divergence_grad(self, p, q, eps, T=100, C=10, mode="unrolled", checkpoint_every=0,
                        grid_of_pair=None, tau=math.inf):
        """S and dS/dp.  mode: "unrolled" (exact adjoint with recompute; balanced or, with a
        finite tau, unbalanced pairs) or "envelope" (balanced)."""
        torch = _torch()
        goi = self._items(p, grid_of_pair, "field")
        n = len(goi)
        prm = self._params(n, eps, tau, T, C, 0.0)
        S = np.zeros(n)
        g = torch.empty_like(p)
        info = (SolveInfo * (3 * n))()
        code = self.lib.shot_sinkhorn_divergence_grad(
            self.handle, _i32_array(goi), n, prm, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr()),
            S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(g.data_ptr()),
            0 if mode == "unrolled" else 1, int(checkpoint_every), info, _stream_ptr())
        _check("shot_sinkhorn_divergence_grad", code, allow=(OK, W_NOT_CONVERGED, E_BREAKDOWN))
        return S, g, self._info_dicts(info, 3 * n)

    # ---------------------------------------------------------------- tuning
    def set_tuning(self, grid=0, items_per_block=0, chains_per_thread=0):
        _check("shot_plan_set_tuning", self.lib.shot_plan_set_tuning(self.handle, grid, items_per_block,
                                                                     chains_per_thread))

    def get_tuning(self, grid=0):
        ib = ctypes.c_int32()
        jpt = ctypes.c_int32()
        _check("shot_plan_get_tuning", self.lib.shot_plan_get_tuning(self.handle, grid, ctypes.byref(ib),
                                                                     ctypes.byref(jpt)))
        return ib.value, jpt.value

    def set_graphs(self, enable=True):
        _check("shot_plan_set_graphs", self.lib.shot_plan_set_graphs(self.handle, int(bool(enable))))

    def autotune(self, grid=0, nitems=1):
        _check("shot_autotune", self.lib.shot_autotune(self.handle, grid, nitems, _stream_ptr()))
        return self.get_tuning(grid)

    # ------------------------------------------------------------- profiling
    def profile(self, enable=True):
        _check("shot_profile_enable", self.lib.shot_profile_enable(self.handle, int(bool(enable))))

    def profile_read(self, kernel_class):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check("shot_profile_read", self.lib.shot_profile_read(self.handle, int(kernel_class),
                                                                ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
