"""Edge cases of the heat apply (Sec. 3.2) on the GPU, against the FP64 oracle.

* An empty batch is rejected before any launch (SHOT_E_INVALID), through the C ABI
  and through the binding.
* Heat time t = 0: h_l = 1 for every kept degree, so HeatConv is analysis then
  synthesis (App. C.1).  Where the quadrature integrates products of degree up to
  2L - 2 exactly (Gauss-Legendre rows with nlat >= L) that is the projection onto
  degrees l < L, and a band-limited field comes back unchanged; every grid is also
  compared with the oracle's t = 0 apply.
* A long heat time leaves only the l = 0 term: the constant field equal to the
  area-weighted mean (the Y_00 coefficient times Y_00).
* The smallest grids a plan accepts (two rows and two columns; a plan refuses one
  row or one column): two rows and no equator row; three rows with one.

Tolerances: float64 plans 1e-12 relative L2, float32 plans 1e-5 (the heat-apply bound).
"""

import ctypes
import math

import numpy as np
import pytest

import oracle as O
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, rel_l2, to_dev, to_np
from parity import check_status, tolerance

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
FORMS = [("fp64", "recurrence"), ("fp32", "recurrence"), ("fp32", "table")]


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _plan(grid, precision, legendre):
    from paper_2605_18389_amd import Plan
    return Plan([grid], precision=precision, legendre=legendre)


def test_empty_batch_is_rejected():
    import torch
    from paper_2605_18389_amd import binding
    announce("empty batch")
    P = _plan(("gl", 17, 36, 18), "fp32", "recurrence")
    lib = P.lib
    v = torch.zeros(17 * 36, dtype=torch.float32, device="cuda")
    out = torch.zeros_like(v)
    goi = (ctypes.c_int32 * 1)(0)
    t = (ctypes.c_double * 1)(1e-3)
    st = lib.shot_heat_apply(P.handle, goi, 0, t, ctypes.c_void_p(v.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), 0, None)
    assert st == binding.E_INVALID
    st = lib.shot_sht_analysis(P.handle, goi, 0, ctypes.c_void_p(v.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), None)
    assert st == binding.E_INVALID
    with pytest.raises(binding.ShotError):
        P.heat_apply(torch.zeros(0, dtype=torch.float32, device="cuda"), [])
    with pytest.raises(binding.ShotError):
        P.divergence(torch.zeros(0, dtype=torch.float32, device="cuda"),
                     torch.zeros(0, dtype=torch.float32, device="cuda"), 0.1, T=2)
    # the plan still works afterwards
    g = O.make_grid("gl", 17, 36, 18)
    f = synth.temperature_like(np.random.default_rng(20), g.x, g.w, g.nlon, K=4)
    got = to_np(P.heat_apply(to_dev(f[None], P.dtype), [1e-3])).reshape(f.shape)
    assert rel_l2(got, O.heat_apply(f, g, 1e-3)) < TOL["fp32"]


@pytest.mark.parametrize("prec,legendre", FORMS)
@pytest.mark.parametrize("grid", [("gl", 32, 64, 32), ("cc", 33, 64, 32), ("gl", 17, 36, 18)])
def test_heat_time_zero_is_the_band_projection(grid, prec, legendre):
    announce(f"t = 0 {grid} {prec} {legendre}")
    P = _plan(grid, prec, legendre)
    g = O.make_grid(*grid)
    v = np.random.default_rng(21).random((g.nlat, g.nlon)) + 0.5
    f = O.synthesis(O.analysis(v, g), g)          # band-limited to l < L
    out = to_np(P.heat_apply(to_dev(np.stack([v, f]), P.dtype), [0.0, 0.0])).reshape(2, *v.shape)
    e_proj = rel_l2(out[0], O.heat_apply(v, g, 0.0))
    e_fix = rel_l2(out[1], f)
    print(f"[t=0] {grid} {prec} {legendre} projection {e_proj:.2e}, band-limited fixed point {e_fix:.2e}",
          flush=True)
    assert e_proj < TOL[prec]
    if grid[0] == "gl" and grid[1] >= grid[3]:   # exact quadrature: a projection
        assert e_fix < TOL[prec]


@pytest.mark.parametrize("prec,legendre", FORMS)
@pytest.mark.parametrize("grid", [("gl", 32, 64, 32), ("cc", 33, 64, 32)])
def test_long_heat_time_leaves_the_area_weighted_mean(grid, prec, legendre):
    announce(f"t = 50 {grid} {prec} {legendre}")
    P = _plan(grid, prec, legendre)
    g = O.make_grid(*grid)
    v = np.random.default_rng(22).random((g.nlat, g.nlon)) + 0.5
    a = np.repeat(np.asarray(g.w)[:, None], g.nlon, axis=1) * 2 * np.pi / g.nlon
    mean = (a * v).sum() / (4 * np.pi)
    out = to_np(P.heat_apply(to_dev(v[None], P.dtype), [50.0])).reshape(v.shape)
    err = np.abs(out - mean).max() / mean
    print(f"[t=50] {grid} {prec} {legendre} max |K v - mean| / mean {err:.2e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec,legendre", FORMS)
@pytest.mark.parametrize("grid", [("gl", 2, 2, 1), ("gl", 2, 3, 2), ("cc", 3, 4, 2), ("gl", 3, 5, 3)])
def test_smallest_grids(grid, prec, legendre):
    announce(f"smallest grid {grid} {prec} {legendre}")
    P = _plan(grid, prec, legendre)
    g = O.make_grid(*grid)
    v = np.random.default_rng(23).random((3, g.nlat, g.nlon)) + 0.5
    t = [1e-2, 0.3, 0.0]
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
    errs = [rel_l2(out[i], O.heat_apply(v[i], g, t[i])) for i in range(3)]
    print(f"[smallest] {grid} {prec} {legendre} rel L2 {max(errs):.2e}", flush=True)
    assert max(errs) < TOL[prec]


def test_invalid_parameters_are_rejected():
    """Non-positive eps or tau, fewer than one iteration or check interval, a negative
    tolerance, and negative or non-finite heat times return SHOT_E_INVALID; the plan is
    still usable afterwards."""
    import math
    import torch
    from paper_2605_18389_amd import binding
    announce("invalid parameters")
    grid = ("gl", 17, 36, 18)
    P = _plan(grid, "fp64", "recurrence")
    g = O.make_grid(*grid)
    p, q = synth.vmf_pair(synth.pair_seed(0, 5), g.x, g.w, g.nlon, K=3)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    for kw in (dict(eps=0.0), dict(eps=-0.1), dict(eps=math.inf), dict(eps=0.1, tau=0.0),
               dict(eps=0.1, T=0), dict(eps=0.1, C=0), dict(eps=0.1, tol=-1.0)):
        with pytest.raises(binding.ShotError) as e:
            P.sinkhorn(pd, qd, **kw)
        assert e.value.code == binding.E_INVALID, kw
    for t in (-1e-3, math.nan, math.inf):
        with pytest.raises(binding.ShotError) as e:
            P.heat_apply(pd, [t])
        assert e.value.code == binding.E_INVALID, t
    got = to_np(P.heat_apply(pd, [1e-2])).reshape(p.shape)
    assert rel_l2(got, O.heat_apply(p, g, 1e-2)) < TOL["fp64"]


@pytest.mark.parametrize("T", [1, 2])
@pytest.mark.parametrize("tau", [math.inf, 1.0])
def test_fewest_iterations_match_the_oracle(T, tau):
    """Alg. 1 stopped after one or two iterations (checked every iteration), balanced and
    unbalanced, float64 on a 32x64 vMF pair: status, cost, potentials and e_marg against
    the oracle's, graded by the rule of tests/parity.py."""
    announce(f"T={T} tau={tau}")
    grid = ("gl", 32, 64, 32)
    P = _plan(grid, "fp64", "recurrence")
    g = O.make_grid(*grid)
    p, q = synth.vmf_pair(synth.pair_seed(0, 6), g.x, g.w, g.nlon, K=4)
    eps = 0.16
    phi, psi, inf = P.sinkhorn(to_dev(p, P.dtype), to_dev(q, P.dtype), eps, tau=tau, T=T, C=1)
    r = O.sinkhorn(p, q, g, eps, tau, T, C=1)
    e_cost = abs(inf[0]["cost"] - r["cost"]) / abs(r["cost"])
    e_phi = rel_l2(to_np(phi).reshape(p.shape), r["phi"])
    e_psi = rel_l2(to_np(psi).reshape(p.shape), r["psi"])
    print(f"[fewest] T={T} tau={tau} iters {inf[0]['iters']} cost {e_cost:.2e} phi {e_phi:.2e} "
          f"psi {e_psi:.2e} err {inf[0]['err']:.3e} / {r['err']:.3e}", flush=True)
    assert inf[0]["iters"] == T and inf[0]["status"] == 0 and r["breakdown"] == 0
    assert check_status(inf[0], r, "fp64")
    tol = tolerance(r, "fp64")
    print(f"[fewest] bound {tol:.1e} (cost), {10 * tol:.1e} (potentials)", flush=True)
    assert e_cost <= tol
    assert e_phi < 10 * tol and e_psi < 10 * tol
    assert abs(inf[0]["err"] - r["err"]) <= 1e-3 * r["err"] + 10 * tol


@pytest.mark.parametrize("bad", ["zero", "negative", "nan"])
def test_marginal_without_positive_mass_is_rejected(bad):
    """A marginal whose area-weighted mass is not positive and finite makes the solve,
    divergence and gradient calls return SHOT_E_INVALID, with the item named in
    shot_last_error(); a valid batch on the same plan still solves afterwards."""
    from paper_2605_18389_amd import binding
    announce(f"marginal mass {bad}")
    grid = ("gl", 17, 36, 18)
    P = _plan(grid, "fp32", "recurrence")
    g = O.make_grid(*grid)
    p, q = synth.vmf_pair(synth.pair_seed(0, 7), g.x, g.w, g.nlon, K=3)
    pb = {"zero": np.zeros_like(p), "negative": -p, "nan": np.where(np.arange(p.size).reshape(p.shape) == 5, np.nan, p)}[bad]
    pd, qd, pbd = to_dev(p, P.dtype), to_dev(q, P.dtype), to_dev(np.stack([p, pb]), P.dtype)
    qq = to_dev(np.stack([q, q]), P.dtype)
    with pytest.raises(binding.ShotError) as e:
        P.sinkhorn(pbd, qq, 0.1, T=5)
    assert e.value.code == binding.E_INVALID
    assert b"item 1" in P.lib.shot_last_error()
    with pytest.raises(binding.ShotError) as e:
        P.divergence(pbd, qq, 0.1, T=5)
    assert e.value.code == binding.E_INVALID
    with pytest.raises(binding.ShotError) as e:
        P.divergence_grad(pbd, qq, 0.1, T=5)
    assert e.value.code == binding.E_INVALID
    # eps = 1 stays clear of breakdown here (oracle kernel ratio 4e-3)
    _, _, inf = P.sinkhorn(pd, qd, 1.0, T=5)
    assert inf[0]["status"] == 0
