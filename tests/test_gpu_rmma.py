"""Recurrence-fed matrix-core Legendre kernel (Sec. 3.2, App. C.1) against the oracle.

The float64 recurrence feeds matrix-core contractions of 8 or 16 items per
workgroup in three operand forms.  Bounds, set from the operand precision
before any run (relative L2 of the heat apply):
* float32 operands (float32 plans tuned to the kernel): 1e-5, the float32 bound;
* split bfloat16 (hi + lo, three products; SHOT_BF16X3_MFMA): 1e-4 -- each
  product carries about 2^-16 relative error, the float32 accumulation adds
  little;
* bfloat16 (SHOT_BF16_MFMA with recurrence): 1e-2, as for the bfloat16 table.
Cases cover partial column tiles, latitude counts that are not a multiple of
64 (idle lanes), odd nlat (equator row), orders whose row count is not a
multiple of 32, and batches mixing two grids.
"""

import numpy as np
import pytest

import oracle as O
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

BOUND = {"fp32": 1e-5, "bf16x3": 1e-4, "bf16": 1e-2}


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _plan(grids, precision):
    from paper_2605_18389_amd import Plan
    return Plan(grids, precision=precision, legendre="recurrence")


GRIDS = [("gl", 32, 64, 32), ("cc", 33, 64, 32), ("gl", 45, 90, 45), ("gl", 90, 180, 90),
         ("cc", 129, 256, 128), ("gl", 180, 360, 180)]


@pytest.mark.parametrize("prec,ipb", [("fp32", 8), ("fp32", 16), ("bf16x3", 0), ("bf16x3", 8), ("bf16", 0)])
@pytest.mark.parametrize("grid", GRIDS)
def test_rmma_heat_apply_matches_oracle(grid, prec, ipb):
    announce(f"rmma heat apply {grid} {prec} ipb={ipb}")
    P = _plan([grid], prec)
    if ipb:
        P.set_tuning(0, ipb, 0)
    g = O.make_grid(*grid)
    rng = np.random.default_rng(5)
    for nitems in (1, 3, 9, 17):
        v = np.stack([synth.temperature_like(rng, g.x, g.w, g.nlon, K=8) for _ in range(nitems)])
        t = np.geomspace(1e-4, 4e-2, nitems)
        out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
        errs = [rel_l2(out[i], O.heat_apply(v[i], g, t[i])) for i in range(nitems)]
        print(f"  items={nitems}: max rel L2 {max(errs):.2e} (bound {BOUND[prec]:.0e})", flush=True)
        assert max(errs) < BOUND[prec], errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_rmma_mixed_grid_batch(prec):
    """Two grids in one call (one Legendre launch per grid group)."""
    grids = [("gl", 90, 180, 90), ("gl", 180, 360, 180)]
    announce(f"rmma mixed batch {prec}")
    P = _plan(grids, prec)
    if prec == "fp32":
        P.set_tuning(0, 16, 0)
        P.set_tuning(1, 8, 0)
    gs = [O.make_grid(*gr) for gr in grids]
    goi = [1, 0, 1, 1, 0, 0, 0, 1, 0, 1, 0]
    rng = np.random.default_rng(9)
    fields = [synth.temperature_like(rng, gs[k].x, gs[k].w, gs[k].nlon, K=8) for k in goi]
    t = np.geomspace(1e-3, 1e-2, len(goi))
    v = to_dev(np.concatenate([f.ravel() for f in fields]), P.dtype)
    out = to_np(P.heat_apply(v, t, grid_of_item=goi))
    off = 0
    for k, f, tk in zip(goi, fields, t):
        n = gs[k].n
        err = rel_l2(out[off:off + n].reshape(f.shape), O.heat_apply(f, gs[k], tk))
        assert err < BOUND[prec], (k, err)
        off += n


def test_rmma_tuning_and_autotune():
    """Float32 recurrence grids accept 8 or 16 items per workgroup (matrix cores);
    the autotuner of a bfloat16 plan chooses among matrix-core shapes only."""
    announce("rmma tuning")
    from paper_2605_18389_amd.binding import ShotError
    P = _plan([("gl", 90, 180, 90)], "fp32")
    P.set_tuning(0, 16, 0)
    assert P.get_tuning(0) == (16, 0)
    Pb = _plan([("gl", 90, 180, 90)], "bf16x3")
    ib, _ = Pb.autotune(0, 24)
    assert ib in (8, 16)
    Pt = _plan([("gl", 90, 180, 90)], "fp64")
    with pytest.raises(ShotError):
        from paper_2605_18389_amd import Plan
        Plan([("gl", 90, 180, 90)], precision="bf16x3", legendre="table")


@pytest.mark.parametrize("prec,ipb", [("fp32", 8), ("bf16x3", 0), ("bf16", 0)])
def test_rmma_rough_input_and_item_independence(prec, ipb):
    """White noise (energy at every degree the grid holds, unlike the smooth
    temperature-like fields): the heat apply against the oracle at the same
    bounds, and each item of a batch equal bit for bit to the same item alone
    (items never share arithmetic)."""
    grid = ("gl", 180, 360, 180)
    announce(f"rmma rough input {prec} ipb={ipb}")
    P = _plan([grid], prec)
    if ipb:
        P.set_tuning(0, ipb, 0)
    g = O.make_grid(*grid)
    rng = np.random.default_rng(17)
    v = rng.random((5, g.nlat, g.nlon))
    t = [1e-3, 1e-4, 4e-2, 1e-3, 2e-3]
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
    for i in (0, 2):
        err = rel_l2(out[i], O.heat_apply(v[i], g, t[i]))
        print(f"  item {i} t={t[i]}: rel L2 {err:.2e} (bound {BOUND[prec]:.0e})", flush=True)
        assert err < BOUND[prec]
    for i in range(5):
        alone = to_np(P.heat_apply(to_dev(v[i:i + 1], P.dtype), [t[i]])).reshape(v.shape[1:])
        assert np.array_equal(alone, out[i]), i
