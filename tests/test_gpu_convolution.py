"""Heat versus matrix convolution (appendix on convolution on S^2) with the
heat side on the GPU.

A vMF measure (kappa = 10, seeded mean direction) is smoothed by the library's
batched heat apply at t = eps / 4 for eight eps log-spaced in [1e-3, 10] (one
item per eps, one launch sequence), on Clenshaw-Curtis grids of band limit
L (L + 1 rows with both poles, 2L columns) and HEALPix grids with L = 2 Nside.
The matrix convolution is the oracle's dense sum.  Checked: the GPU heat
outputs against the oracle's heat convolution element by element, and the
rescaled mean absolute error table against the oracle's own table.  The paper
prints no values for this study, so the table itself is parity unpinned beyond
the oracle's pins (C(eps) closed form, delta and constant images, limits).
"""

import numpy as np
import pytest

import oracle as O
from oracle import convolution as C
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, rel_l2, to_dev, to_np
from parity import report

pytestmark = pytest.mark.gpu

EPS8 = np.logspace(-3, 1, 8)


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _grid(kind, n):
    if kind == "cc":
        return ("cc", n + 1, 2 * n, n), O.make_grid("cc", n + 1, 2 * n, n)
    return ("hp", n, 2 * n), O.HealpixGrid(n, 2 * n)


@pytest.mark.parametrize("prec,tol_heat", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("kind,n", [("cc", 8), ("cc", 16), ("cc", 32), ("hp", 4), ("hp", 8), ("hp", 16)])
def test_heat_vs_matrix_table(kind, n, prec, tol_heat):
    from paper_2605_18389_amd import Plan
    announce(f"heat vs matrix {kind} {n} {prec}")
    spec, g = _grid(kind, n)
    X = g.points()
    f, _ = synth.vmf_at(4, X[..., 2], np.arctan2(X[..., 1], X[..., 0]), 10.0)
    P = Plan([spec], precision=prec)
    v = np.broadcast_to(f, (len(EPS8),) + f.shape)
    heat = to_np(P.heat_apply(to_dev(v, P.dtype), EPS8 / 4.0)).reshape(v.shape)
    mae_gpu, mae_ref = [], []
    for i, eps in enumerate(EPS8):
        ref = C.heat_convolution(f, g, eps)
        assert rel_l2(heat[i], ref) < tol_heat, (eps, rel_l2(heat[i], ref))
        km = C.matrix_convolution(f, g, eps)
        mae_gpu.append(C.rescaled_mae(heat[i], km, eps))
        mae_ref.append(C.rescaled_mae(ref, km, eps))
    mae_gpu, mae_ref = np.array(mae_gpu), np.array(mae_ref)
    for eps, a, b in zip(EPS8, mae_gpu, mae_ref):
        report(f"heat-vs-matrix {kind}{n} {prec} eps={eps:.3g}", mae=a, mae_ref=b)
    # |MAE_gpu - MAE_ref| <= C(eps) mean|heat_gpu - heat_ref| <= C(eps) rms(heat_ref) tol_heat
    bound = np.array([C.geodesic_kernel_integral(e) * np.sqrt(np.mean(C.heat_convolution(f, g, e) ** 2))
                      for e in EPS8]) * tol_heat
    assert np.all(np.abs(mae_gpu - mae_ref) <= bound), (mae_gpu, mae_ref, bound)
