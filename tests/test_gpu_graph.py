"""Graph-captured fixed-T solves replay to the same bits as eager launches."""

import math

import numpy as np
import pytest

import oracle as O
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def test_graph_replay_matches_eager():
    from paper_2605_18389_amd import Plan
    grids = [("gl", 24, 48, 24), ("cc", 33, 64, 32)]
    announce("graph replay")
    P = Plan(grids, precision="fp32", legendre="recurrence")
    gs = [O.make_grid(*g) for g in grids]
    goi = [0, 1, 1]
    ps, qs = [], []
    for i, k in enumerate(goi):
        p, q = synth.temperature_pair(50 + i, gs[k].x, gs[k].w, gs[k].nlon, K=4,
                                      q_mass=1.0 if i != 1 else 1.05)
        ps.append(p.ravel())
        qs.append(q.ravel())
    pf = to_dev(np.concatenate(ps), P.dtype)
    qf = to_dev(np.concatenate(qs), P.dtype)
    taus = [math.inf, 1.0, math.inf]
    P.set_graphs(False)
    e_phi, e_psi, e_inf = P.sinkhorn(pf, qf, 0.2, taus, T=40, grid_of_item=goi)
    P.set_graphs(True)
    for rep in range(3):   # first call records, later calls replay
        phi, psi, inf = P.sinkhorn(pf, qf, 0.2, taus, T=40, grid_of_item=goi)
        assert np.array_equal(to_np(phi), to_np(e_phi), equal_nan=True), rep
        assert np.array_equal(to_np(psi), to_np(e_psi), equal_nan=True), rep
        assert [x["cost"] for x in inf] == [x["cost"] for x in e_inf]
        assert [x["kratio"] for x in inf] == [x["kratio"] for x in e_inf]
    # new inputs through the same replayed graph
    pf2 = pf.flip(0).contiguous()
    P.set_graphs(False)
    e2 = P.sinkhorn(pf2, qf, 0.2, taus, T=40, grid_of_item=goi)
    P.set_graphs(True)
    g2 = P.sinkhorn(pf2, qf, 0.2, taus, T=40, grid_of_item=goi)
    assert np.array_equal(to_np(g2[0]), to_np(e2[0]), equal_nan=True)
    # a different layout records a new graph
    g3 = P.sinkhorn(pf[:gs[0].n].contiguous(), qf[:gs[0].n].contiguous(), 0.2, T=40, grid_of_item=[0])
    P.set_graphs(False)
    e3 = P.sinkhorn(pf[:gs[0].n].contiguous(), qf[:gs[0].n].contiguous(), 0.2, T=40, grid_of_item=[0])
    assert np.array_equal(to_np(g3[0]), to_np(e3[0]), equal_nan=True)


def test_profiling_inside_graphs():
    from paper_2605_18389_amd import Plan
    grid = ("gl", 32, 64, 32)
    announce("graph profiling")
    P = Plan([grid], precision="fp32", legendre="recurrence")
    g = O.make_grid(*grid)
    p, q = synth.temperature_pair(3, g.x, g.w, g.nlon)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    ref = P.sinkhorn(pd, qd, 0.1, T=20)
    P.profile(True)
    for _ in range(2):
        out = P.sinkhorn(pd, qd, 0.1, T=20)
        assert np.array_equal(to_np(out[0]), to_np(ref[0]), equal_nan=True)
    n, ms = P.profile_read(0)
    P.profile(False)
    assert n >= 40 and ms > 0
