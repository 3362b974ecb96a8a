"""Grading rules for GPU-vs-oracle Sinkhorn parity (test infrastructure).

The scaling form of Alg. 1 breaks down when a truncated heat-kernel output
goes non-positive (App. C.4).  The spectral heat apply is accurate to about
u * max|K v| in absolute terms (u = unit roundoff of the arithmetic), so an
output whose true value is below that cannot be told from zero.  Hence:

* margin: an item is value-graded only if the oracle never breaks down and its
  kernel ratio min(K.)/max(K.) stays above MARGIN[prec] for the whole run;
* status: the GPU may report a breakdown only at an iteration where the
  oracle's ratio is below the margin, or, for an item the oracle also breaks
  down on, where that ratio is already within 100 times the margin: a ratio
  collapsing towards zero crosses it a few iterations earlier or later as the
  iterates drift by rounding (seen in float32 on 90x180 at t = 4.5e-4: oracle
  breakdown at iteration 93, GPU at 84 where the oracle's ratio was 5.3e-4);
  an item graded by value must not break down on the GPU;
* tolerance: graded values agree to max(base, 10 u / kratio) relative, the
  error of the smallest heat-kernel output carried into u = p / K v; the
  GPU's running kernel ratio itself, usually smallest at the first
  iterations, to max(that, 10 E_APPLY / kratio), E_APPLY being one heat
  apply's error relative to max|K v|.

Matrix-core forms, bounds fixed from the operand precision before any run:
* split bfloat16 (hi + lo, three products): about 2^-16 relative per product,
  so u = 1.5e-5; margin 2e-3; costs at 1e-3;
* bfloat16: u = 2^-8 = 3.9e-3; margin 0.5, so nearly every solve is judged on
  its status only; costs at 5e-2.
The divergence S (Def. 2.3) is a difference of three costs and can be orders of
magnitude smaller than each; s_bound states how it is graded.
"""

import json
import os

U = {"fp64": 1.1e-16, "fp32": 6.0e-8, "bf16x3": 1.5e-5, "bf16": 3.9e-3}
# error of one heat apply relative to max|K v|: float32 plans may contract on
# matrix cores, accumulating in float32 over up to L terms (about sqrt(L) u,
# 1.6e-6 at L = 720); the other forms as u
E_APPLY = {"fp64": 1e-15, "fp32": 2e-6, "bf16x3": 1.5e-4, "bf16": 3.9e-2}
MARGIN = {"fp64": 1e-13, "fp32": 1e-5, "bf16x3": 2e-3, "bf16": 0.5}
BASE = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-3, "bf16": 5e-2}


def check_status(gpu, oref, prec):
    """Assert status consistency; return True when the item is value-graded."""
    margin = MARGIN[prec]
    kb = int(oref["breakdown"])
    kg = int(gpu["breakdown_iter"])
    hist = oref["kratio_hist"]
    if kg:
        assert gpu["status"] == 17
        assert kg <= len(hist), (kg, len(hist))
        ratio = float(hist[kg - 1])
        assert ratio < margin or (kb and (kg >= kb or ratio < 100.0 * margin)), (
            f"GPU broke down at iteration {kg} where the oracle ratio is {ratio:.3e}")
    graded = kb == 0 and float(oref["kratio"]) > margin
    if graded:
        assert kg == 0, "item above the margin broke down on the GPU"
        # the GPU's own running kernel ratio: its minimum is usually reached at
        # the first iterations, where min(K.) carries the heat apply's own
        # error, E_APPLY of max|K.|, undamped by the iteration
        kr = float(oref["kratio"])
        kr_tol = max(tolerance(oref, prec), 10.0 * E_APPLY[prec] / kr)
        assert abs(gpu["kratio"] - kr) <= kr_tol * kr, (gpu["kratio"], kr, kr_tol)
    return graded


def tolerance(oref, prec):
    kr = float(oref["kratio"])
    return max(BASE[prec], 10.0 * U[prec] / kr)


def well_conditioned(solves, prec):
    """Every solve clear of the breakdown by 10x the margin."""
    return all(int(s["breakdown"]) == 0 and float(s["kratio"]) > 10.0 * MARGIN[prec] for s in solves)


def s_bound(solves, S_ref, prec):
    """Relative bound on S for a pair whose three solves are value-graded.

    float64 and float32: the stated bound (1e-10, 1e-4) when the pair is well
    conditioned, else (borderline) the summed tolerances of the three costs.
    Matrix-core forms: the rounding of the costs S is the difference of,
    10 u (|R_pq| + (|R_pp| + |R_qq|)/2), relative to |S|, at least BASE."""
    R = [abs(float(s["cost"])) for s in solves]
    if prec in ("fp64", "fp32"):
        if well_conditioned(solves, prec):
            return BASE[prec]
        return sum(w * tolerance(s, prec) * r for w, s, r in zip((1.0, 0.5, 0.5), solves, R)) / abs(S_ref)
    return max(BASE[prec], 10.0 * U[prec] * (R[0] + 0.5 * (R[1] + R[2])) / abs(S_ref))


def report(case, **kw):
    path = os.environ.get("SHOT_PARITY_LOG")
    if not path:
        return
    rec = {"case": case}
    for k, v in kw.items():
        try:
            rec[k] = float(v)
        except (TypeError, ValueError):
            rec[k] = str(v)
    with open(path, "a") as fh:
        fh.write(json.dumps(rec) + "\n")
