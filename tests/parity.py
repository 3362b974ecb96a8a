"""Grading rules for GPU-vs-oracle Sinkhorn parity (test infrastructure).

The scaling form of Alg. 1 breaks down when a truncated heat-kernel output
goes non-positive (App. C.4).  The spectral heat apply is accurate to about
u * max|K v| in absolute terms (u = unit roundoff of the arithmetic), so an
output whose true value is below that cannot be told from zero.  Hence:

* margin: an item is value-graded only if the oracle never breaks down and its
  kernel ratio min(K.)/max(K.) stays above MARGIN[prec] for the whole run;
* status: the GPU may report a breakdown only at an iteration where the
  oracle's ratio is below the margin (or the oracle has broken down already);
  an item graded by value must not break down on the GPU;
* tolerance: graded values agree to max(base, 10 u / kratio) relative, the
  error of the smallest heat-kernel output carried into u = p / K v.
"""

import json
import os

U = {"fp64": 1.1e-16, "fp32": 6.0e-8}
MARGIN = {"fp64": 1e-13, "fp32": 1e-5}
BASE = {"fp64": 1e-10, "fp32": 1e-4}


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
        assert ratio < margin or (kb and kg >= kb), (
            f"GPU broke down at iteration {kg} where the oracle ratio is {ratio:.3e}")
    graded = kb == 0 and float(oref["kratio"]) > margin
    if graded:
        assert kg == 0, "item above the margin broke down on the GPU"
        # the GPU's own running kernel ratio agrees with the oracle's to the
        # accuracy of the smallest heat-kernel output
        kr = float(oref["kratio"])
        assert abs(gpu["kratio"] - kr) <= 10.0 * U[prec] / kr * kr + 1e-6 * kr, (gpu["kratio"], kr)
    return graded


def tolerance(oref, prec):
    kr = float(oref["kratio"])
    return max(BASE[prec], 10.0 * U[prec] / kr)


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
