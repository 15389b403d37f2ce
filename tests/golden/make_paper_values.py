"""Writes paper_values.json: closed-form constants from the paper's experiments.

Sources (paper sections):
* section 3.1 (after the ROF updates) and section 4.1 print a two-valued
  minimiser for the disc indicator I = 1_{|x - c| <= r} on [0,1]^2 with Neumann
  boundary.  As printed, (1 - 2/(lambda r)) I + 2 pi r / (lambda (1 - pi r^2)),
  it does not preserve the mean of I, which every Neumann ROF minimiser must
  (lambda (u - I) = div p integrates to zero).  The corrected form takes the
  value a = 1 - 2/(lambda r) on the disc and b = 2 pi r / (lambda (1 - pi r^2))
  off it; a pi r^2 + b (1 - pi r^2) = pi r^2.  It holds when a > b, i.e.
  lambda > 2/r + 2 pi r / (1 - pi r^2).
* section 4.2: when rho1 is rho0 translated by v the EMD equals |v|; the
  paper's pairs are translated by (1/4, 1/4), so EMD = 1/sqrt(8).
This script uses only these formulas (no solver code).
"""
import json
import math
import os

r, lam = 0.25, 20.0
a = 1.0 - 2.0 / (lam * r)
b = 2.0 * math.pi * r / (lam * (1.0 - math.pi * r * r))
out = {
    "rof_disc": {
        "cite": "section 3.1 (disc example) and section 4.1 (experiment set-up); corrected for mean preservation",
        "radius": r,
        "lambda": lam,
        "inside_corrected": a,
        "outside_corrected": b,
        "inside_as_printed": a + b,
        "lambda_threshold_corrected": 2.0 / r + 2.0 * math.pi * r / (1.0 - math.pi * r * r),
        "lambda_threshold_as_printed": 2.0 / r,
    },
    "emd_translation": {
        "cite": "section 4.2: translated measures, EMD = |v| with v = (1/4, 1/4)",
        "shift": [0.25, 0.25],
        "emd": 1.0 / math.sqrt(8.0),
    },
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_values.json"), "w") as fh:
    json.dump(out, fh, indent=2)
