"""Calibrates the source rate of the unstructured workload (2,000,000 seeded
Voronoi cells; run by hand, the result is the constant C3_RATE in
problems/grids.py and is stored in c3_rate.json next to this file).

With kappa = exp(2p) a strong sink can leave the discrete problem without a
solution, so the rate is chosen such that the linear (kappa = 1) pressure
has alpha max |p| = 0.5.  The linear pressure scales with the rate, so one
solve at rate 1 fixes it: the oracle's reduced cell system (flux block
eliminated), by a sparse direct solve.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from problems.grids import c3_problem     # noqa: E402
from oracle.fv import linear_pressure      # noqa: E402

if __name__ == "__main__":
    t = time.time()
    prob = c3_problem(rate=1.0)
    p = linear_pressure(prob)
    mx = float(np.abs(p).max())
    out = {"max_abs_p_at_rate_1": mx, "alpha": prob.alpha, "rate": 0.5 / (prob.alpha * mx),
           "seconds": time.time() - t}
    print(out)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_rate.json"), "w") as fh:
        json.dump(out, fh, indent=1)
