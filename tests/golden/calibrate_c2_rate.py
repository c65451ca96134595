"""Calibrates the well rate of the 60x220x85 workload (run by hand; the
result is the constant C2_WELL_RATE in problems/grids.py and is stored in
c2_rate.json next to this file).

With kappa = exp(p) a strong sink can leave the discrete problem without a
solution, so the rate is chosen such that the linear (kappa = 1) pressure has
max |p| = 0.5.  The linear pressure scales with the rate, so one solve at
rate 1 fixes it.  The system is the oracle's level-0 system reduced to the
cell unknowns (diagonal flux block eliminated); it is solved by conjugate
gradients preconditioned with exact solves along the vertical cell columns
(the mesh couples cells 100 times more strongly in z than in x), to a
relative residual of 1e-9.  A sparse direct solve of this 3-D system does not
finish in reasonable time on one host.
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from problems import c2_problem          # noqa: E402
from oracle.fv import FineSystem          # noqa: E402


def reduced_matrix(fs):
    n = fs.n_cells
    w = 1.0 / (1.0 / fs.TK + np.where(fs.inner, 1.0 / np.where(fs.inner, fs.TL, 1.0), 0.0))
    K, L, inner = fs.K, fs.L, fs.inner
    rows = np.concatenate([K, L[inner], K[inner], L[inner]])
    cols = np.concatenate([K, L[inner], L[inner], K[inner]])
    vals = np.concatenate([w, w[inner], -w[inner], -w[inner]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def column_pcg(S, b, shape, tol=1e-9, maxit=20000):
    nx, ny, nz = shape
    n = nx * ny * nz
    plane = nx * ny
    d = S.diagonal().reshape(nz, plane)
    off = np.asarray(S[np.arange(n - plane), np.arange(plane, n)]).ravel().reshape(nz - 1, plane)

    def column_solve(r):      # Thomas algorithm on every vertical column at once
        r = r.reshape(nz, plane)
        cp = np.zeros_like(off)
        dp = np.zeros_like(r)
        cp[0] = off[0] / d[0]
        dp[0] = r[0] / d[0]
        for k in range(1, nz):
            den = d[k] - off[k - 1] * cp[k - 1]
            if k < nz - 1:
                cp[k] = off[k] / den
            dp[k] = (r[k] - off[k - 1] * dp[k - 1]) / den
        x = np.zeros_like(r)
        x[-1] = dp[-1]
        for k in range(nz - 2, -1, -1):
            x[k] = dp[k] - cp[k] * x[k + 1]
        return x.ravel()

    x = np.zeros(n)
    r = b.copy()
    z = column_solve(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for it in range(maxit):
        q = S @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) < tol * bn:
            return x, it + 1
        z = column_solve(r)
        rz2 = r @ z
        p = z + (rz2 / rz) * p
        rz = rz2
    raise RuntimeError("column-preconditioned CG did not converge")


if __name__ == "__main__":
    t = time.time()
    prob = c2_problem(rate=1.0, permute=False)     # cell id = i + nx (j + ny k)
    fs = FineSystem(prob)
    p, its = column_pcg(reduced_matrix(fs), fs.f, (60, 220, 85))
    mx = float(np.abs(p).max())
    out = {"max_abs_p_at_rate_1": mx, "rate": 0.5 / mx, "cg_iterations": its, "seconds": time.time() - t}
    print(out)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_rate.json"), "w") as fh:
        json.dump(out, fh, indent=1)
