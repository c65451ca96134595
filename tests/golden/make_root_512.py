"""Writes the oracle's root x* of the 512 x 512 parity case (calls only the
oracle and the seeded generators).

The case has 262,144 cells, above the row count where the library switches
its level-0 products to the SELL-64 layout, so a GPU solve of it exercises
those paths.  Storing the pressure is enough: at the root the flux rows of
the residual vanish, so sigma* = -M(p*)^{-1} (D^T p* + g) follows from p*
face by face (the test recomputes it with the oracle).

Run from the repository root:  python tests/golden/make_root_512.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from problems import small_problem  # noqa: E402
from oracle.coarsen import build_hierarchy  # noqa: E402
from oracle.solvers import result_solve  # noqa: E402

# the recipe; tests/test_gpu_large.py builds the same problem
RECIPE = dict(shape=(512, 512), seed=11, box=(4, 4), m=2, n_levels=3, permute=True, src_scale=200.0,
              g_d_scale=0.3)


def main():
    prob = small_problem(**RECIPE)
    h = build_hierarchy(prob, n_levels=1)
    x = result_solve(h)
    nf = h.levels[0].n_flux
    p = np.ascontiguousarray(x[nf:], dtype=np.float64)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "root_512x512_p.npy")
    np.save(out, p)
    meta = dict(recipe={k: list(v) if isinstance(v, tuple) else v for k, v in RECIPE.items()},
                n_cells=int(p.size), sha256=hashlib.sha256(p.tobytes()).hexdigest(),
                max_abs_p=float(np.abs(p).max()))
    with open(out.replace(".npy", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main()
