"""The full-size workload generators: the batched configuration's 512
instances keep every box aggregate within the 512 cells the local dense
solvers take and total about 1e8 cells; the unstructured workload's source
rate is the one the oracle-only calibration script stored."""
import json
import os

import numpy as np

from oracle.coarsen import box_blocks
from problems.grids import C3_RATE, c4_problem, c4_shape

HERE = os.path.dirname(os.path.abspath(__file__))


def blocks(n, a):
    nb = box_blocks(n, a)
    return [a] * (nb - 1) + [n - a * (nb - 1)]


def test_c4_instances_fit_the_local_solvers():
    total = 0
    seen_a = set()
    for i in range(512):
        shape, a = c4_shape(i)
        assert 4 <= a <= 8
        assert all(16 <= n <= 96 for n in shape)
        biggest = int(np.prod([max(blocks(n, a)) for n in shape]))
        assert biggest <= 512, (i, shape, a, biggest)
        total += int(np.prod(shape))
        seen_a.add(a)
    assert seen_a == {4, 5, 6, 7, 8}
    assert 0.9e8 < total < 1.1e8


def test_c4_problem_matches_its_shape_and_levels():
    for i in (0, 3):
        shape, a = c4_shape(i)
        pr = c4_problem(i)
        assert pr.mesh.n_cells == int(np.prod(shape))
        assert pr.box == (a, a, a) and pr.m == 3
        assert pr.n_levels == 2 if a >= 5 else 2 <= pr.n_levels <= 4
        assert abs(pr.source.mean()) < 1e-12


def test_c3_rate_is_the_calibrated_one():
    with open(os.path.join(HERE, "golden", "c3_rate.json")) as fh:
        assert json.load(fh)["rate"] == C3_RATE
