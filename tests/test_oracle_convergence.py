"""Pins of the oracle's convergence measure between iterations (the
Frobenius distance of unit-norm binary occupancy matrices of a 2-D
projection, 20 x 20 cells of 0.8 A in the paper).

Expected values: 0 for identical occupancy, sqrt(2) for disjoint occupancy,
sqrt(2 - sqrt(2)) for {c1, c2} against {c2}, and on random sets the closed
form 2 - 2 |A & B| / sqrt(|A| |B|) evaluated on Python sets of cell tuples.
"""
import math

import numpy as np
import pytest

import oracle as O

GRID = dict(x0=0.0, y0=0.0, cell=0.8, nx=20, ny=20)


def test_identical_disjoint_and_half_overlap():
    a = [[0.1, 0.1], [0.9, 0.1], [0.95, 0.12]]           # cells (0,0) and (1,0); a repeat changes nothing
    assert O.path_distance(a, a, **GRID) == 0.0
    assert O.path_distance(a, [[5.0, 5.0]], **GRID) == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert O.path_distance(a, [[0.85, 0.7]], **GRID) == pytest.approx(math.sqrt(2.0 - math.sqrt(2.0)), rel=1e-15)


def test_points_outside_are_ignored_and_cells_are_half_open():
    a = [[0.5, 0.5], [-0.1, 3.0], [16.0, 1.0], [3.0, 16.0]]   # only (0.5, 0.5) is inside the 16 A square
    assert O.path_distance(a, [[0.5, 0.5]], **GRID) == 0.0
    # 0.8 belongs to cell 1, not cell 0
    assert O.path_distance([[0.8, 0.0]], [[0.0, 0.0]], **GRID) == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert O.path_distance([[0.8, 0.0]], [[1.5, 0.7]], **GRID) == 0.0


@pytest.mark.parametrize("seed", range(5))
def test_random_sets_against_the_set_formula(seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(8.0, 2.5, size=(300, 2))
    b = rng.normal(8.5, 2.5, size=(250, 2))

    def cells(xy):
        return {(int(math.floor(x / 0.8)), int(math.floor(y / 0.8))) for x, y in xy
                if 0 <= math.floor(x / 0.8) < 20 and 0 <= math.floor(y / 0.8) < 20}
    A, B = cells(a), cells(b)
    want = math.sqrt(max(0.0, 2.0 - 2.0 * len(A & B) / math.sqrt(len(A) * len(B))))
    assert O.path_distance(a, b, **GRID) == pytest.approx(want, rel=1e-12, abs=1e-15)
