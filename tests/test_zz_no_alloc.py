"""scps_path_distance_noalloc (the convergence measure with its scratch in a
fixed device array, for callers that cannot allocate) against
scps_path_distance, both through the C ABI, on two calls in a row -- the
second with a smaller input, so whatever the first left in the shared array
must not leak into it -- and against the oracle's plain definition."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02180_amd import scps
    return scps


def _points(n, seed, lo, hi):
    import torch
    rng = np.random.default_rng(seed)
    xy = rng.uniform(lo, hi, size=(n, 2)).astype(np.float32)
    return xy, torch.as_tensor(xy, device="cuda")


def test_noalloc_variant_matches_path_distance_on_two_calls(S):
    # call 1: the largest grid (2^20 cells) and many points; call 2: a small grid, few points
    cases = [(1024, 1024, 0.05, 400_000, 300_000, (-1.0, 52.0)),
             (40, 30, 0.25, 3000, 5000, (-0.5, 9.0))]
    for nx, ny, cell, na, nb, (lo, hi) in cases:
        a, ta = _points(na, 11 + nx, lo, hi)
        b, tb = _points(nb, 12 + ny, lo + 0.3, hi - 0.2)
        d_ref = S.path_distance(ta, tb, 0.0, 0.0, cell, nx, ny)
        d_new = S.path_distance_noalloc(ta, tb, 0.0, 0.0, cell, nx, ny)
        want = O.path_distance(a, b, 0.0, 0.0, cell, nx, ny)
        print(f"  grid {nx} x {ny}, {na} + {nb} points: D {d_new:.12f} (allocating call {d_ref:.12f}, "
              f"oracle {want:.12f})", flush=True)
        assert d_new == d_ref
        assert abs(d_new - want) <= 1e-12
    # the call after the small one with the large grid again: still the allocating call's result
    nx, ny, cell, na, nb, (lo, hi) = cases[0]
    a, ta = _points(na, 99, lo, hi)
    b, tb = _points(nb, 98, lo, hi)
    assert S.path_distance_noalloc(ta, tb, 0.0, 0.0, cell, nx, ny) == S.path_distance(ta, tb, 0.0, 0.0, cell, nx, ny)


def test_noalloc_variant_rejects_grids_beyond_its_array(S):
    a, ta = _points(100, 1, 0.0, 10.0)
    with pytest.raises(S.ScpsError) as e:
        S.path_distance_noalloc(ta, ta, 0.0, 0.0, 0.01, 1025, 1024)
    assert e.value.status == -2
    with pytest.raises(S.ScpsError) as e:          # no point inside the grid
        S.path_distance_noalloc(ta, ta, 100.0, 100.0, 1.0, 8, 8)
    assert e.value.status == -1
    assert S.path_distance_noalloc(ta, ta, 0.0, 0.0, 1.0, 10, 10) == 0.0
