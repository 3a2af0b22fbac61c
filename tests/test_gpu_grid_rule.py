"""The library resolves the same grids and levels as the pinned oracle rule:
the grids the paper quotes for its slab (Sec. III.C, Tables I and II) and
the auto level rule on the workload boxes."""
import numpy as np
import pytest

from oracle import mls as M

from gpu_common import say

pytestmark = pytest.mark.gpu

SLAB = (11.01, 11.01, 176.16)
CASES = [
    (SLAB, 0.92, 3, [12, 12, 192]),       # Sec. III.C
    (SLAB, 2.75, 3, [4, 4, 64]),          # Table I
    (SLAB, 1.38, 3, [8, 8, 128]),
    (SLAB, 0.69, 3, [16, 16, 256]),
    (SLAB, 0.688, 5, [16, 16, 256]),      # Table II
]


@pytest.mark.parametrize("box,h,levels,grid", CASES)
def test_library_grid_matches_paper(box, h, levels, grid):
    from paper_1308_4005_amd import Plan
    say(f"[grid rule] box={box} h={h} l={levels}")
    plan = Plan(box, 3.0, h, 4, levels, n_max=1)
    assert list(plan.info["grid"]) == grid
    n1, h1 = M.resolve_grid(box, h, levels)
    assert list(n1) == grid
    assert np.allclose(plan.info["h_eff"], h1, rtol=0, atol=1e-15)
    plan.close()


@pytest.mark.parametrize("box,levels", [((10.77,) * 3, 2), ((28.884, 28.884, 115.534), 4)])
def test_library_auto_levels(box, levels):
    from paper_1308_4005_amd import Plan
    plan = Plan(box, 3.0, 1.0, 4, 0, n_max=1)
    assert plan.info["levels"] == levels == M.resolve_levels(box, 1.0, 4)
    plan.close()
