"""Parameter selection (Sec. III.E) on the GPU: for two targets the chosen
cutoff meets the target on a 32,000-atom cube, the spacing does not depend on
the target (eq:optimal-spacing), and a tighter target takes a larger cutoff."""
import pytest

from paper_1308_4005_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu


def test_selection_meets_the_target():
    import torch
    from paper_1308_4005_amd.params import select_parameters
    w = W.cube(32000, 0.8, seed=31)
    pos = torch.tensor(w.pos, device="cuda")
    c6 = torch.tensor(w.c6, device="cuda")
    sel = {}
    for target in (1e-3, 1e-4):
        s = select_parameters(pos, c6, w.box, target)
        say(f"[params] target {target:.0e}: a={s.a:.3f} h={s.h:.3f} l={s.levels} error={s.error:.2e} "
            f"C_local={s.C_local:.3e} C_grids={s.C_grids:.3e} history={s.history}")
        assert 0.4 * target < s.error < 2.0 * target
        sel[target] = s
    assert sel[1e-4].a > sel[1e-3].a
    assert sel[1e-4].h == pytest.approx(sel[1e-3].h, rel=0.2)
