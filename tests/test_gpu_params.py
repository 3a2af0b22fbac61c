"""Parameter selection (Sec. III.E) on the GPU: for two targets the chosen
cutoff meets the target on a 32,000-atom cube, the spacing does not depend on
the target (eq:optimal-spacing), and a tighter target takes a larger cutoff.

The selector measures its error against an evaluation with a larger cutoff.
eq:accuracy-tolerance defines the error against the exact forces, so each
selected (a, h) is also evaluated against the exact periodic forces (Ewald,
from the oracle) of 512 sampled atoms of the same cube, stored in
tests/golden/cube32k_exact.json."""
import json
import os

import numpy as np
import pytest

from paper_1308_4005_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _exact():
    with open(os.path.join(HERE, "golden", "cube32k_exact.json")) as f:
        return json.load(f)


def test_selection_meets_the_target():
    import torch
    from paper_1308_4005_amd import Plan
    from paper_1308_4005_amd.params import select_parameters
    ex = _exact()
    w = W.cube(32000, 0.8, seed=31)
    assert ex["workload"] == "cube32k" and ex["n"] == w.n and ex["seed"] == 31
    assert np.allclose(ex["box"], w.box, rtol=0, atol=1e-12)
    idx = np.asarray(ex["sample"])
    Fex = np.asarray(ex["forces"])
    pos = torch.tensor(w.pos, device="cuda")
    c6 = torch.tensor(w.c6, device="cuda")
    sel = {}
    for target in (1e-3, 1e-4):
        s = select_parameters(pos, c6, w.box, target)
        plan = Plan(w.box, s.a, s.h, 4, 0, n_max=w.n)
        F = plan.evaluate(pos, c6).forces[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        plan.close()
        exact_err = float(np.sqrt(np.sum((F - Fex) ** 2) / np.sum(Fex ** 2)))
        say(f"[params] target {target:.0e}: a={s.a:.3f} h={s.h:.3f} l={s.levels} error={s.error:.2e} "
            f"exact error={exact_err:.2e} C_local={s.C_local:.3e} C_grids={s.C_grids:.3e} history={s.history}")
        assert 0.4 * target < s.error < 2.0 * target
        # the error of eq:accuracy-tolerance, against the exact periodic sum
        assert 0.5 * target < exact_err < 2.0 * target
        sel[target] = s
    assert sel[1e-4].a > sel[1e-3].a
    assert sel[1e-4].h == pytest.approx(sel[1e-3].h, rel=0.2)
