"""Discretisation error against the exact periodic sum (stored Ewald forces of
512 atoms of the 32,000-atom cube, tests/golden/cube32k_exact.json) at the
1M-atom parameters a = 3, h = 1, p = 4: the FP64 path has the oracle's error
(the two agree to 1e-10), and the FP32-mixed path's own rounding error is far
below the method's, so its error against the exact sum is the same to 1%."""
import json
import os

import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import force_errors, gpu_eval, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_error_against_the_exact_sum():
    with open(os.path.join(GOLDEN, "cube32k_exact.json")) as f:
        g = json.load(f)
    w = W.cube(g["n"], g["density"], seed=g["seed"])
    idx = np.asarray(g["sample"])
    Fx = np.asarray(g["forces"])
    say("[exact] oracle on the 32,000-atom cube")
    ro = M.mls(w.pos, w.c6, w.box, 3.0, 1.0, 4, 0)
    e_or = force_errors(ro["F"][idx], Fx)
    errs = {}
    for p in ("fp64", "mixed"):
        say(f"[exact] {p}")
        plan, r = gpu_eval(w.pos, w.c6, w.box, 3.0, 1.0, 4, 0, precision=p)
        assert plan.info["levels"] == ro["levels"]
        plan.close()
        errs[p] = force_errors(r["F"][idx], Fx)
    say(f"[exact] rms/paper/max oracle {e_or} fp64 {errs['fp64']} mixed {errs['mixed']}")
    np.testing.assert_allclose(errs["fp64"], e_or, rtol=1e-6)
    np.testing.assert_allclose(errs["mixed"], errs["fp64"], rtol=1e-2)
    assert errs["fp64"][1] < 2e-3
