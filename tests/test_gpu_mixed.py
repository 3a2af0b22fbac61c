"""FP32-mixed path against the FP64 oracle: the deviation must stay below the
stated bound (RMS-relative force error 1e-5, energy 1e-6) on every case."""
import numpy as np
import pytest

from oracle import mls as M

from gpu_common import force_errors, gpu_eval, say
from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mixed_within_bound(case):
    name, w, prm = case
    ref = M.mls(w.pos, w.c6, w.box, prm["a"], prm["h"], prm["order"], prm["levels"])
    plan, out = gpu_eval(w.pos, w.c6, w.box, prm["a"], prm["h"], prm["order"], prm["levels"],
                         precision="mixed")
    rms, dF, mx = force_errors(out["F"], ref["F"])
    dE = abs(out["energy"] - ref["energy"]) / abs(ref["energy"])
    say(f"[mixed] {name}: dE={dE:.3e} rmsF={rms:.3e} dF={dF:.3e} max={mx:.3e}")
    assert dE < 1e-6
    assert rms < 1e-5
    assert np.max(np.abs(out["u"] - ref["u"])) < 1e-5 * np.max(np.abs(ref["u"]))
