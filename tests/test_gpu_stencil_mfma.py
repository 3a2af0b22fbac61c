"""The MFMA level stencil (MLS_STENCIL_TILE_MFMA_F32, mixed plans with
windows R <= 6): the FP32 tile recast as banded Toeplitz products on
v_mfma_f32_16x16x4_f32, selected at plan creation by MLS_STENCIL_MFMA=1.
Checked against the FP64 oracle within the mixed bound (end to end), its
e^k grids against the FP64 plan's (FP32 rounding of the grid sums), under
Lorentz-Berthelot mixing (per-vector means), and at 10^6 atoms on the
stored oracle sample."""
import json
import os

import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import force_errors, gpu_eval, say, stages

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _with_mfma(fn, *args, **kw):
    old = os.environ.get("MLS_STENCIL_MFMA")
    os.environ["MLS_STENCIL_MFMA"] = "1"
    try:
        return fn(*args, **kw)
    finally:
        if old is None:
            del os.environ["MLS_STENCIL_MFMA"]
        else:
            os.environ["MLS_STENCIL_MFMA"] = old


# name, workload, a, h, levels (windows R from 3 to 6: both kernel templates)
CASES = [
    ("cube1k_a3_h1_l2", lambda: W.named("cube1k"), 3.0, 1.0, 2),
    ("cube2k_a25_h125_l2", lambda: W.cube(2000, 0.8, seed=71), 2.5, 1.25, 2),
    ("slab_a25_h09_l3", lambda: W.slab(2000, (12.0, 12.0, 36.0), 0.3, 0.7, seed=9), 2.5, 0.9, 3),
    ("slab32k_a3_h1_l4", lambda: W.named("slab32k"), 3.0, 1.0, 4),
]


@pytest.mark.parametrize("name,make,a,h,levels", CASES, ids=[c[0] for c in CASES])
def test_mfma_stencil(name, make, a, h, levels):
    w = make()
    plan, out = _with_mfma(gpu_eval, w.pos, w.c6, w.box, a, h, 4, levels, precision="mixed")
    assert plan.info["stencil_path"] == "tile_mfma_f32"
    n1 = np.asarray(plan.info["grid"])
    R = max(int(np.floor(2 * a / hh * (1 - 1e-12))) for hh in np.asarray(w.box) / n1)
    say(f"[mfma stencil] {name}: n={w.n} R={R}")
    assert 1 <= R <= 6
    ref64, out64 = gpu_eval(w.pos, w.c6, w.box, a, h, 4, levels, precision="fp64")
    # e^k of every stencil level against the FP64 plan (same charges up to FP32 weights)
    st, st64 = stages(plan, w.n), stages(ref64, w.n)
    for k in range(levels - 1):
        de = np.max(np.abs(st["e"][k] - st64["e"][k])) / np.max(np.abs(st64["e"][k]))
        assert de < 2e-6, (k, de)
    rms, dF, mx = force_errors(out["F"], out64["F"])
    dE = abs(out["energy"] - out64["energy"]) / abs(out64["energy"])
    say(f"  vs FP64 plan: dE={dE:.2e} rmsF={rms:.2e}")
    assert dE < 1e-6 and rms < 1e-5
    if w.n <= 2000:
        ref = M.mls(w.pos, w.c6, w.box, a, h, 4, levels)
        rms, dF, mx = force_errors(out["F"], ref["F"])
        assert abs(out["energy"] - ref["energy"]) / abs(ref["energy"]) < 1e-6
        assert rms < 1e-5
    plan.close()
    ref64.close()


def test_mfma_stencil_lorentz_berthelot():
    import torch
    from paper_1308_4005_amd import Plan
    w = W.slab(2000, (12.0, 12.0, 36.0), 0.3, 0.7, seed=9)
    rng = np.random.default_rng(5)
    eps = np.where(rng.uniform(size=w.n) < 0.5, 1.0, 0.6)
    sig = np.where(rng.uniform(size=w.n) < 0.5, 1.0, 1.25)
    ref = M.mls_lb(w.pos, eps, sig, w.box, 2.5, 0.9, 4, 3)
    plan = _with_mfma(Plan, w.box, 2.5, 0.9, 4, 3, precision="mixed", n_max=w.n, mixing="lorentz-berthelot")
    assert plan.info["stencil_path"] == "tile_mfma_f32"
    t = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    r = plan.evaluate_lb(t(w.pos), t(eps), t(sig))
    torch.cuda.synchronize()
    E, F = float(r.energy.cpu()[0]), r.forces.cpu().numpy()
    rms, dF, mx = force_errors(F, ref["F"])
    assert abs(E - ref["energy"]) / abs(ref["energy"]) < 1e-6
    assert rms < 1e-5


def test_mfma_stencil_full_size_sample():
    import torch
    from paper_1308_4005_amd import Plan
    gold = json.load(open(os.path.join(GOLDEN, "cube1M_a3_h1_p4_l5.json")))
    w = W.named(gold["workload"])
    plan = _with_mfma(Plan, w.box, gold["a"], gold["h"], gold["order"], gold["levels"], precision="mixed", n_max=w.n)
    assert plan.info["stencil_path"] == "tile_mfma_f32"
    r = plan.evaluate(torch.tensor(w.pos, device="cuda"), torch.tensor(w.c6, device="cuda"))
    torch.cuda.synchronize()
    idx = np.asarray(gold["sample"])
    rms, dF, mx = force_errors(r.forces.cpu().numpy()[idx], np.asarray(gold["forces"]))
    dE = abs(float(r.energy.cpu()[0]) - gold["energy"]) / abs(gold["energy"])
    say(f"[mfma stencil] cube1M: dE={dE:.2e} rmsF={rms:.2e}")
    assert dE < 1e-6 and rms < 1e-5
