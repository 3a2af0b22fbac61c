"""Lorentz-Berthelot mixing on the GPU (mls_evaluate_lb, Sec. II.D): against
the FP64 oracle (1e-10) on two-species systems for both interpolation orders,
a box narrower than 2a and a non-default smoothing member; the mixed-precision
plans against the same oracle within the mixed bound; equal sigma equals the
geometric evaluation; calls that do not match the plan are refused."""
import ctypes

import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import force_errors, rel_err, say

pytestmark = pytest.mark.gpu


def _species(n, seed):
    rng = np.random.default_rng(seed)
    eps = np.where(rng.uniform(size=n) < 0.5, 1.0, 0.6)
    sig = np.where(rng.uniform(size=n) < 0.5, 1.0, 1.25)
    return eps, sig


# mixed precision: the bounds of the geometric mixed path (RMS-relative force
# error, relative energy error)
MIXED_RMS_BOUND = 1e-5
MIXED_E_BOUND = 1e-6


def _lb_eval(w, eps, sig, prm, continuity=2, precision="fp64"):
    import torch
    from paper_1308_4005_amd import Plan
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n, continuity=continuity,
                mixing="lorentz-berthelot", precision=precision)
    r = plan.evaluate_lb(torch.tensor(w.pos, device="cuda"), torch.tensor(eps, device="cuda"),
                         torch.tensor(sig, device="cuda"))
    torch.cuda.synchronize()
    return plan, float(r.energy.cpu()[0]), r.forces.cpu().numpy()


CASES = [
    ("cube1k_p4", lambda: W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 2),
    ("cube1k_p6", lambda: W.named("cube1k"), dict(a=3.0, h=1.0, order=6, levels=2), 2),
    ("narrow_l1", lambda: W.fill_box(120, (5.3, 5.3, 9.0), seed=5), dict(a=3.0, h=1.0, order=4, levels=1), 2),
    ("slab_l3_c3", lambda: W.slab(2000, (12.0, 12.0, 36.0), 0.3, 0.7, seed=9), dict(a=2.5, h=0.9, order=4, levels=3), 3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_lb_matches_oracle(case):
    name, make, prm, k = case
    w = make()
    eps, sig = _species(w.n, 17)
    ref = M.mls_lb(w.pos, eps, sig, w.box, prm["a"], prm["h"], prm["order"], prm["levels"], continuity=k)
    plan, E, F = _lb_eval(w, eps, sig, prm, continuity=k)
    assert plan.info["mixing"] == 1
    dE = abs(E - ref["energy"]) / abs(ref["energy"])
    say(f"[lb] {name}: dE={dE:.2e} F={rel_err(F, ref['F']):.2e}")
    assert dE < 1e-10
    assert rel_err(F, ref["F"]) < 1e-10


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_lb_mixed_matches_oracle(case):
    name, make, prm, k = case
    w = make()
    eps, sig = _species(w.n, 17)
    ref = M.mls_lb(w.pos, eps, sig, w.box, prm["a"], prm["h"], prm["order"], prm["levels"], continuity=k)
    plan, E, F = _lb_eval(w, eps, sig, prm, continuity=k, precision="mixed")
    rms, dF, mx = force_errors(F, ref["F"])
    dE = abs(E - ref["energy"]) / abs(ref["energy"])
    say(f"[lb mixed] {name}: dE={dE:.2e} rmsF={rms:.2e} max={mx:.2e}")
    assert dE < MIXED_E_BOUND
    assert rms < MIXED_RMS_BOUND


def test_lb_mixed_slab_against_fp64():
    # the 32,000-atom slab (four levels, the FP32 stencil on every level but
    # the coarsest): mixed against the FP64 plan, which the cases above pin to
    # the oracle
    w = W.named("slab32k")
    eps, sig = _species(w.n, 23)
    prm = dict(a=3.0, h=1.0, order=4, levels=4)
    _, E64, F64 = _lb_eval(w, eps, sig, prm)
    plan, E32, F32 = _lb_eval(w, eps, sig, prm, precision="mixed")
    assert plan.info["stencil_path"] == "tile_f32"
    rms, dF, mx = force_errors(F32, F64)
    dE = abs(E32 - E64) / abs(E64)
    say(f"[lb mixed] slab32k: dE={dE:.2e} rmsF={rms:.2e} max={mx:.2e}")
    assert dE < MIXED_E_BOUND
    assert rms < MIXED_RMS_BOUND


def test_equal_sigma_equals_geometric():
    import torch
    from paper_1308_4005_amd import Plan
    w = W.named("cube1k")
    eps, _ = _species(w.n, 3)
    sig = np.full(w.n, 1.1)
    prm = dict(a=3.0, h=1.0, order=4, levels=2)
    _, E, F = _lb_eval(w, eps, sig, prm)
    g = Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n)
    r = g.evaluate(torch.tensor(w.pos, device="cuda"), torch.tensor(2.0 * eps * sig ** 6, device="cuda"))
    torch.cuda.synchronize()
    assert E == pytest.approx(float(r.energy.cpu()[0]), rel=1e-12)
    assert rel_err(F, r.forces.cpu().numpy()) < 1e-12


def test_bad_sigma_is_flagged():
    import torch
    w = W.named("cube1k")
    eps, sig = _species(w.n, 5)
    sig[7] = -1.0
    prm = dict(a=3.0, h=1.0, order=4, levels=2)
    plan, _, _ = _lb_eval(w, eps, sig, prm)
    assert plan.status() & 2


def test_mismatched_calls_are_refused():
    import torch
    from paper_1308_4005_amd import BatchPlan, MLSError, Plan, _lib, _params
    plan = Plan((10.0, 10.0, 10.0), 3.0, 1.0, 4, 2, n_max=10, mixing="lorentz-berthelot")
    pos = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    c6 = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(MLSError):
        plan.evaluate(pos, c6)
    geo = Plan((10.0, 10.0, 10.0), 3.0, 1.0, 4, 2, n_max=10)
    with pytest.raises(MLSError):
        geo.evaluate_lb(pos, c6, c6)
    bl = BatchPlan([(10.0, 10.0, 10.0)], [4], 3.0, 1.0, 4, 2, mixing="lorentz-berthelot")
    with pytest.raises(MLSError):
        bl.evaluate(pos, c6)
    bg = BatchPlan([(10.0, 10.0, 10.0)], [4], 3.0, 1.0, 4, 2)
    with pytest.raises(MLSError):
        bg.evaluate_lb(pos, c6, c6)
    # boxes of one batch share the mixing rule
    lib = _lib.load()
    prm = (_lib.MLSParams * 2)()
    prm[0] = _params((10.0,) * 3, 3.0, 1.0, 4, 2, None, "fp64", 2, "geometric")
    prm[1] = _params((10.0,) * 3, 3.0, 1.0, 4, 2, None, "fp64", 2, "lorentz-berthelot")
    out = ctypes.c_void_p()
    st = lib.mls_batch_create(2, prm, (ctypes.c_int64 * 2)(4, 4), 0, ctypes.byref(out))
    assert st == _lib.MLS_ERR_INVALID_ARG and not out.value
