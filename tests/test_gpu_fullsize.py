"""Full-size GPU checks against stored oracle results and invariants.

The stored values (tests/golden/*.json) come from ``tests/golden/make_golden.py``,
which runs only the FP64 oracle on the same seeded workloads; the GPU result is
compared on the stored sample of atoms (FP64: rel. 1e-10; mixed: the stated
bound) and through properties that hold at any size.
"""
import json
import os

import numpy as np
import pytest

from paper_1308_4005_amd import workloads as W

from gpu_common import force_errors, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MIXED_RMS_BOUND = 1e-5     # RMS-relative force error of the mixed path vs FP64
MIXED_E_BOUND = 1e-6


def _run(w, gold, precision):
    import torch
    from paper_1308_4005_amd import Plan
    plan = Plan(w.box, gold["a"], gold["h"], gold["order"], gold["levels"], precision=precision, n_max=w.n)
    assert list(plan.info["grid"]) == gold["grid"]
    pos = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    c6 = torch.tensor(w.c6, dtype=torch.float64, device="cuda")
    r = plan.evaluate(pos, c6, forces=True, potential=True, dE_dc6=True)
    torch.cuda.synchronize()
    out = dict(E=float(r.energy.cpu()[0]), F=r.forces.cpu().numpy(), u=r.potential.cpu().numpy(),
               d=r.dE_dc6.cpu().numpy())
    q = [plan.copy_stage("q", k).sum().item() for k in range(1, plan.info["levels"] + 1)]
    plan.close()
    return out, q


# the precision-at-scale sweep: every stored 10^6-atom setting (a in {2.5, 3,
# 4}, h in {0.8, 1, 1.25}, p in {4, 6}, five levels) besides the slab
_SWEEP = sorted(f[:-5] for f in os.listdir(GOLDEN) if f.startswith("cube1M_a") and f.endswith("_l5.json"))


@pytest.fixture(scope="module", params=["slab32k_a3_h1_p4_l4", "mixture100k_a3_h1_p4_l0"] + _SWEEP)
def golden_case(request):
    gold = json.load(open(os.path.join(GOLDEN, request.param + ".json")))
    say(f"[fullsize] {request.param}: building workload")
    w = W.named(gold["workload"])
    assert w.n == gold["n"]
    return request.param, w, gold


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_golden_sample(golden_case, precision):
    name, w, gold = golden_case
    say(f"[fullsize] {name} {precision}")
    out, qsums = _run(w, gold, precision)
    idx = np.asarray(gold["sample"])
    Fr = np.asarray(gold["forces"])
    rms, dF, mx = force_errors(out["F"][idx], Fr)
    dE = abs(out["E"] - gold["energy"]) / abs(gold["energy"])
    say(f"[fullsize] {name} {precision}: dE={dE:.3e} rmsF={rms:.3e} dF={dF:.3e} max={mx:.3e}")
    if precision == "fp64":
        assert dE < 1e-10
        assert np.max(np.abs(out["F"][idx] - Fr)) < 1e-10 * gold["force_rms"]
        np.testing.assert_allclose(out["u"][idx], gold["potential"], rtol=1e-10)
        np.testing.assert_allclose(out["d"][idx], gold["dE_dc6"], rtol=1e-10)
    else:
        assert dE < MIXED_E_BOUND
        assert rms < MIXED_RMS_BOUND
    # properties at any size: partition of unity on every level, Euler's
    # relation for the degree-1 homogeneity in C6.  The mixed path computes
    # the anterpolation weights in FP32, so its grid sums keep the partition
    # of unity to FP32 rounding (about 2e-7 for the quintic basis at 10^6
    # atoms), the FP64 path to FP64 rounding
    xi_sum = float(np.sum(np.sqrt(w.c6)))
    for s in qsums:
        assert s == pytest.approx(xi_sum, rel=1e-9 if precision == "fp64" else 1e-6)
    assert float(np.dot(w.c6, out["d"])) == pytest.approx(out["E"], rel=1e-9)
