"""Differentiable form: torch.autograd through MLSDispersion against central
finite differences of the GPU energy (step 1e-5) and against the oracle's
analytic gradient, on the binary-mixture workload (100,000 atoms, C6 in
{4, 9}) and on a small cube."""
import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu


def _energy(plan, pos, c6):
    import torch
    r = plan.evaluate(pos, c6, forces=False)
    torch.cuda.synchronize()
    return float(r.energy.cpu()[0])


@pytest.fixture(scope="module")
def mixture():
    import torch
    from paper_1308_4005_amd import Plan
    say("[autograd] building mixture100k")
    w = W.named("mixture100k")
    plan = Plan(w.box, 3.0, 1.0, 4, 0, precision="fp64", n_max=w.n)
    pos = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    c6 = torch.tensor(w.c6, dtype=torch.float64, device="cuda")
    return w, plan, pos, c6


def test_backward_matches_finite_differences(mixture):
    import torch
    from paper_1308_4005_amd import MLSDispersion
    w, plan, pos, c6 = mixture
    p = pos.clone().requires_grad_(True)
    c = c6.clone().requires_grad_(True)
    E = MLSDispersion.apply(p, c, plan)
    E.backward()
    E0 = float(E.detach().cpu())
    gpos = p.grad.cpu().numpy()
    gc6 = c.grad.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(55))
    atoms = rng.choice(w.n, size=64, replace=False)
    h = 1e-5
    # central differences of a total energy |E| ~ 1e6 resolve derivatives only
    # to a few ulps of E over 2h: allow 20 ulps plus 1e-6 relative
    noise = 20 * np.spacing(abs(E0)) / (2 * h)
    worst = 0.0
    for i in atoms:
        for d in range(3):
            pp = pos.clone()
            pp[i, d] += h
            Ep = _energy(plan, pp, c6)
            pp[i, d] -= 2 * h
            Em = _energy(plan, pp, c6)
            fd = (Ep - Em) / (2 * h)
            err = abs(fd - gpos[i, d])
            worst = max(worst, err / (noise + 1e-6 * abs(gpos[i, d])))
        cc = c6.clone()
        cc[i] += h
        Ep = _energy(plan, pos, cc)
        cc[i] -= 2 * h
        Em = _energy(plan, pos, cc)
        fd = (Ep - Em) / (2 * h)
        worst = max(worst, abs(fd - gc6[i]) / (noise + 1e-6 * abs(gc6[i])))
    say(f"[autograd] FD (step {h}) vs backward on 64 atoms: worst error / tolerance = {worst:.3f} "
        f"(tolerance {noise:.2e} + 1e-6 rel)")
    # Phi is C1: within h of a knot plane the FD error is O(h), which the
    # 20-ulp allowance covers at this step
    assert worst < 1.0


def test_backward_matches_wide_step_differences(mixture):
    # E depends on C6_i through sqrt(C6_i) and C6_i, so a central difference
    # has truncation error ~ h^2 / (8 C6^2) relative (8e-9 at h = 1e-3, C6 = 4)
    # and rounding noise ~ 20 ulp(E) / 2h (~1e-6 relative here)
    from paper_1308_4005_amd import MLSDispersion
    w, plan, pos, c6 = mixture
    c = c6.clone().requires_grad_(True)
    E = MLSDispersion.apply(pos, c, plan)
    E.backward()
    gc6 = c.grad.cpu().numpy()
    h = 1e-3
    for i in (3, 777, 50000):
        cc = c6.clone()
        cc[i] += h
        Ep = _energy(plan, pos, cc)
        cc[i] -= 2 * h
        Em = _energy(plan, pos, cc)
        assert (Ep - Em) / (2 * h) == pytest.approx(gc6[i], rel=3e-6)


def test_backward_equals_stored_oracle_gradient(mixture):
    # the 100,000-atom mixture: gradients on the 512 atoms the oracle stored
    # (tests/golden/mixture100k_a3_h1_p4_l0.json, written by make_golden.py)
    import json
    import os
    import torch
    from paper_1308_4005_amd import MLSDispersion
    w, plan, pos, c6 = mixture
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mixture100k_a3_h1_p4_l0.json")))
    assert gold["n"] == w.n and list(plan.info["grid"]) == gold["grid"]
    p = pos.clone().requires_grad_(True)
    c = c6.clone().requires_grad_(True)
    E = MLSDispersion.apply(p, c, plan)
    E.backward()
    idx = np.asarray(gold["sample"])
    assert float(E.detach().cpu()) == pytest.approx(gold["energy"], rel=1e-10)
    np.testing.assert_allclose(p.grad.cpu().numpy()[idx], -np.asarray(gold["forces"]), rtol=0,
                               atol=1e-10 * gold["force_rms"])
    np.testing.assert_allclose(c.grad.cpu().numpy()[idx], gold["dE_dc6"], rtol=1e-10)


def test_backward_equals_oracle_gradient():
    import torch
    from paper_1308_4005_amd import MLSDispersion, Plan
    w = W.cube(400, 0.8, seed=41)
    w.c6 = np.where(np.arange(w.n) % 2 == 0, 4.0, 9.0)
    ref = M.mls(w.pos, w.c6, w.box, 2.5, 0.8, 4, 2)
    plan = Plan(w.box, 2.5, 0.8, 4, 2, n_max=w.n)
    p = torch.tensor(w.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    c = torch.tensor(w.c6, dtype=torch.float64, device="cuda", requires_grad=True)
    E = MLSDispersion.apply(p, c, plan)
    (2.0 * E).backward()
    assert float(E.detach().cpu()) == pytest.approx(ref["energy"], rel=1e-10)
    np.testing.assert_allclose(p.grad.cpu().numpy(), -2.0 * ref["F"], rtol=0, atol=1e-9 * np.abs(ref["F"]).max())
    np.testing.assert_allclose(c.grad.cpu().numpy(), 2.0 * ref["dE_dc6"], rtol=1e-10)


def test_energy_is_translation_invariant_on_coarsest_lattice():
    import torch
    from paper_1308_4005_amd import Plan
    w = W.cube(500, 0.8, seed=42)
    plan = Plan(w.box, 2.5, 0.9, 4, 2, n_max=w.n)
    hl = np.asarray(plan.info["h_eff"]) * 2
    E0 = _energy(plan, torch.tensor(w.pos, device="cuda"), torch.tensor(w.c6, device="cuda"))
    E1 = _energy(plan, torch.tensor(w.pos + hl, device="cuda"), torch.tensor(w.c6, device="cuda"))
    perm = np.random.default_rng(0).permutation(w.n)
    E2 = _energy(plan, torch.tensor(w.pos[perm], device="cuda"), torch.tensor(w.c6[perm], device="cuda"))
    assert E1 == pytest.approx(E0, rel=1e-12)
    assert E2 == pytest.approx(E0, rel=1e-12)
