"""GPU parity of multiple time stepping per MLS level (mls_md_run_mts_levels)
against the MD oracle: local part + repulsion every step, the level-1 grid
part every k_mid steps, levels 2..l every k_mid k_slow steps.  FP64 plans:
rel. 1e-10; mixed plans: bounds from the mixed force bar."""
import numpy as np
import pytest

from oracle import md as MD
from paper_1308_4005_amd import workloads as W

from gpu_common import rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _inputs(w, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(scale=0.3, size=(w.n, 3)), np.where(rng.uniform(size=w.n) < 0.5, 4.0, 2.5),
            rng.uniform(0.5, 2.0, size=w.n))


CASES = [
    ("cube1k_l2_m2_s2", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 3.0, 2, 2),
    ("cube1k_l2_m1_s3", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 3.0, 1, 3),
    ("cube1k_l2_m3_s1", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 3.0, 3, 1),
    ("narrow_box_l1_m2_s2", W.fill_box(120, (5.3, 5.3, 9.0), seed=5), dict(a=3.0, h=1.0, order=4, levels=1), 3.0,
     2, 2),
    ("slab_p6_l3_m2_s2", W.slab(1500, (11.0, 11.0, 40.0), 0.3, 0.7, rho_liquid=0.8, rho_vapour=0.02, seed=21),
     dict(a=2.5, h=0.9, order=6, levels=3), 2.0, 2, 2),
]


@pytest.mark.parametrize("name,w,prm,rc,km,ks", CASES, ids=[c[0] for c in CASES])
def test_levels_mts_fp64_matches_oracle(name, w, prm, rc, km, ks):
    import torch
    from paper_1308_4005_amd import Plan
    say(f"[mts levels] {name}: n={w.n} rc={rc} k_mid={km} k_slow={ks}")
    vel, c12, im = _inputs(w, 11)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n)
    x, v = _t(w.pos), _t(vel)
    nsteps = 2 * km * ks
    F, ep, ek = plan.md_run_mts_levels(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=nsteps, k_mid=km,
                                       k_slow=ks, rc=rc)
    torch.cuda.synchronize()
    assert plan.status() == 0
    xo, vo, Fo, epo, eko = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, im, w.box, prm["a"], prm["h"],
                                                prm["order"], prm["levels"], 0.002, nsteps, km, ks, rc=rc)
    assert rel_err(x.cpu().numpy(), xo) < 1e-13
    assert rel_err(v.cpu().numpy(), vo) < TOL
    assert rel_err(F.cpu().numpy(), Fo) < TOL
    assert rel_err(ep.cpu().numpy(), epo) < TOL
    assert rel_err(ek.cpu().numpy(), eko) < 1e-12


def test_levels_mts_reduces_to_two_scales_and_verlet():
    import torch
    from paper_1308_4005_amd import Plan
    w = W.named("cube1k")
    vel, c12, im = _inputs(w, 12)
    plan = Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n)
    say("[mts levels] k_slow = 1 against mls_md_run_mts, k_mid = k_slow = 1 against mls_md_run")
    x1, v1 = _t(w.pos), _t(vel)
    r1 = plan.md_run_mts(x1, v1, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=4, k_slow=2)
    x2, v2 = _t(w.pos), _t(vel)
    r2 = plan.md_run_mts_levels(x2, v2, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=4, k_mid=2, k_slow=1)
    x3, v3 = _t(w.pos), _t(vel)
    r3 = plan.md_run(x3, v3, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=2)
    x4, v4 = _t(w.pos), _t(vel)
    r4 = plan.md_run_mts_levels(x4, v4, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=2, k_mid=1, k_slow=1)
    torch.cuda.synchronize()
    for a, b in zip((x2, v2) + tuple(r2), (x1, v1) + tuple(r1)):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-12
    for a, b in zip((x4, v4) + tuple(r4), (x3, v3) + tuple(r3)):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-12


def test_levels_mts_mixed_and_edges():
    import torch
    from paper_1308_4005_amd import Plan, _lib
    w = W.named("cube1k")
    vel, c12, im = _inputs(w, 13)
    say("[mts levels] mixed k_mid = 2, k_slow = 2")
    plan = Plan(w.box, 3.0, 1.0, 4, 2, precision="mixed", n_max=w.n)
    x, v = _t(w.pos), _t(vel)
    F, ep, ek = plan.md_run_mts_levels(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=8, k_mid=2, k_slow=2)
    torch.cuda.synchronize()
    assert plan.status() == 0
    xo, vo, Fo, epo, eko = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, im, w.box, 3.0, 1.0, 4, 2, 0.002, 8, 2, 2)
    e_rep, _ = MD.repulsion(w.pos, c12, w.box, 3.0)
    assert np.abs(ep.cpu().numpy() - epo).max() < 1e-6 * (abs(epo[0] - e_rep) + abs(e_rep))
    # per-atom force errors below 1e-4 max|F| over 8 inner steps (as mls_md_run_mts)
    dv = 8 * 0.002 * im.max() * 1e-4 * np.abs(Fo).max()
    assert np.abs(v.cpu().numpy() - vo).max() < dv
    assert np.abs(x.cpu().numpy() - xo).max() < 8 * 0.002 * dv
    say("[mts levels] edges: n = 0, nsteps = 0, argument errors")
    e0 = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    F, ep, ek = plan.md_run_mts_levels(e0, e0.clone(), z, z.clone(), z.clone(), dt=0.002, nsteps=4, k_mid=2,
                                       k_slow=2)
    torch.cuda.synchronize()
    assert np.all(ep.cpu().numpy() == 0.0) and np.all(ek.cpu().numpy() == 0.0)
    x, v = _t(w.pos), _t(vel)
    F, ep, ek = plan.md_run_mts_levels(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=0, k_mid=2, k_slow=3)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), w.pos) and np.array_equal(v.cpu().numpy(), vel)
    assert abs(float(ep.cpu()[0]) - epo[0]) < 1e-6 * (abs(epo[0] - e_rep) + abs(e_rep))
    for km, ks, ns in ((2, 2, 6), (0, 2, 4), (2, 0, 4)):
        with pytest.raises(_lib.MLSError):
            plan.md_run_mts_levels(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=ns, k_mid=km, k_slow=ks)


@pytest.mark.timeout(600)
def test_full_size_levels_mts_equals_two_scales():
    """cube1M (10^6 atoms), FP64: with k_slow = 1 the per-level scheme (level 1
    and levels 2..5 kicked separately at the same instants) equals the
    two-scale mls_md_run_mts over one outer step of two inner steps."""
    import torch
    from paper_1308_4005_amd import Plan
    w = W.named("cube1M")
    prm = w.params
    say(f"[mts levels] full size: n={w.n}")
    vel, c12, im = _inputs(w, 14)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n)
    c6t, c12t, imt = _t(w.c6), _t(c12), _t(im)
    x1, v1 = _t(w.pos), _t(vel)
    r1 = plan.md_run_mts(x1, v1, c6t, c12t, imt, dt=0.001, nsteps=2, k_slow=2)
    x2, v2 = _t(w.pos), _t(vel)
    r2 = plan.md_run_mts_levels(x2, v2, c6t, c12t, imt, dt=0.001, nsteps=2, k_mid=2, k_slow=1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    for a, b in zip((x2, v2) + tuple(r2), (x1, v1) + tuple(r1)):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-10
