"""GPU parity of multiple time stepping (mls_md_run_mts) against the MD
oracle's r-RESPA integrator: local part + repulsion as the fast force, the
grid part as the slow force every k_slow steps.  FP64 plans: rel. 1e-10;
mixed plans: bounds from the mixed force bar."""
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
    ("cube1k_k3", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 3.0, 3),
    ("cube1k_k1", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 3.0, 1),
    ("narrow_box_k2", W.fill_box(120, (5.3, 5.3, 9.0), seed=5), dict(a=3.0, h=1.0, order=4, levels=1), 3.0, 2),
    ("slab_p6_l3_k2", W.slab(1500, (11.0, 11.0, 40.0), 0.3, 0.7, rho_liquid=0.8, rho_vapour=0.02, seed=21),
     dict(a=2.5, h=0.9, order=6, levels=3), 2.0, 2),
]


@pytest.mark.parametrize("name,w,prm,rc,k", CASES, ids=[c[0] for c in CASES])
def test_mts_fp64_matches_oracle(name, w, prm, rc, k):
    import torch
    from paper_1308_4005_amd import Plan
    say(f"[mts] {name}: n={w.n} rc={rc} k={k}")
    vel, c12, im = _inputs(w, 7)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n)
    x, v = _t(w.pos), _t(vel)
    nsteps = 2 * k
    F, ep, ek = plan.md_run_mts(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=nsteps, k_slow=k, rc=rc)
    torch.cuda.synchronize()
    assert plan.status() == 0
    xo, vo, Fo, epo, eko = MD.md_run_mts(w.pos, vel, w.c6, c12, im, w.box, prm["a"], prm["h"], prm["order"],
                                         prm["levels"], 0.002, nsteps, k, rc=rc)
    assert rel_err(x.cpu().numpy(), xo) < 1e-13
    assert rel_err(v.cpu().numpy(), vo) < TOL
    assert rel_err(F.cpu().numpy(), Fo) < TOL
    assert rel_err(ep.cpu().numpy(), epo) < TOL
    assert rel_err(ek.cpu().numpy(), eko) < 1e-12


def test_mts_with_one_inner_step_matches_md_run():
    import torch
    from paper_1308_4005_amd import Plan
    w = W.named("cube1k")
    vel, c12, im = _inputs(w, 8)
    say("[mts] k = 1 against mls_md_run")
    plan = Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n)
    x1, v1 = _t(w.pos), _t(vel)
    F1, ep1, ek1 = plan.md_run(x1, v1, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=4)
    x2, v2 = _t(w.pos), _t(vel)
    F2, ep2, ek2 = plan.md_run_mts(x2, v2, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=4, k_slow=1)
    torch.cuda.synchronize()
    for a, b in ((x2, x1), (v2, v1), (F2, F1), (ep2, ep1), (ek2, ek1)):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-12


def test_mts_mixed_and_edges():
    import torch
    from paper_1308_4005_amd import Plan, _lib
    w = W.named("cube1k")
    vel, c12, im = _inputs(w, 9)
    say("[mts] mixed k = 3")
    plan = Plan(w.box, 3.0, 1.0, 4, 2, precision="mixed", n_max=w.n)
    x, v = _t(w.pos), _t(vel)
    F, ep, ek = plan.md_run_mts(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=6, k_slow=3)
    torch.cuda.synchronize()
    assert plan.status() == 0
    xo, vo, Fo, epo, eko = MD.md_run_mts(w.pos, vel, w.c6, c12, im, w.box, 3.0, 1.0, 4, 2, 0.002, 6, 3)
    e_rep, _ = MD.repulsion(w.pos, c12, w.box, 3.0)
    assert np.abs(ep.cpu().numpy() - epo).max() < 1e-6 * (abs(epo[0] - e_rep) + abs(e_rep))
    # as for mls_md_run: per-atom force errors below 1e-4 max|F| over 6 inner steps
    dv = 6 * 0.002 * im.max() * 1e-4 * np.abs(Fo).max()
    assert np.abs(v.cpu().numpy() - vo).max() < dv
    assert np.abs(x.cpu().numpy() - xo).max() < 6 * 0.002 * dv
    say("[mts] edges: n = 0, nsteps = 0, argument errors")
    e0 = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    F, ep, ek = plan.md_run_mts(e0, e0.clone(), z, z.clone(), z.clone(), dt=0.002, nsteps=4, k_slow=2)
    torch.cuda.synchronize()
    assert np.all(ep.cpu().numpy() == 0.0) and np.all(ek.cpu().numpy() == 0.0)
    x, v = _t(w.pos), _t(vel)
    F, ep, ek = plan.md_run_mts(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=0, k_slow=3)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), w.pos) and np.array_equal(v.cpu().numpy(), vel)
    assert abs(float(ep.cpu()[0]) - epo[0]) < 1e-6 * (abs(epo[0] - e_rep) + abs(e_rep))
    with pytest.raises(_lib.MLSError):
        plan.md_run_mts(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=5, k_slow=2)
    with pytest.raises(_lib.MLSError):
        plan.md_run_mts(x, v, _t(w.c6), _t(c12), _t(im), dt=0.002, nsteps=4, k_slow=0)


@pytest.mark.timeout(600)
def test_full_size_one_inner_step_matches_md_run():
    """cube1M (10^6 atoms, the measured workload), FP64: multiple time stepping
    with k_slow = 1 (split forces: local part and repulsion, then the grid part
    alone, kicked separately) equals mls_md_run (one fused evaluation) over two
    steps, and its kinetic energy matches its own final velocities."""
    import torch
    from paper_1308_4005_amd import Plan
    w = W.named("cube1M")
    prm = w.params
    say(f"[mts] full size: n={w.n}")
    vel, c12, im = _inputs(w, 10)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n)
    c6t, c12t, imt = _t(w.c6), _t(c12), _t(im)
    x1, v1 = _t(w.pos), _t(vel)
    F1, ep1, ek1 = plan.md_run(x1, v1, c6t, c12t, imt, dt=0.001, nsteps=2)
    x2, v2 = _t(w.pos), _t(vel)
    F2, ep2, ek2 = plan.md_run_mts(x2, v2, c6t, c12t, imt, dt=0.001, nsteps=2, k_slow=1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    for a, b in ((x2, x1), (v2, v1), (F2, F1), (ep2, ep1), (ek2, ek1)):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-10
    vv = v2.cpu().numpy()
    assert float(ek2.cpu()[-1]) == pytest.approx(0.5 * np.sum(np.sum(vv * vv, axis=1) / im), rel=1e-12)
