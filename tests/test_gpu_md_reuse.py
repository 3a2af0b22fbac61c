"""Neighbour reuse in molecular dynamics (plans with a skin): mls_md_run keeps
the sorted atoms and cells of one binning while no atom has moved more than
skin/2 since, bins again when one has, and re-gathers the positions through
the stored order otherwise.  The results must not depend on the skin: FP64
equals the MD oracle (which has no neighbour structure at all) to rel.
1e-10 over trajectories long enough that atoms move several times skin/2 and
cross the periodic boundary (a missed re-binning would lose pairs)."""
import numpy as np
import pytest

from oracle import md as MD
from paper_1308_4005_amd import workloads as W

from gpu_common import rel_err, say

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _run(w, prm, vel, c12, im, dt, nsteps, skin, precision="fp64", rc=None):
    import torch
    from paper_1308_4005_amd import Plan
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], precision=precision, n_max=w.n, skin=skin)
    x, v = _t(w.pos), _t(vel)
    F, ep, ek = plan.md_run(x, v, _t(w.c6), _t(c12), _t(im), dt=dt, nsteps=nsteps, rc=rc)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = [x.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy(), ep.cpu().numpy(), ek.cpu().numpy()]
    info = plan.info
    plan.close()
    return out, info


CASES = [
    # name, workload, params, skin, dt, steps, velocity scale
    ("cube1k_skin0.2", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 0.2, 0.004, 16, 1.5),
    ("cube1k_skin0.05", W.named("cube1k"), dict(a=3.0, h=1.0, order=4, levels=2), 0.05, 0.004, 12, 1.5),
    ("narrow_box_skin0.2", W.fill_box(120, (5.3, 5.3, 9.0), seed=5), dict(a=3.0, h=1.0, order=4, levels=1), 0.2,
     0.004, 16, 1.5),
    ("slab_p6_l3_skin0.25", W.slab(1500, (11.0, 11.0, 40.0), 0.3, 0.7, rho_liquid=0.8, rho_vapour=0.02, seed=21),
     dict(a=2.5, h=0.9, order=6, levels=3), 0.25, 0.004, 16, 1.5),
]


@pytest.mark.parametrize("name,w,prm,skin,dt,steps,vs", CASES, ids=[c[0] for c in CASES])
def test_reuse_fp64_matches_oracle(name, w, prm, skin, dt, steps, vs):
    rng = np.random.default_rng(31)
    vel = rng.normal(scale=vs, size=(w.n, 3))
    c12 = np.full(w.n, 4.0)
    im = rng.uniform(0.5, 2.0, size=w.n)
    say(f"[md reuse] {name}: n={w.n} skin={skin} dt={dt} steps={steps}")
    (x, v, F, ep, ek), info = _run(w, prm, vel, c12, im, dt, steps, skin)
    xo, vo, Fo, epo, eko = MD.md_run(w.pos, vel, w.c6, c12, im, w.box, prm["a"], prm["h"], prm["order"],
                                     prm["levels"], dt, steps)
    # the trajectory moves atoms beyond skin (at least one re-binning) and
    # across the box faces
    disp = np.max(np.linalg.norm(xo - w.pos, axis=1))
    crossed = np.any((xo < 0) | (xo >= w.box))
    say(f"  max displacement {disp:.3f} (skin/2 = {skin / 2}), crossed a face: {crossed}, cells {info['cells']}")
    assert disp > skin and crossed
    assert rel_err(x, xo) < 1e-13
    assert rel_err(v, vo) < 1e-10
    assert rel_err(F, Fo) < 1e-10
    assert rel_err(ep, epo) < 1e-10
    assert rel_err(ek, eko) < 1e-10


def test_reuse_mixed_matches_the_run_without_skin():
    w = W.named("cube1k")
    prm = dict(a=3.0, h=1.0, order=4, levels=2)
    rng = np.random.default_rng(32)
    vel = rng.normal(scale=1.5, size=(w.n, 3))
    c12 = np.full(w.n, 4.0)
    im = np.ones(w.n)
    say("[md reuse] mixed, skin 0.2 against no skin")
    a, _ = _run(w, prm, vel, c12, im, 0.004, 16, 0.0, precision="mixed")
    b, _ = _run(w, prm, vel, c12, im, 0.004, 16, 0.2, precision="mixed")
    # same pairs and grids, FP32 pair terms summed in another order (other
    # cells): within the mixed bars over the run.  The energy bar is scaled
    # by |E_disp| + |E_rep| as in the other MD tests: E_pot is their
    # difference and cancels to a fraction of either
    Fr = np.abs(a[2]).max()
    assert np.abs(b[2] - a[2]).max() < 1e-4 * Fr
    e_rep, _ = MD.repulsion(w.pos, c12, w.box, 3.0)
    scale = abs(a[3][0] - e_rep) + abs(e_rep)
    assert np.abs(b[3] - a[3]).max() < 1e-6 * scale
    dv = 16 * 0.004 * 1e-4 * Fr
    assert np.abs(b[1] - a[1]).max() < dv


def test_skin_is_validated_and_widens_cells():
    from paper_1308_4005_amd import Plan, _lib
    w = W.named("cube1k")
    p0 = Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n)
    p1 = Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n, skin=0.5)
    assert all(c1 * 1.0 <= c0 for c0, c1 in zip(p0.info["cells"], p1.info["cells"]))
    assert all(cw >= 0.5 * 3.5 - 1e-12 for cw in p1.info["cell_width"])
    for bad in (-0.1, 3.0, float("nan")):
        with pytest.raises(_lib.MLSError):
            Plan(w.box, 3.0, 1.0, 4, 2, n_max=w.n, skin=bad)
    p0.close()
    p1.close()
