"""The two anterpolation paths of single plans give the same charges: the
two-phase blocked path (per cell block an LDS tile over the points its atoms
reach, then a per-point sum of the tiles) and the owner-computes path with
halo atoms (taken when the blocking does not fit).  Both equal the FP64
oracle's q^1 (1e-12); they agree with each other to rounding order (1e-13),
for both bases, in both precisions, on several box shapes, and the blocked
path raises no consistency flag.  The blocked path has two LDS tile sizes
(14^3 and 16^3 points); a fine grid (one cell 8.3 spacings wide) needs the
larger one."""
import os

import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import rel_err, say

pytestmark = pytest.mark.gpu


def _cases():
    slab = W.slab(3000, (12.0, 12.0, 48.0), 0.3, 0.7, rho_liquid=0.8, rho_vapour=0.02, seed=31)
    cube = W.cube(20000, 0.8, seed=32)
    aniso = W.cube(5000, 0.6, seed=33)
    aniso.box = np.array([19.0, 23.0, 31.0])
    aniso.pos = np.mod(aniso.pos * aniso.box / aniso.box.max(), aniso.box)
    # a = 2.5, h = 0.15: a 1.25-wide cell spans 8.3 grid spacings, so a block of
    # one cell reaches 15 points per dimension at p = 6 (15^3 > 14^3)
    fine = W.cube(600, 0.6, seed=34)
    return [("slab3k_p4", slab, 3.0, 1.0, 4), ("cube20k_p4", cube, 3.0, 1.0, 4),
            ("cube20k_p6", cube, 3.0, 0.8, 6), ("aniso5k_p6", aniso, 2.5, 0.9, 6),
            ("aniso5k_p4_h07", aniso, 2.5, 0.7, 4), ("fine600_p6_h015", fine, 2.5, 0.15, 6)]


def _q1(w, a, h, order, precision, tiles):
    import torch
    from paper_1308_4005_amd import Plan
    old = os.environ.get("MLS_ANTERP_TILES")
    os.environ["MLS_ANTERP_TILES"] = "1" if tiles else "0"
    try:
        plan = Plan(w.box, a, h, order, 2, precision=precision, n_max=w.n)
    finally:
        if old is None:
            del os.environ["MLS_ANTERP_TILES"]
        else:
            os.environ["MLS_ANTERP_TILES"] = old
    tp = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    tc = torch.tensor(w.c6, dtype=torch.float64, device="cuda")
    r = plan.evaluate(tp, tc)
    q = plan.copy_stage("q", 1).cpu().numpy()
    F = r.forces.cpu().numpy()
    assert plan.status() == 0
    n1 = plan.info["grid"]
    plan.close()
    return q, F, n1


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blocked_anterpolation_matches(case, precision):
    name, w, a, h, order = case
    say(f"[anterp] {name} {precision}")
    qt, Ft, n1 = _q1(w, a, h, order, precision, True)
    qo, Fo, _ = _q1(w, a, h, order, precision, False)
    assert rel_err(qt, qo) < 1e-13
    assert rel_err(Ft, Fo) < 1e-12
    if precision == "fp64":
        # the oracle's anterpolation alone (eq:anterpolation)
        q1 = M.anterpolate(M.wrap(w.pos, w.box), np.sqrt(w.c6), w.box, np.array(n1), order)
        assert rel_err(qt, q1.reshape(qt.shape)) < 1e-12
