"""Restriction and prolongation (Sec. II.B) in both forms: a thread per coarse
point, and a group of lanes per coarse point (the form small levels take).
Every level's charges, stencil sums and interpolated potentials against the
FP64 oracle (1e-12) with each form forced on every level, for both orders."""
import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import gpu_eval, rel_err, say, stages

pytestmark = pytest.mark.gpu

FORMS = {"thread_per_point": "0", "group_per_point": "100000000"}


def _cases():
    slab = W.slab(2000, (12.0, 12.0, 48.0), 0.3, 0.7, rho_liquid=0.8, rho_vapour=0.02, seed=21)
    mix = W.cube(700, 0.8, seed=24)
    aniso = W.cube(600, 0.5, seed=22)
    aniso.box = np.array([11.0, 9.0, 13.5])
    aniso.pos = np.mod(aniso.pos * aniso.box / aniso.box.max(), aniso.box)
    return [("slab2k_p4_l3", slab, dict(a=3.0, h=1.0, order=4, levels=3)),
            ("mix_p4_l4", mix, dict(a=2.2, h=0.7, order=4, levels=4)),
            ("aniso_p6_l3", aniso, dict(a=2.5, h=0.9, order=6, levels=3))]


CASES = _cases()


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("k", range(len(CASES)), ids=[c[0] for c in CASES])
def test_transfer_forms_match_oracle(k, form, monkeypatch):
    name, w, prm = CASES[k]
    monkeypatch.setenv("MLS_SPLIT_RESTRICT", FORMS[form])
    monkeypatch.setenv("MLS_SPLIT_PROLONG", FORMS[form])
    ref = M.mls(w.pos, w.c6, w.box, prm["a"], prm["h"], prm["order"], prm["levels"])
    plan, out = gpu_eval(w.pos, w.c6, w.box, prm["a"], prm["h"], prm["order"], prm["levels"])
    st = stages(plan, w.n)
    for lv in range(ref["levels"]):
        dq, de, dE = (rel_err(st[key][lv], ref[key][lv]) for key in ("q", "e", "E"))
        say(f"[transfer] {name} {form} level {lv + 1}: q {dq:.1e} e {de:.1e} E {dE:.1e}")
        assert dq < 1e-12 and de < 1e-12 and dE < 1e-12
    assert out["energy"] == pytest.approx(ref["energy"], rel=1e-10)
    plan.close()
