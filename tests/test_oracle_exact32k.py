"""The stored exact forces of the 32,000-atom cube (tests/golden/cube32k_exact.json,
written by make_exact.py from oracle.exact alone) are pinned independently of
the Ewald splitting used to make them: recomputed at another screening
parameter they agree to rounding (the exact sum does not depend on it).  The
oracle's MLS error against them, at the 1M-atom parameters a = 3, h = 1, p = 4,
is below every entry of Table I (Sec. III.C, a = 3): the RSA cube has larger
per-atom forces than the paper's minimised slab, so only the bound carries
over."""
import json
import os

import numpy as np
import pytest

from oracle import exact
from oracle import mls as M
from paper_1308_4005_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cube32k():
    with open(os.path.join(GOLDEN, "cube32k_exact.json")) as f:
        g = json.load(f)
    w = W.cube(g["n"], g["density"], seed=g["seed"])
    return w, g


def test_golden_describes_the_seeded_cube(cube32k):
    w, g = cube32k
    np.testing.assert_allclose(w.box, g["box"], rtol=0, atol=0)
    idx = np.asarray(g["sample"])
    assert len(idx) == 512 and len(set(idx.tolist())) == 512 and idx.max() < w.n


def test_exact_forces_do_not_depend_on_the_screening(cube32k):
    w, g = cube32k
    sel = np.array([0, 101, 511])
    idx = np.asarray(g["sample"])[sel]
    xi = np.sqrt(w.c6)
    u, gr = exact.ewald_field(w.pos, xi, w.box, beta=0.15, targets=idx, chunk=64)
    F = xi[idx, None] * gr
    Fg = np.asarray(g["forces"])[sel]
    np.testing.assert_allclose(F, Fg, rtol=0, atol=1e-10 * np.abs(Fg).max())
    np.testing.assert_allclose(u, np.asarray(g["potential"])[sel], rtol=1e-11)


def test_oracle_error_at_the_1M_parameters_is_below_table1(cube32k):
    w, g = cube32k
    with open(os.path.join(GOLDEN, "paper_table1.json")) as f:
        t1 = json.load(f)
    r = M.mls(w.pos, w.c6, w.box, 3.0, 1.0, 4, 0)
    idx = np.asarray(g["sample"])
    Fr = np.asarray(g["forces"])
    dF = np.mean(np.linalg.norm(r["F"][idx] - Fr, axis=1) / np.linalg.norm(Fr, axis=1))
    assert 0.0 < dF < min(t1["dF"])
