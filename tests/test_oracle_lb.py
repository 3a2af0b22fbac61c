"""Lorentz-Berthelot mixing in the oracle (Sec. II.D): the seven charge vectors
reproduce the pair coefficient exactly, equal sigma reduces to geometric
mixing, the exact sum by Ewald agrees with a direct pair-coefficient image sum,
the local part equals brute force, atoms on coarsest-grid nodes give the exact
sum, and forces are the energy gradient."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import mls as M
from paper_1308_4005_amd import workloads as W


def _species(n, seed):
    rng = np.random.default_rng(seed)
    eps = np.where(rng.uniform(size=n) < 0.5, 1.0, 0.6)
    sig = np.where(rng.uniform(size=n) < 0.5, 1.0, 1.25)
    return eps, sig


def test_charges_reproduce_the_pair_coefficient():
    rng = np.random.default_rng(0)
    eps = rng.uniform(0.1, 2.0, 50)
    sig = rng.uniform(0.7, 1.6, 50)
    xi = M.lb_charges(eps, sig)
    C = sum(np.outer(xi[k], xi[6 - k]) for k in range(7))
    ref = 2.0 * np.sqrt(np.outer(eps, eps)) * ((sig[:, None] + sig[None, :]) / 2.0) ** 6
    np.testing.assert_allclose(C, ref, rtol=1e-14)
    # the binomial weights: xi_k xi_{6-k} for equal sigma sum to 2 eps sigma^6
    assert sum(math.comb(6, k) for k in range(7)) == 64


def test_equal_sigma_reduces_to_geometric_mixing():
    w = W.cube(150, 0.8, seed=3)
    eps, _ = _species(w.n, 1)
    s = np.full(w.n, 1.1)
    rg = M.mls(w.pos, 2.0 * eps * s ** 6, w.box, 2.5, 0.8, 4, 2)
    rl = M.mls_lb(w.pos, eps, s, w.box, 2.5, 0.8, 4, 2)
    assert rl["energy"] == pytest.approx(rg["energy"], rel=1e-13)
    np.testing.assert_allclose(rl["F"], rg["F"], rtol=0, atol=1e-12 * np.abs(rg["F"]).max())
    Eg, Fg, _ = exact.exact_ewald(w.pos, 2.0 * eps * s ** 6, w.box)
    El, Fl = exact.exact_ewald_lb(w.pos, eps, s, w.box)
    assert El == pytest.approx(Eg, rel=1e-12)
    np.testing.assert_allclose(Fl, Fg, rtol=0, atol=1e-11 * np.abs(Fg).max())


def _direct_lb(pos, eps, sig, box, R):
    """Pair-coefficient image sum to radius R plus the continuum energy tail."""
    n = len(pos)
    E = 0.0
    F = np.zeros((n, 3))
    C = 2.0 * np.sqrt(np.outer(eps, eps)) * ((sig[:, None] + sig[None, :]) / 2.0) ** 6
    nr = np.ceil(R / box).astype(int) + 1
    for nx in range(-nr[0], nr[0] + 1):
        for ny in range(-nr[1], nr[1] + 1):
            for nz in range(-nr[2], nr[2] + 1):
                d = pos[:, None, :] - pos[None, :, :] - np.array([nx, ny, nz]) * box
                r2 = np.sum(d * d, axis=2)
                if nx == 0 and ny == 0 and nz == 0:
                    np.fill_diagonal(r2, np.inf)
                m = r2 <= R * R
                r2m = np.where(m, r2, 1.0)
                E += -0.5 * np.sum(np.where(m, C * r2m ** -3, 0.0))
                F += np.einsum("ij,ijk->ik", np.where(m, C * -6.0 * r2m ** -4, 0.0), d)
    E += -0.5 * 4.0 * math.pi / (3.0 * np.prod(box) * R ** 3) * np.sum(C)
    return E, F


def test_exact_lb_sum_by_ewald_equals_direct_image_sum():
    w = W.cube(12, 0.5, seed=5)
    eps, sig = _species(w.n, 2)
    E, F = exact.exact_ewald_lb(w.pos, eps, sig, w.box)
    Ed, Fd = _direct_lb(w.pos, eps, sig, w.box, 60.0)
    assert E == pytest.approx(Ed, rel=2e-7)
    np.testing.assert_allclose(F, Fd, rtol=0, atol=1e-6 * np.abs(F).max())


def _local_bruteforce_lb(xw, eps, sig, box, a):
    n = len(xw)
    ell = np.zeros(n)
    F = np.zeros((n, 3))
    nr = np.ceil(a / box).astype(int) + 1
    for i in range(n):
        for nx in range(-nr[0], nr[0] + 1):
            for ny in range(-nr[1], nr[1] + 1):
                for nz in range(-nr[2], nr[2] + 1):
                    d = xw[i] - xw - np.array([nx, ny, nz]) * box
                    r = np.sqrt(np.sum(d * d, axis=1))
                    m = r < a
                    if nx == 0 and ny == 0 and nz == 0:
                        m[i] = False
                    C = M.lb_pair_coefficient(eps[i], eps[m], sig[i], sig[m])
                    ell[i] += np.sum(C * M.g0(r[m], a))
                    F[i] += np.sum((C * M.dg0(r[m], a) / r[m])[:, None] * d[m], axis=0)
    return ell, F


@pytest.mark.parametrize("box,n,a", [((9.0, 9.0, 9.0), 60, 2.5), ((4.0, 5.0, 9.0), 30, 3.0)])
def test_local_part_equals_bruteforce(box, n, a):
    box = np.asarray(box)
    rng = np.random.default_rng(7)
    xw = rng.uniform(0, 1, (n, 3)) * box
    eps, sig = _species(n, 3)
    ell, F = M.local_part_lb(xw, eps, sig, box, a)
    ell2, F2 = _local_bruteforce_lb(xw, eps, sig, box, a)
    np.testing.assert_allclose(ell, ell2, rtol=1e-12)
    np.testing.assert_allclose(F, F2, rtol=0, atol=1e-12 * np.abs(F2).max())


@pytest.mark.parametrize("order", (4, 6))
def test_atoms_on_coarsest_nodes_give_the_exact_lb_sum(order):
    box = np.array([8.0, 8.0, 8.0])
    l, h, a = 2, 1.0, 2.5 if order == 4 else 2.0
    n1, h1 = M.resolve_grid(box, h, l)
    pos = np.array([[0, 0, 0], [1, 2, 3], [3, 1, 1], [2, 2, 0]], dtype=float) * h1 * 2
    eps = np.array([1.0, 0.5, 0.8, 1.2])
    sig = np.array([1.0, 1.3, 0.9, 1.1])
    r = M.mls_lb(pos, eps, sig, box, a, h, order, l)
    E, F = exact.exact_ewald_lb(pos, eps, sig, box)
    assert r["energy"] == pytest.approx(E, rel=1e-12)


def test_forces_are_energy_gradient():
    w = W.cube(60, 0.8, seed=9)
    eps, sig = _species(w.n, 4)
    a, h, p, l = 2.2, 0.9, 4, 2
    r = M.mls_lb(w.pos, eps, sig, w.box, a, h, p, l)
    step = 1e-5
    for i in (2, 33):
        for d in range(3):
            pp = w.pos.copy()
            pp[i, d] += step
            Ep = M.mls_lb(pp, eps, sig, w.box, a, h, p, l)["energy"]
            pp[i, d] -= 2 * step
            Em = M.mls_lb(pp, eps, sig, w.box, a, h, p, l)["energy"]
            assert -(Ep - Em) / (2 * step) == pytest.approx(r["F"][i, d], rel=2e-6, abs=1e-7)


def test_lb_accuracy_is_that_of_the_method():
    # the seven grid instances carry the same discretisation error as one
    # geometric instance (Sec. II.D: only the cost changes)
    w = W.cube(200, 0.8, seed=3)
    eps, sig = _species(w.n, 1)
    r = M.mls_lb(w.pos, eps, sig, w.box, 2.5, 0.8, 4, 2)
    E, F = exact.exact_ewald_lb(w.pos, eps, sig, w.box)
    dF = np.mean(np.linalg.norm(r["F"] - F, axis=1) / np.linalg.norm(F, axis=1))
    rg = M.mls(w.pos, 2.0 * eps * sig ** 6, w.box, 2.5, 0.8, 4, 2)
    Eg, Fg, _ = exact.exact_ewald(w.pos, 2.0 * eps * sig ** 6, w.box)
    dFg = np.mean(np.linalg.norm(rg["F"] - Fg, axis=1) / np.linalg.norm(Fg, axis=1))
    assert abs(r["energy"] - E) / abs(E) < 1e-3
    assert dF < 3.0 * dFg
