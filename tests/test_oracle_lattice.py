"""Pins of the periodic r^-6 sums the oracle uses for the coarsest grid and for
the exact reference: Ewald against plain image summation, independence of the
screening parameter, and forces against finite differences."""
import numpy as np
import pytest

from oracle import exact, lattice


def test_simple_cubic_lattice_constant_by_brute_force():
    # sum over the nonzero points of Z^3 of |n|^-6, summed directly to R=40
    # with the continuum tail: agrees with the Ewald value to ~1e-8
    ew = lattice.lattice_r6_sum([[0.0, 0.0, 0.0]], np.ones(3))[0]
    direct = lattice.direct_r6_sum([[0.0, 0.0, 0.0]], np.ones(3), 40.0)[0]
    assert ew == pytest.approx(direct, rel=1e-8)
    assert ew == pytest.approx(8.40192397, rel=1e-8)


def test_ewald_is_independent_of_screening():
    box = np.array([1.0, 1.3, 0.8])
    v = np.array([[0.0, 0.0, 0.0], [0.3, 0.1, 0.45], [0.5, 0.65, 0.4], [0.99, 0.01, 0.2]])
    ref = lattice.lattice_r6_sum(v, box, beta=3.0)
    for beta in (1.5, 4.0, 6.0):
        np.testing.assert_allclose(lattice.lattice_r6_sum(v, box, beta=beta), ref, rtol=1e-12)


def test_ewald_matches_image_sum_off_lattice():
    box = np.array([1.0, 1.3, 0.8])
    v = np.array([[0.3, 0.1, 0.45], [0.5, 0.65, 0.4]])
    np.testing.assert_allclose(lattice.lattice_r6_sum(v, box),
                               lattice.direct_r6_sum(v, box, 30.0), rtol=2e-8)


def _tiny(seed, n=10, box=(3.0, 3.5, 4.0)):
    rng = np.random.default_rng(seed)
    box = np.asarray(box)
    pos = rng.random((n, 3)) * box
    return pos, rng.uniform(1.0, 9.0, n), box


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_ewald_matches_direct(seed):
    pos, c6, box = _tiny(seed)
    E1, F1, u1 = exact.exact_ewald(pos, c6, box)
    E2, F2, u2 = exact.exact_direct(pos, c6, box, R=22.0)
    assert E1 == pytest.approx(E2, rel=1e-9)
    np.testing.assert_allclose(F1, F2, atol=1e-9 * np.abs(F1).max())


def test_exact_forces_are_energy_gradient():
    pos, c6, box = _tiny(3, n=6)
    E, F, _ = exact.exact_ewald(pos, c6, box)
    eps = 1e-5
    for i in (0, 4):
        for d in range(3):
            p = pos.copy()
            p[i, d] += eps
            Ep = exact.exact_ewald(p, c6, box)[0]
            p[i, d] -= 2 * eps
            Em = exact.exact_ewald(p, c6, box)[0]
            assert -(Ep - Em) / (2 * eps) == pytest.approx(F[i, d], rel=1e-6, abs=1e-8)


def test_two_atoms_in_a_huge_box_is_pair_energy():
    # far from every image the energy is the bare pair term -C6/r^6
    box = np.array([200.0, 200.0, 200.0])
    pos = np.array([[10.0, 10.0, 10.0], [11.2, 10.0, 10.0]])
    c6 = np.array([4.0, 4.0])
    E, F, _ = exact.exact_ewald(pos, c6, box)
    assert E == pytest.approx(-4.0 / 1.2 ** 6, rel=1e-6)
    assert F[0, 0] == pytest.approx(6 * 4.0 / 1.2 ** 7, rel=1e-6)
