"""The MD oracle (oracle/md.py): the repulsive term of eq:disp-pair-pot against
the closed form of one pair and its images, Newton's third law and the
energy gradient; velocity Verlet against its invariants: time reversibility
(run forward, flip the velocities, run back: the start is recovered to
rounding) and energy conservation with second-order drift in dt."""
import numpy as np
import pytest

from oracle import md as MD
from paper_1308_4005_amd import workloads as W


def test_one_pair_closed_form():
    box = np.array([20.0, 20.0, 20.0])
    pos = np.array([[1.0, 2.0, 3.0], [2.1, 2.4, 2.7]])
    c12 = np.array([4.0, 9.0])
    E, F = MD.repulsion(pos, c12, box, 3.0)
    d = pos[0] - pos[1]
    r2 = d @ d
    C = np.sqrt(4.0 * 9.0)
    assert E == pytest.approx(C * r2 ** -6, rel=1e-14)
    np.testing.assert_allclose(F[0], 12.0 * C * r2 ** -7 * d, rtol=1e-13)
    np.testing.assert_allclose(F[1], -F[0], rtol=1e-13)


def test_images_in_a_narrow_box():
    # box 2.5 wide in x, cutoff 3: an atom sees its own images at +-2.5 and the
    # other atom's images; compare with the explicit image list
    box = np.array([2.5, 9.0, 9.0])
    pos = np.array([[0.3, 4.0, 4.0], [1.4, 4.5, 4.2]])
    c12 = np.array([1.0, 2.0])
    E, F = MD.repulsion(pos, c12, box, 3.0)
    Eref = 0.0
    for i in range(2):
        for j in range(2):
            for k in range(-3, 4):
                if i == j and k == 0:
                    continue
                d = pos[i] - pos[j] - np.array([k * 2.5, 0, 0])
                r = np.sqrt(d @ d)
                if r < 3.0:
                    Eref += 0.5 * np.sqrt(c12[i] * c12[j]) * r ** -12
    assert E == pytest.approx(Eref, rel=1e-13)
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-12 * np.abs(F).max())


def test_repulsion_forces_are_the_gradient():
    w = W.cube(60, 0.8, seed=2)
    c12 = np.where(np.arange(w.n) % 2 == 0, 4.0, 1.0)
    E, F = MD.repulsion(w.pos, c12, w.box, 2.5)
    eps = 1e-6
    for i in (0, 17):
        for d in range(3):
            p = w.pos.copy()
            p[i, d] += eps
            Ep, _ = MD.repulsion(p, c12, w.box, 2.5)
            p[i, d] -= 2 * eps
            Em, _ = MD.repulsion(p, c12, w.box, 2.5)
            assert -(Ep - Em) / (2 * eps) == pytest.approx(F[i, d], rel=1e-5, abs=1e-6 * np.abs(F).max())


@pytest.fixture(scope="module")
def system():
    w = W.cube(120, 0.5, seed=8)
    rng = np.random.default_rng(4)
    vel = rng.normal(scale=0.3, size=(w.n, 3))
    c12 = np.full(w.n, 4.0)
    inv_m = np.full(w.n, 1.0)
    return w, vel, c12, inv_m


def test_velocity_verlet_is_time_reversible(system):
    w, vel, c12, inv_m = system
    prm = (w.box, 2.5, 0.9, 4, 2)
    x1, v1, _, _, _ = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 8)
    x0, v0, _, _, _ = MD.md_run(x1, -v1, w.c6, c12, inv_m, *prm, 0.002, 8)
    np.testing.assert_allclose(x0, w.pos, rtol=0, atol=1e-11 * np.abs(w.pos).max())
    np.testing.assert_allclose(-v0, vel, rtol=0, atol=1e-9 * np.abs(vel).max())


def test_energy_drift_is_second_order(system):
    w, vel, c12, inv_m = system
    prm = (w.box, 2.5, 0.9, 4, 2)
    drift = []
    for dt in (0.004, 0.002):
        _, _, _, ep, ek = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *prm, dt, int(round(0.04 / dt)))
        tot = ep + ek
        drift.append(np.max(np.abs(tot - tot[0])))
    assert drift[1] < drift[0]
    # halving dt divides the energy error by about four (velocity Verlet is second order)
    assert 2.5 < drift[0] / drift[1] < 6.0


def test_targets_match_the_full_sum():
    w = W.cube(90, 0.8, seed=5)
    c12 = np.linspace(1.0, 5.0, w.n)
    E, F = MD.repulsion(w.pos, c12, w.box, 2.5)
    t = np.array([3, 40, 7, 88])
    Et, Ft = MD.repulsion(w.pos, c12, w.box, 2.5, targets=t)
    np.testing.assert_allclose(Ft, F[t], rtol=1e-13, atol=1e-13 * np.abs(F).max())
    Ea, _ = MD.repulsion(w.pos, c12, w.box, 2.5, targets=np.arange(w.n))
    assert Ea == pytest.approx(E, rel=1e-13)
    # the per-atom halves of all atoms add up to the total; a subset stays below it
    assert 0 < Et < E


def test_shifting_atoms_by_box_vectors_changes_nothing():
    # positions outside the box (an MD trajectory is not wrapped) give the
    # energy and forces of the wrapped ones
    w = W.cube(80, 0.8, seed=6)
    c12 = np.full(w.n, 4.0)
    rng = np.random.default_rng(1)
    shifted = w.pos + rng.integers(-2, 3, size=(w.n, 3)) * w.box
    E, F = MD.repulsion(w.pos, c12, w.box, 2.5)
    Es, Fs = MD.repulsion(shifted, c12, w.box, 2.5)
    assert Es == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(Fs, F, rtol=0, atol=1e-10 * np.abs(F).max())


def test_mts_with_one_inner_step_is_velocity_verlet(system):
    w, vel, c12, inv_m = system
    prm = (w.box, 2.5, 0.9, 4, 2)
    x1, v1, F1, ep1, ek1 = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 4)
    x2, v2, F2, ep2, ek2 = MD.md_run_mts(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 4, 1)
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-13 * np.abs(x1).max())
    np.testing.assert_allclose(v2, v1, rtol=0, atol=1e-12 * np.abs(v1).max())
    np.testing.assert_allclose(F2, F1, rtol=0, atol=1e-12 * np.abs(F1).max())
    np.testing.assert_allclose(ep2, ep1, rtol=1e-12)
    np.testing.assert_allclose(ek2, ek1, rtol=1e-12)


def test_split_adds_up_and_the_slow_part_is_smooth(system):
    w, vel, c12, inv_m = system
    Ef, Ff, Es, Fs = MD.split_forces(w.pos, w.c6, c12, w.box, 2.5, 0.9, 4, 2)
    E, F = MD.forces(w.pos, w.c6, c12, w.box, 2.5, 0.9, 4, 2)
    assert Ef + Es == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(Ff + Fs, F, rtol=0, atol=1e-11 * np.abs(F).max())
    # the grid part is the smooth remainder: far weaker than the local part
    assert np.abs(Fs).max() < 0.1 * np.abs(Ff).max()


def test_mts_is_time_reversible(system):
    w, vel, c12, inv_m = system
    prm = (w.box, 2.5, 0.9, 4, 2)
    x1, v1, _, _, _ = MD.md_run_mts(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 6, 3)
    x0, v0, _, _, _ = MD.md_run_mts(x1, -v1, w.c6, c12, inv_m, *prm, 0.002, 6, 3)
    np.testing.assert_allclose(x0, w.pos, rtol=0, atol=1e-11 * np.abs(w.pos).max())
    np.testing.assert_allclose(-v0, vel, rtol=0, atol=1e-9 * np.abs(vel).max())


def test_mts_conserves_energy_like_verlet(system):
    # the slow force is smooth, so an outer step of 4 dt keeps the energy about
    # as well as velocity Verlet at dt
    w, vel, c12, inv_m = system
    prm = (w.box, 2.5, 0.9, 4, 2)
    _, _, _, ep, ek = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 16)
    tot = ep + ek
    d_vv = np.max(np.abs(tot - tot[0]))
    _, _, _, ep, ek = MD.md_run_mts(w.pos, vel, w.c6, c12, inv_m, *prm, 0.002, 16, 4)
    tot = ep + ek
    d_mts = np.max(np.abs(tot - tot[0]))
    assert d_mts < 3.0 * d_vv


# ---------------------------------------------------------------- multiple time steps per level

PRM3 = lambda w: (w.box, 2.5, 0.9, 4, 3)   # three grid levels: level 1 and levels 2..3 both present


def test_level_split_adds_up_and_is_the_grid_energy_by_level(system):
    from oracle import mls as M
    w, vel, c12, inv_m = system
    Ef, Ff, Em, Fm, Es, Fs = MD.split_forces_levels(w.pos, w.c6, c12, *PRM3(w))
    E, F = MD.forces(w.pos, w.c6, c12, *PRM3(w))
    assert Ef + Em + Es == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(Ff + Fm + Fs, F, rtol=0, atol=1e-11 * np.abs(F).max())
    # mid + slow is the two-scale split's slow part
    Ef2, Ff2, Es2, Fs2 = MD.split_forces(w.pos, w.c6, c12, *PRM3(w))
    assert Em + Es == pytest.approx(Es2, rel=1e-11)
    np.testing.assert_allclose(Fm + Fs, Fs2, rtol=0, atol=1e-11 * np.abs(Fs2).max())
    # independent of the atom-side interpolation: interpolation is the
    # transpose of anterpolation, so the mid energy is -1/2 <q^1, e^1> and the
    # slow energy -1/2 sum_{k>=2} <q^k, e^k> plus the self term
    r = M.mls(w.pos, w.c6, *PRM3(w))
    qe = [float(np.sum(q * e)) for q, e in zip(r["q"], r["e"])]
    xi = np.sqrt(w.c6)
    cself = M.gamma(np.zeros(1))[0] / 2.5 ** 6
    assert Em == pytest.approx(-0.5 * qe[0], rel=1e-11)
    assert Es == pytest.approx(-0.5 * sum(qe[1:]) + 0.5 * cself * float(xi @ xi), rel=1e-11)
    # ordered by smoothness: each class is far weaker than the faster one
    assert np.abs(Fs).max() < 0.1 * np.abs(Fm).max()
    assert np.abs(Fm).max() < 0.1 * np.abs(Ff).max()


def test_level_split_with_one_level_has_no_mid_class():
    w = W.cube(60, 0.5, seed=9)
    c12 = np.full(w.n, 4.0)
    Ef, Ff, Em, Fm, Es, Fs = MD.split_forces_levels(w.pos, w.c6, c12, w.box, 2.0, 0.8, 4, 1)
    assert Em == 0.0 and not np.any(Fm)
    Ef2, Ff2, Es2, Fs2 = MD.split_forces(w.pos, w.c6, c12, w.box, 2.0, 0.8, 4, 1)
    assert Es == pytest.approx(Es2, rel=1e-12)
    np.testing.assert_allclose(Fs, Fs2, rtol=0, atol=1e-12 * np.abs(Fs2).max())


def test_levels_mts_reduces_to_verlet_and_to_two_scales(system):
    w, vel, c12, inv_m = system
    a = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 2)
    b = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 2, 1, 1)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-12 * np.abs(x).max())
    # with k_slow = 1 the mid and slow kicks fall on the same instants: the
    # two-scale scheme with the whole grid part every k_mid steps
    a = MD.md_run_mts(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 4, 2)
    b = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 4, 2, 1)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-11 * np.abs(x).max())


def test_levels_mts_is_time_reversible(system):
    w, vel, c12, inv_m = system
    x1, v1, _, _, _ = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 8, 2, 2)
    x0, v0, _, _, _ = MD.md_run_mts_levels(x1, -v1, w.c6, c12, inv_m, *PRM3(w), 0.002, 8, 2, 2)
    np.testing.assert_allclose(x0, w.pos, rtol=0, atol=1e-11 * np.abs(w.pos).max())
    np.testing.assert_allclose(-v0, vel, rtol=0, atol=1e-9 * np.abs(vel).max())


def test_levels_mts_conserves_energy_like_verlet(system):
    # level 1 every 2 steps and levels 2..3 every 4: the energy stays about as
    # well conserved as velocity Verlet at dt
    w, vel, c12, inv_m = system
    _, _, _, ep, ek = MD.md_run(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 16)
    d_vv = np.max(np.abs((ep + ek) - (ep[0] + ek[0])))
    _, _, _, ep, ek = MD.md_run_mts_levels(w.pos, vel, w.c6, c12, inv_m, *PRM3(w), 0.002, 16, 2, 2)
    d_lv = np.max(np.abs((ep + ek) - (ep[0] + ek[0])))
    assert d_lv < 3.0 * d_vv
