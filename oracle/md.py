"""Molecular dynamics around MLS dispersion (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it shares nothing with the GPU library.

The pair potential is eq:disp-pair-pot, V_ij = C^rep_ij r^-12 - C^disp_ij r^-6
(Sec. II.D).  The dispersion part is the MLS evaluation of ``oracle.mls``
(geometric mixing, C^disp_ij = sqrt(C6_i C6_j)).  The repulsive part, which
the paper leaves out of the MLS analysis because it is negligible beyond
sigma, is a plain cutoff sum over every periodic image closer than a
repulsion cutoff r_c (by default the MLS cutoff a), with geometric mixing
C^rep_ij = sqrt(C12_i C12_j).  The paper's
MD runs (Sec. III.A) do not name their integrator; velocity Verlet is used
here (a reading).
"""
from __future__ import annotations

import numpy as np

from . import mls as M

__all__ = ["repulsion", "forces", "md_run", "split_forces", "md_run_mts", "split_forces_levels",
           "md_run_mts_levels"]


def repulsion(pos, c12, box, rc, targets=None):
    """E_rep = 1/2 sum_i sum'_{(j,n), r < rc} sqrt(C12_i C12_j) r^-12 and
    F_rep = -grad E_rep, over all images (brute force: small systems).  With
    ``targets`` (atom indices) only those atoms' terms: E is 1/2 their
    per-atom sums and F their forces, in the order given."""
    box = np.asarray(box, dtype=np.float64)
    # the sum is periodic in every coordinate: wrap first, so that differences
    # lie in (-L, L) and images |n_d| <= ceil(rc / L_d) cover every r < rc
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    x12 = np.sqrt(np.asarray(c12, dtype=np.float64))
    tidx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    E = 0.0
    F = np.zeros((len(tidx), 3))
    nr = np.ceil(rc / box).astype(int)
    for ix in range(-nr[0], nr[0] + 1):
        for iy in range(-nr[1], nr[1] + 1):
            for iz in range(-nr[2], nr[2] + 1):
                d = pos[tidx, None, :] - pos[None, :, :] - np.array([ix, iy, iz]) * box
                r2 = np.sum(d * d, axis=2)
                if ix == 0 and iy == 0 and iz == 0:
                    r2[np.arange(len(tidx)), tidx] = np.inf
                ti, j = np.nonzero(r2 < rc * rc)
                r2p = r2[ti, j]
                C = x12[tidx][ti] * x12[j]
                E += 0.5 * np.sum(C * r2p ** -6)
                # -d/dx_i of C r^-12 = 12 C r^-14 (x_i - x_j)
                np.add.at(F, ti, (12.0 * C * r2p ** -7)[:, None] * d[ti, j])
    return E, F


def forces(pos, c6, c12, box, a, h, order, levels, continuity=2, rc=None):
    """Potential energy and forces of eq:disp-pair-pot: MLS dispersion plus the
    cutoff repulsion (c12 None: dispersion only; rc None: rc = a)."""
    r = M.mls(pos, c6, box, a, h, order, levels, continuity=continuity)
    E, F = r["energy"], r["F"]
    if c12 is not None:
        Er, Fr = repulsion(pos, c12, box, a if rc is None else rc)
        E, F = E + Er, F + Fr
    return E, F


def md_run(pos, vel, c6, c12, inv_mass, box, a, h, order, levels, dt, nsteps, continuity=2, rc=None):
    """Velocity Verlet: v += dt/2 F/m; x += dt v; F = F(x); v += dt/2 F/m.

    Returns the final positions and velocities, the forces at the final
    positions, and the potential and kinetic energies after each of the
    nsteps + 1 force evaluations (E_kin = 1/2 sum_i |v_i|^2 / inv_mass_i)."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    im = np.asarray(inv_mass, dtype=np.float64)[:, None]

    def ekin(v_):
        return 0.5 * float(np.sum(np.sum(v_ * v_, axis=1) / im[:, 0]))

    E, F = forces(x, c6, c12, box, a, h, order, levels, continuity, rc)
    epot, kin = [E], [ekin(v)]
    for _ in range(nsteps):
        v = v + 0.5 * dt * F * im
        x = x + dt * v
        E, F = forces(x, c6, c12, box, a, h, order, levels, continuity, rc)
        v = v + 0.5 * dt * F * im
        epot.append(E)
        kin.append(ekin(v))
    return x, v, F, np.array(epot), np.array(kin)


def split_forces(pos, c6, c12, box, a, h, order, levels, continuity=2, rc=None):
    """The fast/slow split of multiple time stepping: fast = the local part of
    eq:evaluation (k = 0: energy -1/2 sum_i xi_i e0_i and its forces) plus the
    repulsion; slow = the rest of the MLS result (the grid part, levels 1..l,
    with the self-energy correction).  Returns (E_fast, F_fast, E_slow, F_slow)."""
    r = M.mls(pos, c6, box, a, h, order, levels, continuity=continuity)
    xi = np.sqrt(np.asarray(c6, dtype=np.float64))
    E_loc = -0.5 * float(np.dot(xi, r["e0"]))
    E_fast, F_fast = E_loc, np.array(r["Floc"], dtype=np.float64)
    E_slow, F_slow = r["energy"] - E_loc, r["F"] - F_fast
    Er, Fr = repulsion(pos, c12, box, a if rc is None else rc)
    return E_fast + Er, F_fast + Fr, E_slow, F_slow


def md_run_mts(pos, vel, c6, c12, inv_mass, box, a, h, order, levels, dt, nsteps, k_slow, continuity=2, rc=None):
    """Multiple time stepping (r-RESPA) with the split of ``split_forces``: per
    outer step of k_slow dt,
        v += (k_slow dt/2) F_slow/m
        k_slow times: v += dt/2 F_fast/m; x += dt v; F_fast(x); v += dt/2 F_fast/m
        F_slow(x); v += (k_slow dt/2) F_slow/m.
    nsteps (inner steps) is a multiple of k_slow.  Returns final x, v, the
    total force F_fast + F_slow at the final positions, and E_pot, E_kin at
    the nsteps / k_slow + 1 outer-step boundaries."""
    assert nsteps % k_slow == 0
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    im = np.asarray(inv_mass, dtype=np.float64)[:, None]
    hs = 0.5 * k_slow * dt

    def ekin(v_):
        return 0.5 * float(np.sum(np.sum(v_ * v_, axis=1) / im[:, 0]))

    Ef, Ff, Es, Fs = split_forces(x, c6, c12, box, a, h, order, levels, continuity, rc)
    epot, kin = [Ef + Es], [ekin(v)]
    for _ in range(nsteps // k_slow):
        v = v + hs * Fs * im
        for _ in range(k_slow):
            v = v + 0.5 * dt * Ff * im
            x = x + dt * v
            Ef, Ff, _, _ = split_forces(x, c6, c12, box, a, h, order, levels, continuity, rc)
            v = v + 0.5 * dt * Ff * im
        _, _, Es, Fs = split_forces(x, c6, c12, box, a, h, order, levels, continuity, rc)
        v = v + hs * Fs * im
        epot.append(Ef + Es)
        kin.append(ekin(v))
    return x, v, Ff + Fs, np.array(epot), np.array(kin)


def split_forces_levels(pos, c6, c12, box, a, h, order, levels, continuity=2, rc=None):
    """The split of multiple time stepping by MLS level: fast = the local part
    (eq:evaluation with k = 0) plus the repulsion, as in ``split_forces``;
    mid = the level-1 grid part alone, the interpolation (eq:interpolation)
    of e^1 (for l >= 2; with l = 1 the only grid is the coarsest and the mid
    class is empty); slow = the rest of the MLS result, the interpolation of
    the prolongation of E^2 (levels 2..l, without e^1) with the self-energy
    term.  Interpolation is linear, so mid + slow is the whole grid part.
    Returns (E_fast, F_fast, E_mid, F_mid, E_slow, F_slow)."""
    r = M.mls(pos, c6, box, a, h, order, levels, continuity=continuity)
    xi = np.sqrt(np.asarray(c6, dtype=np.float64))
    l = r["levels"]
    E_loc = -0.5 * float(np.dot(xi, r["e0"]))
    Er, Fr = repulsion(pos, c12, box, a if rc is None else rc)
    E_fast, F_fast = E_loc + Er, np.array(r["Floc"], dtype=np.float64) + Fr
    if l >= 2:
        u1, g1 = M.interpolate(r["xw"], r["e"][0], box, r["n1"], order)
        E_mid, F_mid = -0.5 * float(np.dot(xi, u1)), xi[:, None] * g1
    else:
        E_mid, F_mid = 0.0, np.zeros_like(F_fast)
    E_slow = r["energy"] - E_loc - E_mid
    F_slow = r["F"] - np.array(r["Floc"], dtype=np.float64) - F_mid
    return E_fast, F_fast, E_mid, F_mid, E_slow, F_slow


def md_run_mts_levels(pos, vel, c6, c12, inv_mass, box, a, h, order, levels, dt, nsteps, k_mid, k_slow,
                      continuity=2, rc=None):
    """r-RESPA with three time scales on the split of ``split_forces_levels``:
    the fast force every step dt, the mid force every k_mid steps and the
    slow force every k_mid k_slow steps.  Per outer step of k_slow k_mid dt:
        v += (k_slow k_mid dt/2) F_slow/m
        k_slow times:
            v += (k_mid dt/2) F_mid/m
            k_mid times: v += dt/2 F_fast/m; x += dt v; F_fast(x); v += dt/2 F_fast/m
            F_mid(x); v += (k_mid dt/2) F_mid/m
        F_slow(x); v += (k_slow k_mid dt/2) F_slow/m.
    nsteps (inner steps) is a multiple of k_mid k_slow.  Returns the final x,
    v, the total force at the final positions, and E_pot, E_kin at the
    nsteps / (k_mid k_slow) + 1 outer-step boundaries."""
    outer = k_mid * k_slow
    assert nsteps % outer == 0
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    im = np.asarray(inv_mass, dtype=np.float64)[:, None]
    hs, hm = 0.5 * outer * dt, 0.5 * k_mid * dt

    def ekin(v_):
        return 0.5 * float(np.sum(np.sum(v_ * v_, axis=1) / im[:, 0]))

    def split(x_):
        return split_forces_levels(x_, c6, c12, box, a, h, order, levels, continuity, rc)

    Ef, Ff, Em, Fm, Es, Fs = split(x)
    epot, kin = [Ef + Em + Es], [ekin(v)]
    for _ in range(nsteps // outer):
        v = v + hs * Fs * im
        for _ in range(k_slow):
            v = v + hm * Fm * im
            for _ in range(k_mid):
                v = v + 0.5 * dt * Ff * im
                x = x + dt * v
                Ef, Ff, _, _, _, _ = split(x)
                v = v + 0.5 * dt * Ff * im
            _, _, Em, Fm, _, _ = split(x)
            v = v + hm * Fm * im
        _, _, _, _, Es, Fs = split(x)
        v = v + hs * Fs * im
        epot.append(Ef + Em + Es)
        kin.append(ekin(v))
    return x, v, Ff + Fm + Fs, np.array(epot), np.array(kin)
