"""Pins of the oracle's grid and level rules against the grids the paper quotes.

The rule under test (oracle.mls.resolve_grid): level-k spacing 2^(k-1) h and
n_1,d = 2^(l-1) max(1, floor(L_d / (2^(l-1) h) + 1/2)), i.e. the finest grid
rounded to the nearest multiple of 2^(l-1).  It is a reading: eq:def-phi,
taken literally, scales the level-k basis by 2^k h, which would make the
finest spacing 2h.  The paper fixes the answer independently:

* Sec. III.C: h = 0.92 sigma on the 11.01 x 11.01 x 176.16 sigma slab (three
  levels) "corresponds to" a 12 x 12 x 192 grid.
* Table I: the four spacings 2.75, 1.38, 0.69, 0.34 sigma on that slab with
  three levels are 11.01/4, /8, /16, /32, i.e. 4, 8, 16 and 32 points along
  the short sides.
* Table II: h = 0.688 sigma with l = 3, 4, 5 keeps one finest grid (11.01 /
  0.688 = 16 points along the short side, divisible by 2^4).
* Sec. III.D: the point count of level k is N_k = (2^(k-1) h)^-3 V.

Each test below also checks that a plausible misreading (the literal 2^k h
spacing, floor instead of round) fails the same pin, so the pins
discriminate.
"""
import numpy as np
import pytest

from oracle import mls

SLAB = np.array([11.01, 11.01, 176.16])


def _literal_eq_def_phi(box, h, levels):
    # eq:def-phi read literally: level-k spacing 2^k h, so the finest grid
    # has spacing 2h
    m = 2 ** (levels - 1)
    return m * np.maximum(1, np.floor(np.asarray(box) / (m * 2.0 * h) + 0.5)).astype(np.int64)


def _floor_rule(box, h, levels):
    m = 2 ** (levels - 1)
    return m * np.maximum(1, np.floor(np.asarray(box) / (m * h))).astype(np.int64)


def test_slab_h092_gives_12x12x192():
    n1, h1 = mls.resolve_grid(SLAB, 0.92, 3)
    assert n1.tolist() == [12, 12, 192]
    assert np.allclose(h1, SLAB / n1)
    # the misreadings do not reproduce the quoted grid
    assert _literal_eq_def_phi(SLAB, 0.92, 3).tolist() != [12, 12, 192]
    assert _floor_rule(SLAB, 0.92, 3).tolist() != [12, 12, 192]


@pytest.mark.parametrize("h,short", [(2.75, 4), (1.38, 8), (0.69, 16), (0.34, 32)])
def test_table1_spacings(h, short):
    n1, h1 = mls.resolve_grid(SLAB, h, 3)
    assert n1[0] == n1[1] == short
    # every effective spacing is the quoted one to its printed precision (the
    # printed h are rounded, so the long side's count is not fixed by them:
    # h = 0.34 gives 520 points of 0.3388 there, 11.01/32 = 0.344 would give 512)
    assert np.all(np.abs(h1 - h) < 0.006)


def test_table1_misreadings_fail():
    hs = [2.75, 1.38, 0.69, 0.34]
    lit = [int(_literal_eq_def_phi(SLAB, h, 3)[0]) for h in hs]
    flo = [int(_floor_rule(SLAB, h, 3)[0]) for h in hs]
    assert lit != [4, 8, 16, 32]
    assert flo != [4, 8, 16, 32]


@pytest.mark.parametrize("levels", [3, 4, 5])
def test_table2_same_finest_grid(levels):
    n1, _ = mls.resolve_grid(SLAB, 0.688, levels)
    assert n1.tolist() == [16, 16, 256]


def test_level_point_counts_sec3d():
    # N_k = (2^(k-1) h)^-3 V with h the effective spacing of each dimension
    n1, h1 = mls.resolve_grid(SLAB, 0.92, 3)
    V = float(np.prod(SLAB))
    for k in (1, 2, 3):
        nk = n1 // 2 ** (k - 1)
        assert int(np.prod(nk)) == pytest.approx(V / np.prod(2 ** (k - 1) * h1), rel=1e-12)


def test_levels_rule_configs():
    # the auto level rule: coarsest grid keeps >= p points per dimension.
    # The 1000-atom cube at h = 1 (L = 10.77) takes 2 levels and the
    # 32,000-atom slab (28.88^2 x 115.53) 4 levels, as the workload
    # definitions state
    assert mls.resolve_levels([10.77] * 3, 1.0, 4) == 2
    assert mls.resolve_levels([28.884, 28.884, 115.534], 1.0, 4) == 4


def test_levels_rule_adds_one_level_per_8x_atoms():
    # Sec. III.F: scaling the slab by 2 per side (8x the atoms at fixed
    # density) adds one level
    ls = [mls.resolve_levels(SLAB * s, 0.92, 4) for s in (0.5, 1.0, 2.0, 4.0)]
    assert np.all(np.diff(ls) == 1), ls


def test_explicit_grid_overrides_and_checks_divisibility():
    n1, h1 = mls.resolve_grid(SLAB, 0.92, 3, grid=(12, 12, 192))
    assert n1.tolist() == [12, 12, 192]
    with pytest.raises(ValueError):
        mls.resolve_grid(SLAB, 0.92, 3, grid=(10, 12, 192))
