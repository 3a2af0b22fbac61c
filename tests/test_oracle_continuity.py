"""The smoothing-function family of Sec. III.B (continuity C^1 .. C^4) in the
oracle: gamma_k is the order-k Taylor polynomial of rho^-6 = (1+u)^(-1/2) in
u = rho^12 - 1 (eq:gamma is k = 2).  Pinned against exact rational expansions
written here from the binomial series, the derivatives of rho^-6 at the join,
the telescoping of the multilevel kernels, exact sums for atoms on
coarsest-grid nodes, energy gradients, and the error trends the paper reports
for the family."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from oracle import mls as M
from paper_1308_4005_amd import workloads as W

KS = (1, 2, 3, 4)


def exact_coeffs(k):
    """gamma_k inside the unit ball as exact coefficients of rho^(12 j)."""
    b = [Fraction(1)]
    for m in range(1, k + 1):
        b.append(b[-1] * (Fraction(-1, 2) - (m - 1)) / m)
    c = [Fraction(0)] * (k + 1)
    for m, bm in enumerate(b):
        # (v - 1)^m = sum_j C(m, j) v^j (-1)^(m - j)
        binom = Fraction(1)
        for j in range(m + 1):
            c[j] += bm * binom * (-1) ** (m - j)
            binom = binom * (m - j) / (j + 1)
    return c


def falling(x, n):
    out = Fraction(1)
    for i in range(n):
        out *= x - i
    return out


def test_k2_is_eq_gamma():
    assert exact_coeffs(2) == [Fraction(15, 8), Fraction(-5, 4), Fraction(3, 8)]


@pytest.mark.parametrize("k", KS)
def test_joins_rho6_with_exactly_k_derivatives(k):
    c = exact_coeffs(k)
    for n in range(k + 2):
        poly = sum(cj * falling(12 * j, n) for j, cj in enumerate(c))   # d^n/drho^n at rho = 1
        target = falling(-6, n)                                           # d^n rho^-6 at rho = 1
        if n <= k:
            assert poly == target, (k, n)
        else:
            assert poly != target, (k, n)


@pytest.mark.parametrize("k", KS)
def test_oracle_gamma_equals_the_expansion(k):
    c = [float(x) for x in exact_coeffs(k)]
    rho = np.concatenate([np.linspace(0.0, 0.999, 41), [1.0, 1.3, 2.0]])
    with np.errstate(divide="ignore"):
        ref = np.where(rho < 1.0, sum(cj * rho ** (12 * j) for j, cj in enumerate(c)), rho ** -6.0)
    np.testing.assert_allclose(M.gamma(rho, k), ref, rtol=1e-13, atol=1e-13)
    # gamma_k(0): partial sums of the binomial series at u = -1
    assert M.gamma(np.zeros(1), k)[0] == pytest.approx(
        {1: 3 / 2, 2: 15 / 8, 3: 35 / 16, 4: 315 / 128}[k], rel=1e-15)


@pytest.mark.parametrize("k", KS)
def test_dgamma_is_the_derivative(k):
    rho = np.array([0.1, 0.5, 0.8, 0.95, 0.999, 1.2])
    eps = 1e-6
    fd = (M.gamma(rho + eps, k) - M.gamma(rho - eps, k)) / (2 * eps)
    np.testing.assert_allclose(M.dgamma(rho, k), fd, rtol=2e-6, atol=1e-7)


@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("l", (1, 2, 4))
def test_kernel_pieces_telescope(k, l):
    a = 1.7
    r = np.linspace(0.3, 2.0 ** l * a * 1.3, 200)
    total = M.g0(r, a, k) + sum(M.gk(r, a, j, k) for j in range(1, l)) + M.g_last(r, a, l, k)
    np.testing.assert_allclose(total, r ** -6.0, rtol=1e-12)


NODE_CASES = [
    ((8.0, 8.0, 8.0), 1.0, 2, 4, 2.5, [[0, 0, 0], [1, 2, 3], [3, 1, 1], [2, 2, 0]]),
    ((8.0, 8.0, 8.0), 1.0, 2, 6, 2.0, [[0, 0, 0], [1, 2, 3], [3, 1, 1]]),
    ((6.0, 8.0, 10.0), 0.5, 2, 4, 1.7, [[0, 0, 0], [2, 3, 4], [5, 7, 9]]),
]


@pytest.mark.parametrize("k", (1, 3, 4))
@pytest.mark.parametrize("case", NODE_CASES)
def test_atoms_on_coarsest_nodes_give_the_exact_sum(k, case):
    # the splitting is an identity for any gamma: with every interpolation
    # exact, MLS returns the periodic r^-6 sum
    box, h, l, order, a, nodes = case
    box = np.asarray(box)
    n1, h1 = M.resolve_grid(box, h, l)
    pos = np.asarray(nodes, dtype=float) * h1 * 2 ** (l - 1)
    c6 = np.linspace(1.0, 9.0, len(pos))
    r = M.mls(pos, c6, box, a, h, order, l, continuity=k)
    E, F, u = exact.exact_ewald(pos, c6, box)
    assert r["energy"] == pytest.approx(E, rel=1e-12)
    g0 = M.gamma(np.zeros(1), k)[0]
    np.testing.assert_allclose(r["u"] - g0 * a ** -6 * np.sqrt(c6), u, rtol=1e-11)


@pytest.mark.parametrize("k", (1, 4))
def test_forces_are_energy_gradient(k):
    w = W.cube(80, 0.8, seed=21)
    a, h, p, l = 2.2, 0.9, 4, 2
    r = M.mls(w.pos, w.c6, w.box, a, h, p, l, continuity=k)
    eps = 1e-5
    for i in (3, 41):
        for d in range(3):
            pp = w.pos.copy()
            pp[i, d] += eps
            Ep = M.mls(pp, w.c6, w.box, a, h, p, l, continuity=k)["energy"]
            pp[i, d] -= 2 * eps
            Em = M.mls(pp, w.c6, w.box, a, h, p, l, continuity=k)["energy"]
            assert -(Ep - Em) / (2 * eps) == pytest.approx(r["F"][i, d], rel=2e-6, abs=1e-7)


@pytest.fixture(scope="module")
def cube300_exact():
    w = W.cube(300, 0.8, seed=11)
    E, F, u = exact.exact_ewald(w.pos, w.c6, w.box, beta=5.0 / w.box[0])
    return w, F


def _dF(r, F):
    return np.mean(np.linalg.norm(r["F"] - F, axis=1) / np.linalg.norm(F, axis=1))


def test_continuity_trends_for_the_cubic_basis(cube300_exact):
    # Sec. III.B (Fig. 6, order 3 = the cubic Phi): as the cutoff grows the C^1
    # error decays more slowly than the others, and continuity beyond C^2 does
    # not help: the error grows slightly with k
    w, F = cube300_exact
    err = {k: [_dF(M.mls(w.pos, w.c6, w.box, a, 0.8, 4, 2, continuity=k), F) for a in (1.6, 3.0)]
           for k in KS}
    decay = {k: err[k][0] / err[k][1] for k in KS}
    assert decay[1] < min(decay[2], decay[3], decay[4])
    for a_i in range(2):
        assert err[2][a_i] < err[3][a_i] < err[4][a_i]
