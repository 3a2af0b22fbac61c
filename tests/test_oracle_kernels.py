"""Pins of the oracle's closed-form pieces: gamma, g_k, Phi, restriction weights.

Each check ties a function to something other than its own formula: the
stated smoothness and cutoff properties (Sec. II.A.3-4), a Taylor-series
origin of gamma, textbook interpolation kernels, polynomial reproduction, and
finite differences.
"""
import numpy as np
import pytest

from oracle import mls as M


# ---------------------------------------------------------------- gamma
def test_gamma_matches_r6_at_the_cutoff_to_second_order():
    # eq:gamma: C2 join with rho^-6 at rho = 1 (values 1, -6, 42)
    assert M.gamma(np.array([1.0]))[0] == 1.0
    assert M.dgamma(np.array([1.0 - 1e-15]))[0] == pytest.approx(-6.0, rel=1e-12)
    assert M.dgamma(np.array([1.0 + 1e-15]))[0] == pytest.approx(-6.0, rel=1e-12)
    eps = 1e-7
    d2_in = (M.dgamma(np.array([1.0 - eps]))[0] - M.dgamma(np.array([1.0 - 2 * eps]))[0]) / eps
    d2_out = (M.dgamma(np.array([1.0 + 2 * eps]))[0] - M.dgamma(np.array([1.0 + eps]))[0]) / eps
    assert d2_in == pytest.approx(42.0, rel=1e-4)
    assert d2_out == pytest.approx(42.0, rel=1e-4)
    # third derivative jumps (exactly C2)
    t = 1e-3
    def d3(x):
        return (M.dgamma(np.array([x + t]))[0] - 2 * M.dgamma(np.array([x]))[0]
                + M.dgamma(np.array([x - t]))[0]) / t ** 2
    assert abs(d3(1.0 - 0.01) - d3(1.0 + 0.01)) > 100.0


def test_gamma_is_second_order_taylor_of_inverse_sqrt():
    # gamma(rho) = 1 - u/2 + 3u^2/8 with u = rho^12 - 1: the series of
    # (1+u)^(-1/2) to second order, the electrostatic-style smoothing the
    # paper adopts (Sec. II.A.3)
    rho = np.linspace(0.0, 0.999, 57)
    u = rho ** 12 - 1.0
    series = 1.0 - 0.5 * u + 0.375 * u * u
    np.testing.assert_allclose(M.gamma(rho), series, rtol=1e-14, atol=1e-15)
    assert M.gamma(np.array([0.0]))[0] == 15.0 / 8.0


def test_dgamma_is_derivative():
    rho = np.linspace(0.05, 1.9, 101)
    rho = rho[np.abs(rho - 1.0) > 1e-3]
    eps = 1e-6
    fd = (M.gamma(rho + eps) - M.gamma(rho - eps)) / (2 * eps)
    np.testing.assert_allclose(M.dgamma(rho), fd, rtol=1e-7, atol=1e-8)


# ---------------------------------------------------------------- g_k
@pytest.mark.parametrize("l", [1, 2, 3, 5])
def test_kernel_pieces_telescope_to_r6(l):
    a = 2.7
    r = np.concatenate([np.linspace(0.3, 2 ** l * a * 1.5, 400), [a, 2 * a, 4 * a]])
    total = M.g0(r, a) + sum(M.gk(r, a, k) for k in range(1, l)) + M.g_last(r, a, l)
    np.testing.assert_allclose(total, r ** -6.0, rtol=1e-12)


def test_kernel_cutoffs():
    a = 3.0
    r = np.linspace(a, 40.0, 500)
    assert np.all(M.g0(r, a) == 0.0)
    for k in range(1, 5):
        rk = np.linspace(2 ** k * a, 200.0, 300)
        assert np.all(np.abs(M.gk(rk, a, k)) < 1e-30)
    # g_0 vanishes to third order at a: g0, g0', g0'' all zero
    eps = 1e-3
    g1, g2 = M.g0(np.array([a - eps, a - 2 * eps]), a)
    assert g2 / g1 == pytest.approx(8.0, rel=2e-2)
    d1, d2 = M.dg0(np.array([a - eps, a - 2 * eps]), a)
    assert d2 / d1 == pytest.approx(4.0, rel=2e-2)


def test_same_gamma_arguments_on_every_level():
    # Sec. II.A.4: with spacing and cutoff doubling per level the kernels are
    # the same function up to 2^(-6(k-1)):  g_k(2^(k-1) s) = 2^(-6(k-1)) g_1(s)
    a = 2.5
    s = np.linspace(0.0, 2 * a * 1.2, 300)
    for k in range(2, 6):
        np.testing.assert_allclose(M.gk(2 ** (k - 1) * s, a, k),
                                   2.0 ** (-6 * (k - 1)) * M.gk(s, a, 1), rtol=1e-13, atol=1e-300)


def test_dg0_is_derivative():
    a = 3.0
    r = np.linspace(0.7, 3.5, 200)
    eps = 1e-6
    fd = (M.g0(r + eps, a) - M.g0(r - eps, a)) / (2 * eps)
    np.testing.assert_allclose(M.dg0(r, a), fd, rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------- Phi
def test_cubic_phi_is_catmull_rom():
    # eq:Phi-Hermite equals Keys' cubic convolution kernel with a = -1/2
    t = np.linspace(-2.5, 2.5, 1001)
    x = np.abs(t)
    A = -0.5
    keys = np.where(x <= 1, (A + 2) * x ** 3 - (A + 3) * x ** 2 + 1,
                    np.where(x < 2, A * x ** 3 - 5 * A * x ** 2 + 8 * A * x - 4 * A, 0.0))
    np.testing.assert_allclose(M.phi(t, 4), keys, atol=1e-15)


@pytest.mark.parametrize("order,deg_ok", [(4, 2), (6, 4)])
def test_phi_interpolates_and_reproduces_polynomials(order, deg_ok):
    half = order // 2
    ints = np.arange(-half - 1, half + 2).astype(float)
    vals = M.phi(ints, order)
    np.testing.assert_array_equal(vals, (ints == 0).astype(float))
    t = np.linspace(-0.5, 0.5, 41)
    m = np.arange(-10, 11)
    W = M.phi(t[:, None] - m[None, :], order)
    for q in range(deg_ok + 1):
        np.testing.assert_allclose(W @ (m.astype(float) ** q), t ** q, atol=1e-12)
    # and fails one degree higher
    q = deg_ok + 1
    assert np.max(np.abs(W @ (m.astype(float) ** q) - t ** q)) > 1e-4


@pytest.mark.parametrize("order", [4, 6])
def test_phi_is_c1(order):
    for knot in range(1, order // 2 + 1):
        eps = 1e-9
        left = M.phi(np.array([knot - eps]), order)[0]
        right = M.phi(np.array([knot + eps]), order)[0]
        assert abs(left - right) < 1e-7
        dl = M.dphi(np.array([knot - 1e-12]), order)[0]
        dr = M.dphi(np.array([knot + 1e-12]), order)[0]
        assert abs(dl - dr) < 1e-9
    if order == 4:
        assert M.dphi(np.array([1.0]), 4)[0] == pytest.approx(-0.5)


@pytest.mark.parametrize("order", [4, 6])
def test_dphi_is_derivative(order):
    t = np.linspace(-3.2, 3.2, 333)
    eps = 1e-6
    fd = (M.phi(t + eps, order) - M.phi(t - eps, order)) / (2 * eps)
    np.testing.assert_allclose(M.dphi(t, order), fd, atol=1e-7)


def test_restriction_weights_are_lagrange_midpoint_rules():
    # grid k nodes sit on every second node of grid k-1; Phi(o/2) at odd o are
    # the textbook 4-point (cubic) and 6-point (quintic) midpoint weights
    o, c = M.restriction_weights(4)
    np.testing.assert_array_equal(o, np.arange(-3, 4))
    np.testing.assert_allclose(c, [-1 / 16, 0, 9 / 16, 1, 9 / 16, 0, -1 / 16], atol=1e-16)
    o, c = M.restriction_weights(6)
    np.testing.assert_allclose(c, [3 / 256, 0, -25 / 256, 0, 75 / 128, 1, 75 / 128, 0,
                                   -25 / 256, 0, 3 / 256], atol=1e-16)
    # Lagrange midpoint weights from scratch
    for p in (4, 6):
        nodes = np.arange(p) - (p - 1) / 2.0
        lw = [np.prod([(0 - nodes[m]) / (nodes[j] - nodes[m]) for m in range(p) if m != j])
              for j in range(p)]
        o, c = M.restriction_weights(p)
        odd = c[(np.abs(o) % 2) == 1]
        np.testing.assert_allclose(odd, lw, atol=1e-15)
