"""Parameter selection of Sec. III.E: the closed forms of eq:optimal-cutoff and
eq:optimal-spacing against the models they come from (eq:accuracy-tolerance,
eq:cost2), checked numerically; the constant fits invert the models."""
import numpy as np
import pytest

from paper_1308_4005_amd import params as S


@pytest.mark.parametrize("n", (1, 2, 3, 4))
def test_optimal_cutoff_meets_the_accuracy(n):
    C, d, h = 3.7, 1.08, 0.95
    for eps in (1e-3, 1e-5):
        a = S.optimal_cutoff(C, d, h, n, eps)
        assert S.accuracy(C, h, d, a, n) == pytest.approx(eps, rel=1e-12)


@pytest.mark.parametrize("n", (1, 2, 4))
def test_optimal_spacing_minimises_the_cost_at_fixed_accuracy(n):
    Cl, Cg, C, d, N = 2.0e-9, 7.0e-11, 5.0, 1.08, 1e6
    h_opt = S.optimal_spacing(Cl, Cg, n, d)
    for eps in (1e-3, 1e-6):       # independent of the accuracy
        hs = np.linspace(0.3 * h_opt, 3.0 * h_opt, 20001)
        c = [S.cost(Cl, Cg, S.optimal_cutoff(C, d, h, n, eps), h, d, N) for h in hs]
        assert hs[int(np.argmin(c))] == pytest.approx(h_opt, rel=2e-3)


def test_fits_invert_the_models():
    d, N, a, h, n = 1.08, 32000, 3.0, 1.0, 2
    Cl, Cg = 1.3e-9, 4.0e-11
    t_local = Cl * (a / d) ** 3 * N
    t_grids = Cg * (a / h) ** 3 * (d / h) ** 3 * N
    assert S.fit_cost_constants(t_local, t_grids, a, h, d, N) == pytest.approx((Cl, Cg), rel=1e-12)
    eps = S.accuracy(2.5, h, d, a, n)
    assert S.fit_accuracy_constant(eps, a, h, d, n) == pytest.approx(2.5, rel=1e-12)
    assert S.mean_spacing((10.0, 20.0, 40.0), 1000) == pytest.approx(2.0, rel=1e-12)
