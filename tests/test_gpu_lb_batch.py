"""Batched Lorentz-Berthelot form (mls_batch_evaluate_lb, Sec. II.D): every
box of a batch gives what a single Lorentz-Berthelot plan gives for that box
(same kernels and summation order: 1e-12 in FP64), the boxes match the FP64 oracle
(1e-10; mixed precision within its bound), graph replays equal eager launches
and an autotuned launch shape gives the default shape's result."""
import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import force_errors, rel_err, say

pytestmark = pytest.mark.gpu

A, H, P = 3.0, 1.0, 4
MIXED_RMS_BOUND = 1e-5
MIXED_E_BOUND = 1e-6


def _boxes(seed=31, nbox=6, n_hi=700):
    """Uneven boxes of the batched workload's recipe (small enough for the
    oracle), a box narrower than 2a, a one-level box and an empty box; two
    species each in eps and sigma."""
    ws = W.batch_boxes(nbox, seed=seed, n_lo=60, n_hi=n_hi)
    ws.append(W.fill_box(120, (5.3, 5.3, 9.0), seed=5))
    one = W.cube_box(200, 7.7, seed=6)
    one.params = dict(levels=1)
    ws.append(one)
    ws.append(W.Workload("empty", np.zeros((0, 3)), np.zeros(0), np.array([6.0, 6.0, 6.0]), dict(levels=0)))
    rng = np.random.default_rng(seed)
    for w in ws:
        w.eps = np.where(rng.uniform(size=w.n) < 0.5, 1.0, 0.6)
        w.sig = np.where(rng.uniform(size=w.n) < 0.5, 1.0, 1.25)
        w.pos = w.pos + rng.integers(-2, 3, size=w.pos.shape) * w.box
    return ws


def _levels(ws):
    return [int(w.params.get("levels", 0)) for w in ws]


def _batch(ws, precision):
    import torch
    from paper_1308_4005_amd import BatchPlan
    bp = BatchPlan([w.box for w in ws], [w.n for w in ws], A, H, P, _levels(ws), precision=precision,
                   mixing="lorentz-berthelot")
    t = lambda a: torch.tensor(np.concatenate(a), dtype=torch.float64, device="cuda")
    return bp, t([w.pos for w in ws]), t([w.eps for w in ws]), t([w.sig for w in ws])


def _run(bp, pos, eps, sig):
    import torch
    r = bp.evaluate_lb(pos, eps, sig)
    torch.cuda.synchronize()
    return r.energies.cpu().numpy(), r.forces.cpu().numpy()


def _single(w, precision):
    import torch
    from paper_1308_4005_amd import Plan
    plan = Plan(w.box, A, H, P, int(w.params.get("levels", 0)), precision=precision, n_max=w.n,
                mixing="lorentz-berthelot")
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    r = plan.evaluate_lb(t(w.pos.reshape(-1, 3)), t(w.eps), t(w.sig))
    torch.cuda.synchronize()
    return float(r.energy.cpu()[0]), r.forces.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_lb_equals_single_plans(precision):
    ws = _boxes()
    bp, pos, eps, sig = _batch(ws, precision)
    E, F = _run(bp, pos, eps, sig)
    off = bp.offsets
    # FP64: the same kernels and summation order.  Mixed: the batch runs the
    # FP32 level stencil on its shared tile shapes (window rounded up to 4, 6
    # or 8, tuned tile depth), which group the FP32 sums differently, so the
    # two agree to FP32 rounding of the grid part (~1e-7 of it)
    tol = 1e-12 if precision == "fp64" else 1e-7
    for b, w in enumerate(ws):
        Es, Fs = _single(w, precision)
        if w.n == 0:
            assert E[b] == 0.0
            continue
        assert E[b] == pytest.approx(Es, rel=tol), (b, w.name)
        assert rel_err(F[off[b]:off[b + 1]], Fs) < tol, (b, w.name)
    say(f"[lb batch] {precision}: {len(ws)} boxes equal single plans")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_lb_matches_oracle(precision):
    ws = _boxes()
    bp, pos, eps, sig = _batch(ws, precision)
    E, F = _run(bp, pos, eps, sig)
    off = bp.offsets
    worst = 0.0
    for b, w in enumerate(ws):
        if w.n == 0:
            continue
        ref = M.mls_lb(w.pos, w.eps, w.sig, w.box, A, H, P, int(w.params.get("levels", 0)))
        dE = abs(E[b] - ref["energy"]) / abs(ref["energy"])
        Fb = F[off[b]:off[b + 1]]
        if precision == "fp64":
            assert dE < 1e-10, (b, w.name, dE)
            err = rel_err(Fb, ref["F"])
            assert err < 1e-10, (b, w.name, err)
        else:
            assert dE < MIXED_E_BOUND, (b, w.name, dE)
            err = force_errors(Fb, ref["F"])[0]
            assert err < MIXED_RMS_BOUND, (b, w.name, err)
        worst = max(worst, err)
    say(f"[lb batch] {precision}: worst force error against the oracle {worst:.2e}")


def test_batch_lb_graph_replays_equal_eager():
    # boxes whose anterpolation takes the atomic kernel sum in a varying
    # order, hence 1e-12 rather than bit equality
    import torch
    ws = _boxes(seed=32)
    bp, pos, eps, sig = _batch(ws, "fp64")
    bp.set_graph(False)
    E0, F0 = _run(bp, pos, eps, sig)
    bp.set_graph(True)
    out = bp.evaluate_lb(pos, eps, sig)
    for rep in range(4):
        if rep:
            # eager work of the program between replays
            torch.cuda.synchronize()
            out.energies.fill_(7.0)
            out.forces.zero_()
            bp.evaluate_lb(pos, eps, sig, out=out)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.energies.cpu().numpy(), E0, rtol=1e-12, atol=0)
        assert rel_err(out.forces.cpu().numpy(), F0) < 1e-12, rep


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_lb_autotuned_shape_agrees(precision):
    # a launch shape changes no FP64 arithmetic; in mixed precision the tuned
    # stencil tile depth regroups the FP32 stencil sums (FP32 rounding)
    from paper_1308_4005_amd import BatchPlan
    ws = _boxes(seed=33)
    bp, pos, eps, sig = _batch(ws, precision)
    E0, F0 = _run(bp, pos, eps, sig)
    tuned = BatchPlan([w.box for w in ws], [w.n for w in ws], A, H, P, _levels(ws), precision=precision,
                      mixing="lorentz-berthelot", autotune=True)
    E1, F1 = _run(tuned, pos, eps, sig)
    t = tuned.tuning()
    say(f"[lb batch] {precision} tuned {t['tuned_ms']:.3f} ms, blocks {t['blocks']}, zc {t['stencil_zc']}")
    tol = 1e-12 if precision == "fp64" else 1e-7
    np.testing.assert_allclose(E1, E0, rtol=tol, atol=0)
    assert rel_err(F1, F0) < tol
