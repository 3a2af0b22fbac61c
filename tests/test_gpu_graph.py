"""A single-plan evaluation captured into a graph (the benchmark's timing
mode) must give what eager evaluation gives: replayed several times, with
eager work and new input values between the replays, every replay is checked
against an eager evaluation of the same inputs."""
import numpy as np
import pytest

from paper_1308_4005_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_equal_eager(precision):
    import torch
    from paper_1308_4005_amd import Plan, Result
    say(f"[graph] {precision}")
    w = W.cube(6000, 0.8, seed=41)
    rng = np.random.default_rng(3)
    c6 = np.where(rng.uniform(size=w.n) < 0.5, 4.0, 9.0)
    plan = Plan(w.box, 3.0, 1.0, 4, 0, precision=precision, n_max=w.n)
    other = Plan(w.box, 2.5, 0.9, 4, 0, precision=precision, n_max=w.n)
    pos = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    tc6 = torch.tensor(c6, dtype=torch.float64, device="cuda")
    out = Result(torch.empty(1, dtype=torch.float64, device="cuda"),
                 torch.empty((w.n, 3), dtype=torch.float64, device="cuda"))
    plan.evaluate(pos, tc6, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.evaluate(pos, tc6, out=out)
    for rep in range(4):
        # new input values in the captured buffers
        p_new = w.pos + rng.normal(scale=0.02, size=w.pos.shape)
        pos.copy_(torch.tensor(p_new, dtype=torch.float64))
        g.replay()
        torch.cuda.synchronize()
        E_g = float(out.energy.cpu()[0])
        F_g = out.forces.cpu().numpy().copy()
        # eager work between the replays, on another plan and on this one
        other.evaluate(pos, tc6)
        ref = plan.evaluate(pos, tc6)
        torch.cuda.synchronize()
        E_e = float(ref.energy.cpu()[0])
        F_e = ref.forces.cpu().numpy()
        assert E_g == pytest.approx(E_e, rel=TOL[precision]), rep
        np.testing.assert_allclose(F_g, F_e, rtol=0, atol=TOL[precision] * np.abs(F_e).max())
    assert plan.status() == 0
    del g
    plan.close()
    other.close()


@pytest.mark.parametrize("mode", ["md_run", "md_run_mts"])
def test_md_graph_replays_equal_eager(mode):
    """The MD entry points captured into a graph (the benchmark's MD timing
    mode): every replay, started from reset positions and velocities, equals
    an eager call from the same state."""
    import torch
    from paper_1308_4005_amd import Plan
    say(f"[graph] {mode}")
    w = W.cube(6000, 0.8, seed=42)
    rng = np.random.default_rng(4)
    vel0 = rng.normal(scale=0.5, size=(w.n, 3))
    plan = Plan(w.box, 3.0, 1.0, 4, 0, precision="mixed", n_max=w.n)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    c6, c12, im = t(w.c6), t(np.full(w.n, 4.0)), t(np.ones(w.n))
    x, v = t(w.pos), t(vel0)
    F = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    nout = 5 if mode == "md_run" else 3
    ep = torch.empty(nout, dtype=torch.float64, device="cuda")
    ek = torch.empty(nout, dtype=torch.float64, device="cuda")

    def call(xx, vv, FF, ee, kk):
        if mode == "md_run":
            return plan.md_run(xx, vv, c6, c12, im, 0.001, 4, forces=FF, epot=ee, ekin=kk)
        return plan.md_run_mts(xx, vv, c6, c12, im, 0.001, 4, 2, forces=FF, epot=ee, ekin=kk)

    call(x, v, F, ep, ek)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call(x, v, F, ep, ek)
    for rep in range(3):
        start = w.pos + rng.normal(scale=0.01, size=w.pos.shape)
        x.copy_(t(start))
        v.copy_(t(vel0))
        g.replay()
        torch.cuda.synchronize()
        got = [a.cpu().numpy().copy() for a in (x, v, F, ep, ek)]
        xe, ve = t(start), t(vel0)
        Fe, epe, eke = call(xe, ve, None, None, None)
        torch.cuda.synchronize()
        want = [a.cpu().numpy() for a in (xe, ve, Fe, epe, eke)]
        for a, b in zip(got, want):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-9 * np.abs(b).max())
    assert plan.status() == 0
    del g
    plan.close()
