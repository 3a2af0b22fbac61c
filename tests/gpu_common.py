"""Helpers shared by the GPU tests: run the library through its C ABI and the
oracle on the same seeded inputs, and compare."""
import sys

import numpy as np

from oracle import mls as M


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_eval(pos, c6, box, a, h, order, levels, precision="fp64", grid=None, n_max=None, continuity=2):
    import torch
    from paper_1308_4005_amd import Plan
    n = len(pos)
    plan = Plan(box, a, h, order, levels, grid=grid, precision=precision,
                n_max=n if n_max is None else n_max, continuity=continuity)
    tp = torch.tensor(np.ascontiguousarray(pos), dtype=torch.float64, device="cuda")
    tc = torch.tensor(np.ascontiguousarray(c6), dtype=torch.float64, device="cuda")
    res = plan.evaluate(tp, tc, forces=True, potential=True, dE_dc6=True)
    torch.cuda.synchronize()
    out = dict(energy=float(res.energy.cpu()[0]), F=res.forces.cpu().numpy(),
               u=res.potential.cpu().numpy(), dE_dc6=res.dE_dc6.cpu().numpy())
    return plan, out


def stages(plan, n):
    import torch
    l = plan.info["levels"]
    st = dict(perm=plan.copy_stage("perm", n=n).cpu().numpy(),
              cell_start=plan.copy_stage("cell_start").cpu().numpy(),
              e0=plan.copy_stage("e0", n=n).cpu().numpy(),
              Floc=plan.copy_stage("floc", n=n).cpu().numpy(),
              q=[plan.copy_stage("q", k).cpu().numpy() for k in range(1, l + 1)],
              e=[plan.copy_stage("e", k).cpu().numpy() for k in range(1, l + 1)],
              E=[plan.copy_stage("E", k).cpu().numpy() for k in range(1, l + 1)])
    torch.cuda.synchronize()
    return st


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def force_errors(F, Fref):
    """RMS-relative, the paper's mean per-atom relative error (eq:error-measure-force), max."""
    diff = np.linalg.norm(F - Fref, axis=1)
    nref = np.linalg.norm(Fref, axis=1)
    rms = float(np.sqrt(np.sum(diff ** 2) / np.sum(nref ** 2)))
    dF = float(np.mean(diff / np.maximum(nref, 1e-300)))
    mx = float(np.max(diff) / np.sqrt(np.mean(nref ** 2)))
    return rms, dF, mx
