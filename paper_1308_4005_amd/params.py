"""Accuracy-targeted choice of the cutoff a and the finest spacing h (Sec. III.E).

The paper's model, for homogeneous systems with mean nearest-neighbour
distance d = (V/N)^(1/3) and a smoothing function of continuity C^n:

    accuracy   eps = C h^n d^7 / a^(n+7)                         (eq:accuracy-tolerance)
    cutoff     a = (C d^7 h^n / eps)^(1/(n+7))                   (eq:optimal-cutoff)
    cost       c = C_local (a/d)^3 N + C_grids (a/h)^3 (d/h)^3 N (eq:cost2)
    spacing    h = (C_grids / C_local (n+14)/n)^(1/6) d          (eq:optimal-spacing)

``select_parameters`` fits C_local and C_grids from the library's own stage
timings (local part, level stencils) on the caller's system, takes h from
eq:optimal-spacing, and solves eq:optimal-cutoff for a with the accuracy
constant C re-fitted from the measured force error at the current a, until the
measured error meets the target.  The force error of an evaluation is measured
against a reference evaluation with a cutoff ``ref_factor`` times larger (same
h and order), whose own error is smaller by about ref_factor^-(n+7).  Every
evaluation runs through the C ABI; this module is host-side arithmetic only.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

__all__ = ["mean_spacing", "accuracy", "optimal_cutoff", "cost", "optimal_spacing", "fit_cost_constants",
           "fit_accuracy_constant", "Selection", "select_parameters"]


def mean_spacing(box, n):
    """d = (V / N)^(1/3)."""
    return (box[0] * box[1] * box[2] / n) ** (1.0 / 3.0)


def accuracy(C, h, d, a, n):
    """eq:accuracy-tolerance."""
    return C * h ** n * d ** 7 / a ** (n + 7)


def optimal_cutoff(C, d, h, n, eps):
    """eq:optimal-cutoff."""
    return (C * d ** 7 * h ** n / eps) ** (1.0 / (n + 7))


def cost(C_local, C_grids, a, h, d, N):
    """eq:cost2."""
    return C_local * (a / d) ** 3 * N + C_grids * (a / h) ** 3 * (d / h) ** 3 * N


def optimal_spacing(C_local, C_grids, n, d):
    """eq:optimal-spacing."""
    return (C_grids / C_local * (n + 14) / n) ** (1.0 / 6.0) * d


def fit_cost_constants(t_local, t_grids, a, h, d, N):
    """C_local and C_grids from the times of the local part and of the level
    stencils measured at (a, h) (the two terms of eq:cost2)."""
    return t_local / ((a / d) ** 3 * N), t_grids / ((a / h) ** 3 * (d / h) ** 3 * N)


def fit_accuracy_constant(eps, a, h, d, n):
    """C of eq:accuracy-tolerance from an error measured at (a, h)."""
    return eps * a ** (n + 7) / (h ** n * d ** 7)


@dataclass
class Selection:
    a: float
    h: float
    levels: int
    error: float                  # measured RMS-relative force error at (a, h)
    target: float
    d: float
    C_local: float
    C_grids: float
    C: float
    history: List[dict] = field(default_factory=list)


def _rms_rel(F, Fref):
    import torch
    return float(torch.sqrt(torch.sum((F - Fref) ** 2) / torch.sum(Fref ** 2)))


def select_parameters(pos, c6, box, target, order=4, continuity=2, precision="fp64", a0=None, h0=None,
                      ref_factor=1.7, max_iter=6, rtol=0.02, timing_steps=5, device=None):
    """Choose (a, h) for a target RMS-relative force error on this system.

    pos (n,3), c6 (n,) float64 tensors on the device.  The cutoff is capped so
    that the reference cutoff stays below half the smallest box side.  Returns
    a ``Selection`` with the measured error at the chosen parameters, the
    fitted constants and the iteration history.
    """
    import torch
    from . import Plan

    n_atoms = pos.shape[0]
    d = mean_spacing(box, n_atoms)
    n = continuity
    a_max = 0.5 * min(box) / ref_factor
    a = min(a0 if a0 is not None else 2.8 * d, a_max)
    h = h0 if h0 is not None else d

    def evaluate(a_, h_):
        plan = Plan(box, a_, h_, order, 0, precision=precision, n_max=n_atoms, device=device, continuity=n)
        r = plan.evaluate(pos, c6)
        torch.cuda.synchronize()
        return plan, r

    # 1. cost constants from the stage times at the probe point
    plan, _ = evaluate(a, h)
    plan.set_timing(True)
    for _ in range(timing_steps):
        plan.evaluate(pos, c6)
    torch.cuda.synchronize()
    ms, cnt = plan.read_timing()
    plan.set_timing(False)
    t_local = ms["pair"] / cnt
    t_grids = ms["stencil"] / cnt
    C_local, C_grids = fit_cost_constants(t_local, t_grids, a, h, d, n_atoms)
    # 2. the spacing of eq:optimal-spacing (independent of the accuracy)
    h = optimal_spacing(C_local, C_grids, n, d)
    # 3. the cutoff of eq:optimal-cutoff, C re-fitted from the measured error
    history = []

    def measure(a_):
        plan_, r_ = evaluate(a_, h)
        _, rr_ = evaluate(ref_factor * a_, h)
        e_ = _rms_rel(r_.forces, rr_.forces)
        return e_, plan_.info["levels"]

    for _ in range(max_iter):
        err, levels = measure(a)
        C = fit_accuracy_constant(err, a, h, d, n)
        history.append(dict(a=a, h=h, error=err, C=C, levels=levels))
        a_new = min(optimal_cutoff(C, d, h, n, target), a_max)
        if abs(a_new - a) <= rtol * a:
            break
        a = a_new
    else:
        err, levels = measure(a)
        history.append(dict(a=a, h=h, error=err, C=C, levels=levels))
    return Selection(a=a, h=h, levels=levels, error=err, target=target, d=d, C_local=C_local, C_grids=C_grids,
                     C=C, history=history)
