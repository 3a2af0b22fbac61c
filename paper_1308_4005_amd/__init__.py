"""Multilevel summation (MLS) for periodic r^-6 dispersion on the MI355X.

Python face of the C-ABI library ``libmlsdisp.so`` (include/mlsdisp.h).  The
method is that of Tameling, Springer, Bientinesi, Ismail (arXiv 1308.4005):
one call evaluates the MLS energy, forces, per-atom potential and dE/dC6 of
a periodic box of atoms with C6 factors under geometric mixing.  PyTorch
supplies device memory and the stream; all arithmetic runs in the library's
HIP kernels.

    plan = Plan(box, cutoff=3.0, h=1.0, order=4, levels=5, n_max=N)
    res = plan.evaluate(pos, c6)            # pos (N,3), c6 (N,) float64 on cuda
    res.energy, res.forces
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

from . import _lib

__all__ = ["Plan", "Result", "MLSError", "precision_code", "MLSDispersion", "BatchPlan"]

MLSError = _lib.MLSError


def precision_code(precision) -> int:
    if precision in (0, "fp64", "f64", "double"):
        return _lib.MLS_FP64
    if precision in (1, "mixed", "fp32", "f32"):
        return _lib.MLS_MIXED
    raise ValueError(f"unknown precision {precision!r}")


def _params(box, cutoff, h, order, levels, grid, precision, continuity=2, mixing=0, skin=0.0):
    p = _lib.MLSParams()
    p.skin = float(skin)
    for d in range(3):
        p.box[d] = float(box[d])
        p.grid[d] = int(grid[d]) if grid is not None else 0
    p.cutoff = float(cutoff)
    p.h = float(h) if h is not None else 0.0
    p.order = int(order)
    p.levels = int(levels)
    p.precision = precision_code(precision)
    p.continuity = int(continuity)
    p.mixing = {"geometric": 0, "lorentz-berthelot": 1, "lb": 1}.get(mixing, mixing) if isinstance(mixing, str) \
        else int(mixing)
    return p


@dataclass
class Result:
    energy: "object"            # torch tensor (1,) float64 on the device
    forces: Optional["object"] = None
    potential: Optional["object"] = None
    dE_dc6: Optional["object"] = None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """A resolved MLS setup for one periodic box (``mls_plan_create``)."""

    def __init__(self, box, cutoff, h=1.0, order=4, levels=0, grid=None, precision="fp64",
                 n_max=0, device=None, continuity=2, mixing="geometric", skin=0.0):
        import torch
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.params = _params(box, cutoff, h, order, levels, grid, precision, continuity, mixing, skin)
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_plan_create(ctypes.byref(self.params), int(n_max),
                                                 ctypes.byref(self._plan)), "mls_plan_create")
        inf = _lib.MLSPlanInfo()
        _lib.check(self._lib.mls_plan_get_info(self._plan, ctypes.byref(inf)), "mls_plan_get_info")
        self.info = dict(levels=inf.levels, grid=tuple(inf.grid), coarsest=tuple(inf.coarsest),
                         cells=tuple(inf.cells), h_eff=tuple(inf.h_eff), taps=int(inf.taps),
                         n_max=int(inf.n_max), workspace_bytes=int(inf.workspace_bytes),
                         precision=int(inf.precision), order=int(inf.order),
                         cell_width=tuple(inf.cell_width), continuity=int(inf.continuity),
                         mixing=int(inf.mixing),
                         stencil_path=_lib.STENCIL_PATHS.get(int(inf.stencil_path), int(inf.stencil_path)))
        self.n_max = int(inf.n_max)

    # ------------------------------------------------------------------
    def _check_inputs(self, pos, c6):
        import torch
        if pos.device != self.device or c6.device != self.device:
            raise ValueError("pos and c6 must live on the plan's device")
        if pos.dtype != torch.float64 or c6.dtype != torch.float64:
            raise TypeError("pos and c6 must be float64")
        if pos.dim() != 2 or pos.shape[1] != 3 or c6.shape != (pos.shape[0],):
            raise ValueError("pos must be (n,3) and c6 (n,)")
        if not (pos.is_contiguous() and c6.is_contiguous()):
            raise ValueError("pos and c6 must be contiguous")

    def evaluate(self, pos, c6, forces=True, potential=False, dE_dc6=False, out=None, stream=None):
        """Enqueue one evaluation on the current torch stream (or ``stream``)."""
        import torch
        self._check_inputs(pos, c6)
        n = pos.shape[0]
        if out is None:
            out = Result(torch.empty(1, dtype=torch.float64, device=self.device),
                         torch.empty((n, 3), dtype=torch.float64, device=self.device) if forces else None,
                         torch.empty(n, dtype=torch.float64, device=self.device) if potential else None,
                         torch.empty(n, dtype=torch.float64, device=self.device) if dE_dc6 else None)
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_evaluate(self._plan, n, _ptr(pos), _ptr(c6), _ptr(out.energy),
                                              _ptr(out.forces), _ptr(out.potential), _ptr(out.dE_dc6),
                                              ctypes.c_void_p(s)), "mls_evaluate")
        return out

    def evaluate_lb(self, pos, eps, sigma, forces=True, out=None, stream=None):
        """Enqueue one Lorentz-Berthelot evaluation (``mls_evaluate_lb``):
        per-atom epsilon and sigma instead of C6; returns energy and forces."""
        import torch
        self._check_inputs(pos, eps)
        self._check_inputs(pos, sigma)
        n = pos.shape[0]
        if out is None:
            out = Result(torch.empty(1, dtype=torch.float64, device=self.device),
                         torch.empty((n, 3), dtype=torch.float64, device=self.device) if forces else None)
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_evaluate_lb(self._plan, n, _ptr(pos), _ptr(eps), _ptr(sigma), _ptr(out.energy),
                                                 _ptr(out.forces), ctypes.c_void_p(s)), "mls_evaluate_lb")
        return out

    def _check_vec(self, t, shape, name):
        import torch
        if t.device != self.device or t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on the plan's device")

    def evaluate_md(self, pos, c6, c12, rc=None, forces=True, out=None, stream=None):
        """Enqueue one evaluation of the full pair potential (``mls_evaluate_md``):
        MLS dispersion plus the cutoff r^-12 repulsion (rc None: the cutoff a)."""
        import torch
        self._check_inputs(pos, c6)
        n = pos.shape[0]
        self._check_vec(c12, (n,), "c12")
        rc = self.params.cutoff if rc is None else float(rc)
        if out is None:
            out = Result(torch.empty(1, dtype=torch.float64, device=self.device),
                         torch.empty((n, 3), dtype=torch.float64, device=self.device) if forces else None)
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_evaluate_md(self._plan, n, _ptr(pos), _ptr(c6), _ptr(c12), ctypes.c_double(rc),
                                                 _ptr(out.energy), _ptr(out.forces), ctypes.c_void_p(s)),
                       "mls_evaluate_md")
        return out

    def md_run(self, pos, vel, c6, c12, inv_mass, dt, nsteps, rc=None, forces=None, epot=None, ekin=None,
               stream=None):
        """Enqueue ``nsteps`` velocity-Verlet steps (``mls_md_run``); ``pos`` and
        ``vel`` advance in place.  Returns (forces, epot, ekin): forces at the
        final positions and the potential / kinetic energies after each of the
        nsteps + 1 force evaluations."""
        import torch
        self._check_inputs(pos, c6)
        n = pos.shape[0]
        self._check_vec(vel, (n, 3), "vel")
        self._check_vec(c12, (n,), "c12")
        self._check_vec(inv_mass, (n,), "inv_mass")
        rc = self.params.cutoff if rc is None else float(rc)
        nsteps = int(nsteps)
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if epot is None:
            epot = torch.empty(max(nsteps, 0) + 1, dtype=torch.float64, device=self.device)
        if ekin is None:
            ekin = torch.empty(max(nsteps, 0) + 1, dtype=torch.float64, device=self.device)
        self._check_vec(forces, (n, 3), "forces")
        self._check_vec(epot, (max(nsteps, 0) + 1,), "epot")
        self._check_vec(ekin, (max(nsteps, 0) + 1,), "ekin")
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_md_run(self._plan, n, _ptr(pos), _ptr(vel), _ptr(c6), _ptr(c12),
                                            ctypes.c_double(rc), _ptr(inv_mass), ctypes.c_double(dt), nsteps,
                                            _ptr(forces), _ptr(epot), _ptr(ekin), ctypes.c_void_p(s)),
                       "mls_md_run")
        return forces, epot, ekin

    def md_run_mts(self, pos, vel, c6, c12, inv_mass, dt, nsteps, k_slow, rc=None, forces=None, epot=None,
                   ekin=None, stream=None):
        """Enqueue ``nsteps`` inner steps of multiple time stepping
        (``mls_md_run_mts``): local part + repulsion every step, grid part
        every ``k_slow`` steps.  Returns (forces, epot, ekin) with
        nsteps // k_slow + 1 energies."""
        import torch
        self._check_inputs(pos, c6)
        n = pos.shape[0]
        self._check_vec(vel, (n, 3), "vel")
        self._check_vec(c12, (n,), "c12")
        self._check_vec(inv_mass, (n,), "inv_mass")
        rc = self.params.cutoff if rc is None else float(rc)
        nsteps, k_slow = int(nsteps), int(k_slow)
        nout = max(nsteps, 0) // max(k_slow, 1) + 1
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if epot is None:
            epot = torch.empty(nout, dtype=torch.float64, device=self.device)
        if ekin is None:
            ekin = torch.empty(nout, dtype=torch.float64, device=self.device)
        self._check_vec(forces, (n, 3), "forces")
        self._check_vec(epot, (nout,), "epot")
        self._check_vec(ekin, (nout,), "ekin")
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_md_run_mts(self._plan, n, _ptr(pos), _ptr(vel), _ptr(c6), _ptr(c12),
                                                ctypes.c_double(rc), _ptr(inv_mass), ctypes.c_double(dt), nsteps,
                                                k_slow, _ptr(forces), _ptr(epot), _ptr(ekin), ctypes.c_void_p(s)),
                       "mls_md_run_mts")
        return forces, epot, ekin

    def md_run_mts_levels(self, pos, vel, c6, c12, inv_mass, dt, nsteps, k_mid, k_slow, rc=None, forces=None,
                          epot=None, ekin=None, stream=None):
        """Enqueue ``nsteps`` inner steps of multiple time stepping per level
        (``mls_md_run_mts_levels``): local part + repulsion every step, the
        level-1 grid part every ``k_mid`` steps, levels 2..l every
        ``k_mid * k_slow`` steps.  Returns (forces, epot, ekin) with
        nsteps // (k_mid * k_slow) + 1 energies."""
        import torch
        self._check_inputs(pos, c6)
        n = pos.shape[0]
        self._check_vec(vel, (n, 3), "vel")
        self._check_vec(c12, (n,), "c12")
        self._check_vec(inv_mass, (n,), "inv_mass")
        rc = self.params.cutoff if rc is None else float(rc)
        nsteps, k_mid, k_slow = int(nsteps), int(k_mid), int(k_slow)
        nout = max(nsteps, 0) // max(k_mid * k_slow, 1) + 1
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if epot is None:
            epot = torch.empty(nout, dtype=torch.float64, device=self.device)
        if ekin is None:
            ekin = torch.empty(nout, dtype=torch.float64, device=self.device)
        self._check_vec(forces, (n, 3), "forces")
        self._check_vec(epot, (nout,), "epot")
        self._check_vec(ekin, (nout,), "ekin")
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_md_run_mts_levels(self._plan, n, _ptr(pos), _ptr(vel), _ptr(c6), _ptr(c12),
                                                       ctypes.c_double(rc), _ptr(inv_mass), ctypes.c_double(dt),
                                                       nsteps, k_mid, k_slow, _ptr(forces), _ptr(epot), _ptr(ekin),
                                                       ctypes.c_void_p(s)),
                       "mls_md_run_mts_levels")
        return forces, epot, ekin

    def copy_stage(self, what, level=1, n=None):
        """Intermediate array of the last evaluation (``mls_plan_copy_stage``)."""
        import torch
        name = what
        what = {"perm": _lib.MLS_STAGE_PERM, "cell_start": _lib.MLS_STAGE_CELL_START,
                "e0": _lib.MLS_STAGE_E0, "floc": _lib.MLS_STAGE_FLOC, "q": _lib.MLS_STAGE_Q,
                "e": _lib.MLS_STAGE_E_LEVEL, "E": _lib.MLS_STAGE_E_TOTAL}[name]
        if what == _lib.MLS_STAGE_PERM:
            t = torch.empty(n, dtype=torch.int32, device=self.device)
        elif what == _lib.MLS_STAGE_CELL_START:
            c = self.info["cells"]
            t = torch.empty(c[0] * c[1] * c[2] + 1, dtype=torch.int32, device=self.device)
        elif what == _lib.MLS_STAGE_E0:
            t = torch.empty(n, dtype=torch.float64, device=self.device)
        elif what == _lib.MLS_STAGE_FLOC:
            t = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        else:
            g = [x >> (level - 1) for x in self.info["grid"]]
            t = torch.empty((g[2], g[1], g[0]), dtype=torch.float64, device=self.device)
        s = torch.cuda.current_stream(self.device).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_plan_copy_stage(self._plan, what, int(level), _ptr(t),
                                                     t.numel() * t.element_size(), ctypes.c_void_p(s)),
                       "mls_plan_copy_stage")
        return t

    def set_timing(self, enable=True):
        """Record per-stage hipEvents in following evaluations."""
        _lib.check(self._lib.mls_plan_set_timing(self._plan, int(bool(enable))), "mls_plan_set_timing")

    def read_timing(self):
        """(dict stage -> summed ms, number of evaluations) since set_timing."""
        ms = (ctypes.c_double * len(_lib.STAGE_NAMES))()
        cnt = ctypes.c_int(0)
        _lib.check(self._lib.mls_plan_read_timing(self._plan, ms, ctypes.byref(cnt)), "mls_plan_read_timing")
        return {k: float(ms[i]) for i, k in enumerate(_lib.STAGE_NAMES)}, int(cnt.value)

    def status(self):
        """Synchronise and return the device input flags (0 = clean)."""
        flags = ctypes.c_int(0)
        st = self._lib.mls_plan_status(self._plan, ctypes.byref(flags))
        if st not in (_lib.MLS_OK, _lib.MLS_ERR_NONFINITE):
            _lib.check(st, "mls_plan_status")
        return flags.value

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            self._lib.mls_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def __getattr__(name):
    if name == "MLSDispersion":
        from .autograd import MLSDispersion
        return MLSDispersion
    if name == "BatchPlan":
        from .batch import BatchPlan
        return BatchPlan
    raise AttributeError(name)
