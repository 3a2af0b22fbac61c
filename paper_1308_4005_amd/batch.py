"""Batched MLS: many independent periodic boxes in one launch sequence.

``BatchPlan(boxes, n_per_box, cutoff, h, order, levels, precision)`` wraps
``mls_batch_create``; ``evaluate(pos, c6)`` takes the atoms of all boxes
concatenated (box b owns rows ``offsets[b]:offsets[b+1]``) and returns the
per-box energies and the concatenated forces (and dE/dC6 on request).  A
batch created with ``mixing="lorentz-berthelot"`` takes ``evaluate_lb(pos,
eps, sigma)`` instead.
Argument marshalling only: every step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

from . import _lib
from . import _params, _ptr

__all__ = ["BatchPlan", "BatchResult"]


@dataclass
class BatchResult:
    energies: "object"               # (nbox,) float64 on the device
    forces: Optional["object"] = None
    dE_dc6: Optional["object"] = None


class BatchPlan:
    def __init__(self, boxes, n_per_box, cutoff, h=1.0, order=4, levels=0, precision="fp64",
                 autotune=False, device=None, continuity=2, mixing="geometric"):
        import numpy as np
        import torch
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        boxes = np.asarray(boxes, dtype=np.float64).reshape(-1, 3)
        self.nbox = len(boxes)
        self.n_per_box = np.asarray(n_per_box, dtype=np.int64).reshape(-1)
        if len(self.n_per_box) != self.nbox:
            raise ValueError("one atom count per box")
        lv = np.broadcast_to(np.asarray(levels, dtype=np.int64), (self.nbox,))
        params = (_lib.MLSParams * self.nbox)()
        for b in range(self.nbox):
            params[b] = _params(boxes[b], cutoff, h, order, int(lv[b]), None, precision, continuity, mixing)
        counts = (ctypes.c_int64 * self.nbox)(*[int(x) for x in self.n_per_box])
        self.offsets = np.concatenate([[0], np.cumsum(self.n_per_box)]).astype(np.int64)
        self.n_total = int(self.offsets[-1])
        self._batch = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_batch_create(self.nbox, params, counts, int(bool(autotune)),
                                                  ctypes.byref(self._batch)), "mls_batch_create")

    def box_info(self, b):
        inf = _lib.MLSPlanInfo()
        _lib.check(self._lib.mls_batch_box_info(self._batch, int(b), ctypes.byref(inf)), "mls_batch_box_info")
        return dict(levels=inf.levels, grid=tuple(inf.grid), coarsest=tuple(inf.coarsest), cells=tuple(inf.cells),
                    h_eff=tuple(inf.h_eff), taps=int(inf.taps), cell_width=tuple(inf.cell_width))

    def evaluate(self, pos, c6, forces=True, dE_dc6=False, out=None, stream=None):
        """Enqueue one batched evaluation on the current torch stream (or ``stream``)."""
        import torch
        if pos.device != self.device or c6.device != self.device:
            raise ValueError("pos and c6 must live on the batch's device")
        if pos.dtype != torch.float64 or c6.dtype != torch.float64:
            raise TypeError("pos and c6 must be float64")
        if tuple(pos.shape) != (self.n_total, 3) or tuple(c6.shape) != (self.n_total,):
            raise ValueError(f"pos must be ({self.n_total}, 3) and c6 ({self.n_total},)")
        if not (pos.is_contiguous() and c6.is_contiguous()):
            raise ValueError("pos and c6 must be contiguous")
        if out is None:
            out = BatchResult(torch.empty(self.nbox, dtype=torch.float64, device=self.device),
                              torch.empty((self.n_total, 3), dtype=torch.float64, device=self.device)
                              if forces else None,
                              torch.empty(self.n_total, dtype=torch.float64, device=self.device)
                              if dE_dc6 else None)
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_batch_evaluate(self._batch, _ptr(pos), _ptr(c6), _ptr(out.energies),
                                                    _ptr(out.forces), _ptr(out.dE_dc6), ctypes.c_void_p(s)),
                       "mls_batch_evaluate")
        return out

    def evaluate_lb(self, pos, eps, sigma, forces=True, out=None, stream=None):
        """Enqueue one batched Lorentz-Berthelot evaluation (``mls_batch_evaluate_lb``):
        per-atom epsilon and sigma in the batch's row layout."""
        import torch
        for name, t, shape in (("pos", pos, (self.n_total, 3)), ("eps", eps, (self.n_total,)),
                               ("sigma", sigma, (self.n_total,))):
            if t.device != self.device or t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 tensor on the batch's device")
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} must have shape {shape}")
        if out is None:
            out = BatchResult(torch.empty(self.nbox, dtype=torch.float64, device=self.device),
                              torch.empty((self.n_total, 3), dtype=torch.float64, device=self.device)
                              if forces else None)
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(self._lib.mls_batch_evaluate_lb(self._batch, _ptr(pos), _ptr(eps), _ptr(sigma),
                                                       _ptr(out.energies), _ptr(out.forces), ctypes.c_void_p(s)),
                       "mls_batch_evaluate_lb")
        return out

    def set_graph(self, enable=True):
        _lib.check(self._lib.mls_batch_set_graph(self._batch, int(bool(enable))), "mls_batch_set_graph")

    def tuning(self):
        t = _lib.MLSBatchTuning()
        _lib.check(self._lib.mls_batch_get_tuning(self._batch, ctypes.byref(t)), "mls_batch_get_tuning")
        return dict(blocks=dict(zip(_lib.STAGE_NAMES, list(t.blocks))), stencil_zc=int(t.stencil_zc),
                    tuned_ms=float(t.tuned_ms), stage_ms=dict(zip(_lib.STAGE_NAMES, list(t.stage_ms))))

    def set_tuning(self, blocks, stencil_zc=16):
        """Force a launch shape: ``blocks`` is one grid size for every stage or a
        dict stage -> grid (0 = one block per work item)."""
        t = _lib.MLSBatchTuning()
        for i, k in enumerate(_lib.STAGE_NAMES):
            t.blocks[i] = int(blocks[k] if isinstance(blocks, dict) else blocks)
        t.stencil_zc = int(stencil_zc)
        _lib.check(self._lib.mls_batch_set_tuning(self._batch, ctypes.byref(t)), "mls_batch_set_tuning")

    def status(self):
        flags = ctypes.c_int(0)
        st = self._lib.mls_batch_status(self._batch, ctypes.byref(flags))
        if st not in (_lib.MLS_OK, _lib.MLS_ERR_NONFINITE):
            _lib.check(st, "mls_batch_status")
        return flags.value

    def close(self):
        if getattr(self, "_batch", None) is not None and self._batch.value:
            self._lib.mls_batch_destroy(self._batch)
            self._batch = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
