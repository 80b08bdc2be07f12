"""Batched boxes: many periodic boxes of uneven sizes, each with its own
coefficients, advanced together through one graph-captured persistent
kernel per step (see include/xfdtd.h, "Batches")."""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B
from .solver import _DT, _stream_handle


class Batch:
    """``boxes``: list of (fields, dt, coeffs[, spacing]) with six CUDA tensors
    (nz, ny, nx) per box, all of one dtype and device.  The fields are
    updated in place; scratch arrays are allocated here."""

    def __init__(self, boxes, allow_unstable=False, tune=True):
        boxes = [tuple(b) for b in boxes]
        if not boxes:
            raise ValueError("need at least one box")
        f0 = boxes[0][0][0]
        if f0.dtype not in _DT or not f0.is_cuda:
            raise ValueError("fields must be float32/float64 CUDA tensors")
        self.dtype, self.device = f0.dtype, f0.device
        m = len(boxes)
        grids = (B.Grid * m)()
        dts = (ctypes.c_double * m)()
        coeffs = (ctypes.c_double * (12 * m))()
        self.fields, self.scratch = [], []
        for i, bx in enumerate(boxes):
            fields, dt, c = bx[0], bx[1], bx[2]
            sp = bx[3] if len(bx) > 3 else (1.0, 1.0, 1.0)
            fields = list(fields)
            if len(fields) != 6:
                raise ValueError("six fields per box")
            for t in fields:
                if t.dtype != self.dtype or t.device != self.device or t.dim() != 3 or \
                        t.shape != fields[0].shape or not t.is_contiguous():
                    raise ValueError(f"box {i}: fields must be contiguous (nz, ny, nx) tensors "
                                     "of the batch dtype and device")
            grids[i] = B.make_grid(fields[0].shape, sp)
            dts[i] = float(dt)
            cv = B.dbl_array(c, 12)  # exactly 12 coefficients per box
            for j in range(12):
                coeffs[12 * i + j] = cv[j]
            self.fields.append(fields)
            self.scratch.append([torch.empty_like(t) for t in fields])
        h = ctypes.c_void_p()
        B.check(B.lib().xfdtd_batch_create(grids, dts, coeffs, m, _DT[self.dtype],
                                           int(bool(allow_unstable)), ctypes.byref(h)))
        self._h = h
        self.m = m
        self._bind()
        self.tuned_ms = None
        if tune:
            self.tune()

    def _bind(self):
        fa = (ctypes.c_void_p * (6 * self.m))(*[t.data_ptr() for f in self.fields for t in f])
        sa = (ctypes.c_void_p * (6 * self.m))(*[t.data_ptr() for f in self.scratch for t in f])
        with torch.cuda.device(self.device):
            B.check(B.lib().xfdtd_batch_bind(self._h, fa, sa, _stream_handle(self.device)))

    def tune(self, force=False):
        ms = ctypes.c_double()
        B.check(B.lib().xfdtd_batch_tune(self._h, int(bool(force)), ctypes.byref(ms)))
        self.tuned_ms = ms.value
        return self.config()

    def set_config(self, tile_y, zsplit, grid, tile_x=64):
        B.check(B.lib().xfdtd_batch_set_config(self._h, int(tile_x), int(tile_y), int(zsplit), int(grid)))

    def set_steps_per_pass(self, steps):
        """1, or 2: the two-step kernel (FP32, 32-column tiles); bitwise the same results."""
        B.check(B.lib().xfdtd_batch_set_steps_per_pass(self._h, int(steps)))

    def config(self):
        v = [ctypes.c_int() for _ in range(5)]
        B.check(B.lib().xfdtd_batch_get_config(self._h, *[ctypes.byref(x) for x in v]))
        spp = ctypes.c_int()
        B.check(B.lib().xfdtd_batch_get_steps_per_pass(self._h, ctypes.byref(spp)))
        return {"tile_x": v[0].value, "tile_y": v[1].value, "zsplit": v[2].value, "grid": v[3].value,
                "items": v[4].value, "steps_per_pass": spp.value}

    def adjoint_config(self):
        """The batched adjoint's tiling of the last grad_backward (zeros
        before the first)."""
        v = [ctypes.c_int() for _ in range(4)]
        B.check(B.lib().xfdtd_batch_get_adjoint_config(self._h, *[ctypes.byref(x) for x in v]))
        return {"tile_x": v[0].value, "tile_y": v[1].value, "zsplit": v[2].value, "slots": v[3].value}

    def run(self, n, graph=True):
        fn = B.lib().xfdtd_batch_run if graph else B.lib().xfdtd_batch_run_eager
        B.check(fn(self._h, int(n)))

    def grad_workspaces(self, n, seg=0):
        """Allocate one gradient workspace per box (uint8 CUDA tensors)."""
        b = (ctypes.c_uint64 * self.m)()
        B.check(B.lib().xfdtd_batch_grad_workspace(self._h, int(n), int(seg), b))
        return [torch.empty(max(256, b[i]), dtype=torch.uint8, device=self.device) for i in range(self.m)]

    def _ws_args(self, ws):
        ws = list(ws)
        if len(ws) != self.m:
            raise ValueError(f"need {self.m} workspaces, got {len(ws)}")
        for w in ws:
            if w.dtype != torch.uint8 or w.device != self.device or not w.is_contiguous():
                raise ValueError("workspaces must be contiguous uint8 tensors on the batch device")
        ptrs = (ctypes.c_void_p * self.m)(*[w.data_ptr() for w in ws])
        sizes = (ctypes.c_uint64 * self.m)(*[w.numel() for w in ws])
        return ptrs, sizes

    def grad_forward(self, n, ws, seg=0):
        """n steps of every box, storing checkpoints in ``ws``."""
        p, sz = self._ws_args(ws)
        B.check(B.lib().xfdtd_batch_grad_forward(self._h, int(n), int(seg), p, sz))

    def grad_backward(self, n, ws, lams, seg=0):
        """lams: per box six tensors dL/d(final state) in, dL/d(initial state)
        out.  Returns the per-box coefficient gradients (m lists of 12).
        Consumes the forward pass stored in ``ws`` (same list, n and seg)."""
        p, sz = self._ws_args(ws)
        lams = [list(l) for l in lams]
        if len(lams) != self.m or any(len(l) != 6 for l in lams):
            raise ValueError("need six adjoint tensors per box")
        for f, l in zip(self.fields, lams):
            for a, t in zip(f, l):
                if t.shape != a.shape or t.dtype != a.dtype or t.device != a.device or not t.is_contiguous():
                    raise ValueError("adjoint tensors must match their box's fields")
        la = (ctypes.c_void_p * (6 * self.m))(*[t.data_ptr() for l in lams for t in l])
        g = (ctypes.c_double * (12 * self.m))()
        B.check(B.lib().xfdtd_batch_grad_backward(self._h, int(n), int(seg), p, sz, la, g))
        return [[g[12 * i + j] for j in range(12)] for i in range(self.m)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            B.lib().xfdtd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
