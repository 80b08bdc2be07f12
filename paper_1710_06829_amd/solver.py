"""Torch-facing wrapper of libxfdtd.  PyTorch provides device memory and the
stream; every numerical step runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B

_DT = {torch.float32: B.XFDTD_F32, torch.float64: B.XFDTD_F64}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def consistent_alpha(coeffs):
    """Return the 12 coefficients with alpha_x, alpha_y, alpha_z set by
    eq.(alpha): alpha_a = 1 - 2 beta_ab - 2 beta_ac - 3 delta_a."""
    arr = B.dbl_array(coeffs, 12)
    B.check(B.lib().xfdtd_consistent_alpha(arr))
    return [arr[i] for i in range(12)]


def cfl_limit(shape, coeffs, spacing=(1.0, 1.0, 1.0)):
    """(dt_max, F_min, F_max) of eq. constraints over the whole zone."""
    g = B.make_grid(shape, spacing)
    dtm, fmn, fmx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    B.check(B.lib().xfdtd_cfl_limit(ctypes.byref(g), B.dbl_array(coeffs, 12), ctypes.byref(dtm),
                                    ctypes.byref(fmn), ctypes.byref(fmx)))
    return dtm.value, fmn.value, fmx.value


def dispersion(k: torch.Tensor, dt: float, coeffs, spacing=(1.0, 1.0, 1.0), want_vg=True,
               allow_unstable=False):
    """omega, v_ph, v_g at wave vectors k (device tensor (n, 3), float64)."""
    if not (k.is_cuda and k.dtype == torch.float64 and k.dim() == 2 and k.shape[1] == 3):
        raise ValueError("k must be a float64 CUDA tensor of shape (n, 3)")
    k = k.contiguous()
    n = k.shape[0]
    om = torch.empty(n, dtype=torch.float64, device=k.device)
    vph = torch.empty(n, dtype=torch.float64, device=k.device)
    vg = torch.empty((n, 3), dtype=torch.float64, device=k.device) if want_vg else None
    g = B.make_grid((1, 1, 1), spacing)
    rc = B.lib().xfdtd_dispersion(ctypes.byref(g), float(dt), B.dbl_array(coeffs, 12), _ptr(k), n,
                                  _ptr(om), _ptr(vph), _ptr(vg) if vg is not None else None,
                                  _stream_handle(k.device))
    if rc != 0 and not (allow_unstable and rc == -2):
        B.check(rc)
    return om, vph, vg


class Solver:
    """One periodic box advanced by the extended-stencil FDTD step.

    ``fields`` are six tensors (Ex, Ey, Ez, Bx, By, Bz) of shape (nz, ny, nx)
    on one HIP device, all float32 or all float64; the solver updates them in
    place.  ``scratch=True`` allocates six more arrays so that ``run`` uses
    the fused out-of-place kernel.
    """

    def __init__(self, fields, dt, coeffs, spacing=(1.0, 1.0, 1.0), scratch=True,
                 allow_unstable=False):
        fields = list(fields)
        if len(fields) != 6:
            raise ValueError("need six field tensors")
        t0 = fields[0]
        if t0.dtype not in _DT:
            raise ValueError("fields must be float32 or float64")
        for t in fields:
            if not t.is_cuda or t.dtype != t0.dtype or t.shape != t0.shape or t.dim() != 3:
                raise ValueError("fields must be CUDA tensors of one dtype and shape (nz, ny, nx)")
            if not t.is_contiguous():
                raise ValueError("fields must be contiguous")
            if t.device != t0.device:
                raise ValueError("fields must be on one device")
        self.shape = tuple(t0.shape)
        self.dtype = t0.dtype
        self.device = t0.device
        self.dt = float(dt)
        self.coeffs = [float(c) for c in coeffs]
        self.spacing = tuple(float(s) for s in spacing)
        self.fields = fields
        self.grid = B.make_grid(self.shape, self.spacing)
        h = ctypes.c_void_p()
        B.check(B.lib().xfdtd_create(ctypes.byref(self.grid), self.dt, B.dbl_array(self.coeffs, 12),
                                     _DT[self.dtype], int(bool(allow_unstable)), ctypes.byref(h)))
        self._h = h
        self.scratch = [torch.empty_like(t) for t in fields] if scratch else None
        self._bind()

    def _bind(self):
        arr = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in self.fields])
        sarr = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in self.scratch]) if self.scratch else None
        with torch.cuda.device(self.device):
            B.check(B.lib().xfdtd_bind(self._h, arr, sarr, _stream_handle(self.device)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            B.lib().xfdtd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def flags(self):
        return B.lib().xfdtd_flags(self._h)

    def step_faraday(self):
        self._bind()
        B.check(B.lib().xfdtd_step_faraday(self._h))

    def step_ampere(self, J=None):
        """E^{n+1} = E^n + dt (D x B^{n+1/2}) [- dt J]: J is None or three
        tensors (Jx, Jy, Jz) of the field dtype and shape."""
        self._bind()
        if J is None:
            B.check(B.lib().xfdtd_step_ampere(self._h))
            return
        J = list(J)
        if len(J) != 3 or any(t.shape != self.fields[0].shape or t.dtype != self.dtype or not t.is_contiguous()
                               or t.device != self.device for t in J):
            raise ValueError("J must be three contiguous tensors of the field dtype, shape and device")
        arr = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in J])
        B.check(B.lib().xfdtd_step_ampere_current(self._h, arr))

    def run(self, n: int, check_every: int = 0):
        """n leapfrog steps.  check_every > 0: stop at the first block of that
        many steps that leaves a non-finite value (XfdtdError with code
        XFDTD_ENONFINITE; self.steps_done holds the steps completed)."""
        self._bind()
        if check_every > 0:
            done = ctypes.c_int64()
            rc = B.lib().xfdtd_run_checked(self._h, int(n), int(check_every), ctypes.byref(done))
            self.steps_done = done.value
            B.check(rc)
            return
        B.check(B.lib().xfdtd_run(self._h, int(n)))

    def set_steps_per_pass(self, steps: int):
        """1: one fused step per launch; 2: the two-step kernel.  The
        results are bitwise the same."""
        B.check(B.lib().xfdtd_set_steps_per_pass(self._h, int(steps)))

    def tune(self, force=False):
        """Autotune run()'s kernel and tiling for this box (needs scratch); the
        fields are left unchanged.  Returns the chosen launch_config()."""
        if self.scratch is None:
            raise ValueError("tuning needs scratch=True")
        self._bind()
        ms = ctypes.c_double()
        B.check(B.lib().xfdtd_tune(self._h, int(bool(force)), ctypes.byref(ms)))
        self.tuned_ms = ms.value
        return self.launch_config()

    def launch_config(self):
        """{'tile_x', 'tile_y', 'zchunk', 'workgroups'} of the fused step for
        this box, 'steps_per_pass' of run() and 'two_step': the same keys for
        the two-step kernel."""
        v = [ctypes.c_int() for _ in range(4)]
        B.check(B.lib().xfdtd_launch_config(self._h, *[ctypes.byref(x) for x in v]))
        u = [ctypes.c_int() for _ in range(5)]
        B.check(B.lib().xfdtd_launch_config2(self._h, *[ctypes.byref(x) for x in u]))
        return {"tile_x": v[0].value, "tile_y": v[1].value, "zchunk": v[2].value, "workgroups": v[3].value,
                "steps_per_pass": u[0].value,
                "two_step": {"tile_x": u[1].value, "tile_y": u[2].value, "zchunk": u[3].value,
                             "workgroups": u[4].value}}

    def stats(self):
        """Counters of what this solver ran (xfdtd_get_stats) as a dict;
        elapsed_ms and gcells_per_s are -1 unless timing is on."""
        st = B.Stats()
        B.check(B.lib().xfdtd_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in B.Stats._fields_}

    def reset_stats(self, timing=False):
        """Zero the counters; timing=True times xfdtd_run on the device."""
        B.check(B.lib().xfdtd_reset_stats(self._h, int(bool(timing))))

    def weights(self):
        w = (ctypes.c_double * 15)()
        nw = ctypes.c_int()
        B.check(B.lib().xfdtd_get_weights(self._h, w, ctypes.byref(nw)))
        return [w[i] for i in range(nw.value)]

    def _check_like(self, tensors, count, what):
        """``count`` contiguous tensors of the field shape, dtype and device
        (the library sees only pointers, so sizes are checked here)."""
        tensors = list(tensors)
        if len(tensors) != count:
            raise ValueError(f"{what}: need {count} tensors")
        for t in tensors:
            if (not isinstance(t, torch.Tensor) or tuple(t.shape) != self.shape or t.dtype != self.dtype
                    or t.device != self.device or not t.is_contiguous()):
                raise ValueError(f"{what}: tensors must be contiguous, of shape {self.shape}, "
                                 f"dtype {self.dtype} and on {self.device}")
        return tensors

    def _check_grad(self, grad):
        if (not isinstance(grad, torch.Tensor) or grad.dtype != torch.float64 or grad.numel() != 12
                or grad.device != self.device or not grad.is_contiguous()):
            raise ValueError(f"grad must be a contiguous float64 tensor of 12 values on {self.device}")

    def _check_ws(self, ws):
        if (not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or ws.device != self.device
                or not ws.is_contiguous()):
            raise ValueError(f"the workspace must be a contiguous uint8 tensor on {self.device}")

    def adjoint_step(self, lam_in, lam_out, e_n, grad):
        """One reverse step: lam_out = adjoint(lam_in) with primal input E ``e_n``;
        adds this step's coefficient gradient to ``grad`` (float64 CUDA (12,))."""
        lam_in = self._check_like(lam_in, 6, "lam_in")
        lam_out = self._check_like(lam_out, 6, "lam_out")
        e_n = self._check_like(e_n, 3, "e_n")
        self._check_grad(grad)
        self._bind()
        li = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in lam_in])
        lo = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in lam_out])
        en = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in e_n])
        B.check(B.lib().xfdtd_adjoint_step(self._h, li, lo, en, _ptr(grad)))

    def grad_workspace_bytes(self, n, seg=0):
        b = ctypes.c_uint64()
        B.check(B.lib().xfdtd_grad_workspace(self._h, int(n), int(seg), ctypes.byref(b)))
        return b.value

    def grad_forward(self, n, ws, seg=0):
        self._check_ws(ws)
        self._bind()
        B.check(B.lib().xfdtd_grad_forward(self._h, int(n), int(seg), _ptr(ws), ws.numel()))

    def grad_backward(self, n, ws, lam, seg=0):
        """lam: six tensors, dL/d(final state) in, dL/d(initial state) out.
        Returns dL/dcoeffs as 12 floats.  Consumes the forward pass stored in
        ``ws`` (same n and seg): a second backward needs a new grad_forward."""
        self._check_ws(ws)
        lam = self._check_like(lam, 6, "lam")
        self._bind()
        arr = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in lam])
        g = (ctypes.c_double * 12)()
        B.check(B.lib().xfdtd_grad_backward(self._h, int(n), int(seg), _ptr(ws), ws.numel(), arr, g))
        return [g[i] for i in range(12)]

    def divergence(self):
        """(D*.B, D.E) as new tensors of the field dtype."""
        self._bind()
        db = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        de = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        B.check(B.lib().xfdtd_divergence(self._h, _ptr(db), _ptr(de)))
        return db, de

    def divergence_max(self, ref_b=None, ref_e=None, raise_nonfinite=True):
        """(max|D*.B - ref_b|, max|D.E - ref_e|, #non-finite) reduced on the GPU."""
        for r, name in ((ref_b, "ref_b"), (ref_e, "ref_e")):
            if r is not None:
                self._check_like([r], 1, name)
        self._bind()
        out = (ctypes.c_double * 3)()
        rc = B.lib().xfdtd_divergence_max(self._h, _ptr(ref_b) if ref_b is not None else None,
                                          _ptr(ref_e) if ref_e is not None else None, out)
        if rc != 0 and (raise_nonfinite or rc != -3):
            B.check(rc)
        return out[0], out[1], int(out[2])
