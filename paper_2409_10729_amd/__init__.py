"""MI355X-native finite-volume right-hand side and SSP-RK3 step for the
two-component five-equation diffuse-interface model (arXiv 2409.10729,
Sec. II).

The solver itself is the HIP library ``libmfx.so`` behind the C ABI in
``include/mfx.h``; this package holds the thin Python binding (names follow
the C calls), the seeded input generators and the build step.  PyTorch
supplies device memory and the HIP stream only.
"""
from __future__ import annotations

import ctypes

from . import _native
from ._native import (MFX_BC_INFLOW, MFX_BC_PERIODIC, MFX_BC_REFLECTIVE, MFX_BC_TRANSMISSIVE, MFX_FP32_MIXED,
                      MFX_FP64, MFX_WENO5_JS, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE, MFX_WENO5_Z, MfxError)

__all__ = ["Solver", "MfxError", "MFX_FP64", "MFX_FP32_MIXED", "MFX_WENO5_JS", "MFX_WENO5_LEARNED",
           "MFX_WENO5_LEARNED_EDGE", "MFX_WENO5_Z",
           "MFX_BC_PERIODIC", "MFX_BC_TRANSMISSIVE", "MFX_BC_REFLECTIVE", "MFX_BC_INFLOW",
           "workspace_bytes", "inflow_states", "rhs_static", "weno5_nu_coefficients"]


def workspace_bytes(spec: dict, precision: int = MFX_FP64, weights: int = MFX_WENO5_JS) -> int:
    d = _native.make_desc(spec, precision, weights)
    return int(_native.lib().mfx_workspace_bytes(ctypes.byref(d)))


def weno5_nu_coefficients(h) -> "np.ndarray":
    """mfx_weno5_nu_coefficients: the 33 WENO5 coefficients the library
    derives for a stencil position from the widths h[0..4] of its five cells
    (candidate coefficients a, b, c as [3][3] each, then the right- and
    left-edge ideal weights).  Host-only."""
    import numpy as np

    h = np.ascontiguousarray(h, dtype=np.float64)
    if h.shape != (5,):
        raise ValueError("h must hold five widths")
    out = np.empty(_native.NU_COEFS)
    _native.check(_native.lib().mfx_weno5_nu_coefficients(ctypes.c_void_p(h.ctypes.data),
                                                          ctypes.c_void_p(out.ctypes.data)))
    return out


def inflow_states(spec: dict, prim) -> "np.ndarray":
    """Conserved ghost states [3][2][7] of inflow sides from primitive
    states prim[3][2][7] (alpha1 rho1, alpha2 rho2, u, v, w, p, alpha1),
    converted on the device by the library's own set_primitive on a
    one-cell grid with the spec's fluids.  Sides whose primitive state is
    all zero stay zero."""
    import numpy as np
    import torch

    nv = _native.nvars(spec)
    prim = np.asarray(prim, dtype=np.float64).reshape(3, 2, nv)
    out = np.zeros((3, 2, nv))
    one = dict(spec, n=(1, 1, 1), bc=((MFX_BC_PERIODIC, MFX_BC_PERIODIC),) * 3)
    one.pop("inflow", None)
    for d in range(3):
        for s in range(2):
            if not prim[d, s].any():
                continue
            sol = Solver(one)
            sol.set_primitive(torch.from_numpy(prim[d, s].reshape(nv, 1, 1, 1).copy()).cuda())
            out[d, s] = sol.get_state().cpu().numpy().reshape(nv)
    return out


def rhs_static(spec: dict, q, out=None, precision: int = MFX_FP64, weights: int = MFX_WENO5_JS, stream=None):
    """mfx_rhs_static: the right-hand side of the state q (float64 device
    tensor [nv, nz, ny, nx]) with no context, no workspace and no device
    allocation in the library (its scratch is a static device array).  out
    (same shape) receives it; it is allocated here (by torch) only if not
    given."""
    import torch

    shape = (_native.nvars(spec), int(spec["n"][2]), int(spec["n"][1]), int(spec["n"][0]))
    for name, t in (("q", q), ("out", out)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 tensor on the device")
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=q.device)
    st = stream if stream is not None else torch.cuda.current_stream(q.device)
    d = _native.make_desc(spec, precision, weights)
    rc = _native.lib().mfx_rhs_static(ctypes.byref(d), ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(st.cuda_stream))
    _native.check(rc, None)
    return out


class Solver:
    """One mfx context on the current CUDA(HIP) device.

    ``spec`` is a problem description (n, dx, bc, gamma, pinf, eps, cfl, and
    optionally weno_order 5 or 3, inflow: the conserved ghost state
    [3][2][7] of MFX_BC_INFLOW sides, and faces: per direction the n + 1
    face coordinates of unequal cells, or None) as produced by
    :mod:`paper_2409_10729_amd.workloads`.  bc per direction and side:
    MFX_BC_PERIODIC, MFX_BC_TRANSMISSIVE, MFX_BC_REFLECTIVE or MFX_BC_INFLOW.
    Arrays passed in and out are torch tensors on the device, float64,
    shape [nv, nz, ny, nx] with nv = 2 * (number of fluids in spec["gamma"]) + 3
    (7 for two fluids).
    """

    def __init__(self, spec: dict, precision: int = MFX_FP64, weights: int = MFX_WENO5_JS, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("mfx needs a HIP device; none is visible to torch")
        self._torch = torch
        self.spec = spec
        self.shape = (_native.nvars(spec), int(spec["n"][2]), int(spec["n"][1]), int(spec["n"][0]))
        L = _native.lib()
        self._desc = _native.make_desc(spec, precision, weights)
        nbytes = int(L.mfx_workspace_bytes(ctypes.byref(self._desc)))
        if nbytes == 0:
            _native.check(L.mfx_init_grid(ctypes.byref(self._desc), None, 0, None, ctypes.byref(ctypes.c_void_p())))
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = L.mfx_init_grid(ctypes.byref(self._desc), ctypes.c_void_p(aligned), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        _native.check(rc, None)
        self._ctx = ctx

    # -- helpers
    def _ptr(self, t, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def _check(self, rc):
        _native.check(rc, self._ctx)

    # -- C ABI, same names
    def set_state(self, q):
        self._check(_native.lib().mfx_set_state(self._ctx, self._ptr(q, "q")))

    def set_primitive(self, w):
        self._check(_native.lib().mfx_set_primitive(self._ctx, self._ptr(w, "w")))

    def get_state(self, out=None):
        if out is None:
            out = self._torch.empty(self.shape, dtype=self._torch.float64, device=self.device)
        self._check(_native.lib().mfx_get_state(self._ctx, self._ptr(out, "out")))
        return out

    def rhs(self, out=None):
        if out is None:
            out = self._torch.empty(self.shape, dtype=self._torch.float64, device=self.device)
        self._check(_native.lib().mfx_rhs(self._ctx, self._ptr(out, "out")))
        return out

    def rk3_step(self, dt: float = 0.0, sync: bool = False):
        """One SSP-RK3 step; dt <= 0 uses the device CFL time step.  With
        sync=True the time step used is returned (one device sync)."""
        if sync:
            used = ctypes.c_double()
            self._check(_native.lib().mfx_rk3_step(self._ctx, float(dt), ctypes.byref(used)))
            return used.value
        self._check(_native.lib().mfx_rk3_step(self._ctx, float(dt), None))
        return None

    def set_mlp(self, params):
        torch = self._torch
        if params.dtype != torch.float32 or params.device != self.device or not params.is_contiguous():
            raise TypeError("params must be a contiguous float32 tensor on the device")
        self._check(_native.lib().mfx_set_mlp(self._ctx, ctypes.c_void_p(params.data_ptr()), params.numel()))

    def stats(self):
        """Time, step count, fallback edges and the status word; "error" holds
        its error bits, "alpha_out" whether alpha1 left [0, 1]."""
        t = ctypes.c_double()
        step = ctypes.c_int64()
        fb = ctypes.c_int64()
        st = ctypes.c_uint32()
        rc = _native.lib().mfx_stats(self._ctx, ctypes.byref(t), ctypes.byref(step), ctypes.byref(fb),
                                     ctypes.byref(st))
        out = {"t": t.value, "step": step.value, "fallback_faces": fb.value, "status": st.value,
               "error": st.value & _native.MFX_STATUS_ERRORS,
               "alpha_out": bool(st.value & _native.MFX_STATUS_ALPHA)}
        if rc not in (_native.MFX_OK, _native.MFX_ESTATE):
            self._check(rc)
        out["rc"] = rc
        return out

    def profile(self, enable: bool = True):
        self._check(_native.lib().mfx_profile(self._ctx, int(bool(enable))))

    def profile_read(self):
        """{(direction, first_pass, output_kind): (total_ms, launches)} since profile()."""
        ms = (ctypes.c_double * _native.PROF_KINDS)()
        n = (ctypes.c_int64 * _native.PROF_KINDS)()
        self._check(_native.lib().mfx_profile_read(self._ctx, ms, n))
        out = {}
        for k in range(_native.PROF_KINDS):
            if n[k]:
                out[(k // 10, (k // 5) % 2, k % 5)] = (ms[k], n[k])
        return out

    def destroy(self):
        if getattr(self, "_ctx", None):
            _native.lib().mfx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
