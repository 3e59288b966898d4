"""ctypes binding of the mfx C ABI (include/mfx.h).

Argument marshalling only: every step of the solver runs in the HIP library
``libmfx.so`` built in-tree next to this file.  Importing this module fails
loudly if the library is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfx.so")

MFX_OK, MFX_EINVAL, MFX_EHIP, MFX_ENOMEM, MFX_ESTATE = 0, -1, -2, -3, -4
MFX_BC_PERIODIC, MFX_BC_TRANSMISSIVE, MFX_BC_REFLECTIVE, MFX_BC_INFLOW = 0, 1, 2, 3
MFX_FP64, MFX_FP32_MIXED = 0, 1
MFX_WENO5_JS, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE, MFX_WENO5_Z = 0, 1, 2, 3
MFX_STATUS_RHO, MFX_STATUS_SOUND, MFX_STATUS_NONFINITE, MFX_STATUS_ALPHA = 1, 2, 4, 8
MFX_STATUS_ERRORS = MFX_STATUS_RHO | MFX_STATUS_SOUND | MFX_STATUS_NONFINITE

EXPORTED = (
    "mfx_workspace_bytes", "mfx_init_grid", "mfx_set_state", "mfx_set_primitive", "mfx_get_state",
    "mfx_rhs", "mfx_rk3_step", "mfx_set_mlp", "mfx_stats", "mfx_profile", "mfx_profile_read",
    "mfx_destroy", "mfx_last_error", "mfx_mlp_sample_stencils", "mfx_mlp_face_targets", "mfx_mlp_features", "mfx_mlp_features_edge",
    "mfx_mlp_packed_bytes",
    "mfx_mlp_pack", "mfx_mlp_forward", "mfx_mlp_grad_workspace", "mfx_mlp_loss_grad", "mfx_mlp_adam",
    "mfx_mlp_last_error", "mfx_rhs_static", "mfx_weno5_nu_coefficients",
)
NU_COEFS = 33
STATIC_SCRATCH_BYTES = 128 << 20
MLP_PARAMS = 1347
MAX_FLUIDS = 3
MAX_VARS = 2 * MAX_FLUIDS + 3


def nvars(spec: dict) -> int:
    """Variables per cell of a problem: 2 * (number of fluids) + 3."""
    return 2 * len(spec["gamma"]) + 3
PROF_KINDS = 40


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("gamma", ctypes.c_double * MAX_FLUIDS),
        ("pi_inf", ctypes.c_double * MAX_FLUIDS),
        ("cfl", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("weights", ctypes.c_int32),
        ("weno_order", ctypes.c_int32),
        ("inflow", ((ctypes.c_double * MAX_VARS) * 2) * 3),
        ("num_fluids", ctypes.c_int32),
        ("faces", ctypes.c_void_p * 3),
    ]


class MfxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mfx error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmfx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_2409_10729_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(GridDesc)
        L.mfx_workspace_bytes.argtypes = [dp]
        L.mfx_workspace_bytes.restype = ctypes.c_size_t
        L.mfx_init_grid.argtypes = [dp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.mfx_init_grid.restype = ctypes.c_int
        for name in ("mfx_set_state", "mfx_set_primitive", "mfx_get_state", "mfx_rhs"):
            f = getattr(L, name)
            f.argtypes = [vp, vp]
            f.restype = ctypes.c_int
        L.mfx_rk3_step.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.mfx_rk3_step.restype = ctypes.c_int
        L.mfx_set_mlp.argtypes = [vp, vp, ctypes.c_int32]
        L.mfx_set_mlp.restype = ctypes.c_int
        L.mfx_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32)]
        L.mfx_stats.restype = ctypes.c_int
        L.mfx_profile.argtypes = [vp, ctypes.c_int]
        L.mfx_profile.restype = ctypes.c_int
        L.mfx_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.mfx_profile_read.restype = ctypes.c_int
        i64 = ctypes.c_int64
        L.mfx_mlp_sample_stencils.argtypes = [dp, vp, vp, vp, vp, vp]
        L.mfx_mlp_sample_stencils.restype = ctypes.c_int
        L.mfx_mlp_face_targets.argtypes = [dp, vp, ctypes.c_int32, vp, vp]
        L.mfx_mlp_face_targets.restype = ctypes.c_int
        L.mfx_mlp_features.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, vp, vp, vp]
        L.mfx_mlp_features.restype = ctypes.c_int
        L.mfx_mlp_features_edge.argtypes = [vp, vp, i64, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp]
        L.mfx_mlp_features_edge.restype = ctypes.c_int
        L.mfx_mlp_packed_bytes.argtypes = []
        L.mfx_mlp_packed_bytes.restype = ctypes.c_size_t
        L.mfx_mlp_pack.argtypes = [vp, vp, vp]
        L.mfx_mlp_pack.restype = ctypes.c_int
        L.mfx_mlp_forward.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.mfx_mlp_forward.restype = ctypes.c_int
        L.mfx_mlp_grad_workspace.argtypes = [i64]
        L.mfx_mlp_grad_workspace.restype = ctypes.c_size_t
        L.mfx_mlp_loss_grad.argtypes = [vp, vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_float, vp, ctypes.c_size_t,
                                         vp, vp, vp]
        L.mfx_mlp_loss_grad.restype = ctypes.c_int
        L.mfx_mlp_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp]
        L.mfx_mlp_adam.restype = ctypes.c_int
        L.mfx_mlp_last_error.argtypes = []
        L.mfx_mlp_last_error.restype = ctypes.c_char_p
        L.mfx_rhs_static.argtypes = [dp, vp, vp, vp]
        L.mfx_rhs_static.restype = ctypes.c_int
        L.mfx_weno5_nu_coefficients.argtypes = [vp, vp]
        L.mfx_weno5_nu_coefficients.restype = ctypes.c_int
        L.mfx_destroy.argtypes = [vp]
        L.mfx_destroy.restype = None
        L.mfx_last_error.argtypes = [vp]
        L.mfx_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def make_desc(spec: dict, precision: int = MFX_FP64, weights: int = MFX_WENO5_JS) -> GridDesc:
    d = GridDesc()
    for k in range(3):
        d.n[k] = int(spec["n"][k])
        d.lo[k] = float(spec.get("lo", (0.0, 0.0, 0.0))[k])
        d.dx[k] = float(spec["dx"][k])
        d.bc[k][0] = int(spec["bc"][k][0])
        d.bc[k][1] = int(spec["bc"][k][1])
    gam, pin = list(map(float, spec["gamma"])), list(map(float, spec["pinf"]))
    if not (2 <= len(gam) <= MAX_FLUIDS and len(pin) == len(gam)):
        raise ValueError(f"gamma and pinf must list 2..{MAX_FLUIDS} fluids alike")
    d.num_fluids = len(gam)
    for f in range(len(gam)):
        d.gamma[f], d.pi_inf[f] = gam[f], pin[f]
    d.cfl = float(spec.get("cfl", 0.4))
    d.weno_eps = float(spec.get("eps", 1e-6))
    d.precision = int(precision)
    d.weights = int(weights)
    d.weno_order = int(spec.get("weno_order", 5))
    faces = spec.get("faces")
    d._faces = []  # host face arrays, alive as long as the descriptor (read at workspace sizing and init)
    if faces is not None:
        import numpy as np

        for k in range(3):
            if faces[k] is None:
                continue
            xf = np.ascontiguousarray(faces[k], dtype=np.float64)
            if xf.shape != (d.n[k] + 1,):
                raise ValueError(f"faces[{k}] must hold n[{k}] + 1 coordinates")
            d._faces.append(xf)
            d.faces[k] = xf.ctypes.data
    if "inflow" in spec:
        nv = 2 * len(gam) + 3
        a = [[list(map(float, side)) for side in pair] for pair in spec["inflow"]]
        for k in range(3):
            for s in range(2):
                for v in range(nv):
                    d.inflow[k][s][v] = a[k][s][v]
    return d


def check_mlp(rc: int):
    if rc != MFX_OK:
        msg = lib().mfx_mlp_last_error()
        raise MfxError(rc, msg.decode() if msg else "")


def check(rc: int, ctx=None):
    if rc != MFX_OK:
        msg = lib().mfx_last_error(ctx)
        raise MfxError(rc, msg.decode() if msg else "")
