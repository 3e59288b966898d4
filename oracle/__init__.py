"""Plain FP64 CPU oracle for the five-equation finite-volume RHS and SSP-RK3 step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this.

The arithmetic lives in ``orc.c`` (built to ``liborc.so`` with
``-O2 -fno-fast-math -ffp-contract=off -fopenmp``); this module only marshals
numpy arrays.  ``exact_riemann`` holds the exact two-material Riemann solution
used to pin the oracle's discretisation.

Paper: arXiv 2409.10729, Sec. II-A (model, stiffened-gas EOS) and Sec. II-B
(eq. discretization and the cell-integrated form below it; HLLC after Toro,
WENO5 after Shu).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

NV = 7  # variables of the two-fluid model
NFMAX = 4  # fluids the oracle takes
NVMAX = 2 * NFMAX + 3


def nvars(nf: int) -> int:
    """Variables of the nf-fluid model: nf partial densities, three momenta,
    energy and nf - 1 volume fractions."""
    return 2 * nf + 3


class OrcGrid(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("gamma", ctypes.c_double * NFMAX),
        ("pinf", ctypes.c_double * NFMAX),
        ("eps", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("weno_z", ctypes.c_int32),
        ("weno_order", ctypes.c_int32),
        ("inflow", ((ctypes.c_double * NVMAX) * 2) * 3),
        ("nf", ctypes.c_int32),
        ("xf", ctypes.c_void_p * 3),
    ]


def build(force: bool = False) -> str:
    """Compile liborc.so with gcc (plain C, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
             "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(OrcGrid)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.orc_weno5.argtypes = [dp, ctypes.c_double, dp, dp]
        L.orc_weno5_betas.argtypes = [dp, dp]
        L.orc_weno5_z.argtypes = [dp, ctypes.c_double, dp, dp]
        L.orc_weno3.argtypes = [dp, ctypes.c_double, dp, dp]
        L.orc_weno5_nu.argtypes = [dp, dp, ctypes.c_double, dp, dp]
        L.orc_weno5_nu_betas.argtypes = [dp, dp, dp]
        L.orc_ideal_weights_nu.argtypes = [dp, dp, dp]
        L.orc_hllc.argtypes = [gp, dp, dp, ctypes.c_int, dp, dp]
        L.orc_sound_speed.argtypes = [gp, dp]
        L.orc_sound_speed.restype = ctypes.c_double
        L.orc_cons_to_prim_cell.argtypes = [gp, dp, dp]
        L.orc_prim_to_cons_cell.argtypes = [gp, dp, dp]
        L.orc_prim_to_cons.argtypes = [gp, dp, dp]
        L.orc_cons_to_prim.argtypes = [gp, dp, dp]
        L.orc_rhs.argtypes = [gp, dp, dp]
        L.orc_rhs_at.argtypes = [gp, dp, ctypes.c_int64, i64p, dp]
        L.orc_rhs_learned.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_int, dp, i64p]
        L.orc_rhs_learned_at.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_int64, i64p, dp]
        L.orc_mlp_omega.argtypes = [dp, ctypes.c_int64, dp, dp, dp]
        L.orc_gelu.argtypes = [ctypes.c_double]
        L.orc_gelu.restype = ctypes.c_double
        L.orc_gelu_tanh.argtypes = [ctypes.c_double]
        L.orc_gelu_tanh.restype = ctypes.c_double
        L.orc_cfl_dt.argtypes = [gp, dp]
        L.orc_cfl_dt.restype = ctypes.c_double
        L.orc_rk3_combine.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp, ctypes.c_double, dp]
        L.orc_rk3_step.argtypes = [gp, dp, ctypes.c_double]
        L.orc_rk3_step.restype = ctypes.c_double
        L.orc_run.argtypes = [gp, dp, ctypes.c_int, dp, dp]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_team_size.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_grid(spec: dict, weno_z: bool = False) -> OrcGrid:
    """Grid from a problem description dict (keys n, dx, bc, gamma, pinf, eps,
    cfl, and optionally weno_order: 5 or 3, weno_z: bool, inflow: the
    conserved ghost state [3][2][7] of inflow sides).  weno_z (argument or
    key) selects the WENO-Z weights (a comparison form) instead of
    Jiang-Shu's.  bc: 0 periodic, 1 transmissive, 2 reflective, 3 inflow."""
    g = OrcGrid()
    for d in range(3):
        g.n[d] = int(spec["n"][d])
        g.dx[d] = float(spec["dx"][d])
        g.bc[d][0] = int(spec["bc"][d][0])
        g.bc[d][1] = int(spec["bc"][d][1])
    gam, pin = list(map(float, spec["gamma"])), list(map(float, spec["pinf"]))
    if not (2 <= len(gam) <= NFMAX and len(pin) == len(gam)):
        raise ValueError(f"gamma and pinf must list 2..{NFMAX} fluids alike")
    g.nf = len(gam)
    for f in range(g.nf):
        g.gamma[f], g.pinf[f] = gam[f], pin[f]
    g.eps = float(spec.get("eps", 1e-6))
    g.cfl = float(spec.get("cfl", 0.4))
    g.weno_z = 1 if (weno_z or spec.get("weno_z", False)) else 0
    g.weno_order = int(spec.get("weno_order", 5))
    if g.weno_order not in (3, 5):
        raise ValueError("weno_order must be 3 or 5")
    for d in range(3):
        kinds = (g.bc[d][0], g.bc[d][1])
        if any(k not in (0, 1, 2, 3) for k in kinds):
            raise ValueError("bc must be 0 (periodic), 1 (transmissive), 2 (reflective) or 3 (inflow)")
        if 2 in kinds and 1 < g.n[d] < 3:
            raise ValueError("a reflective side needs at least 3 cells in its direction")
    faces = spec.get("faces")
    g._faces = []  # keeps the face arrays alive while the grid is used
    if faces is not None:
        for d in range(3):
            if faces[d] is None:
                continue
            xf = np.ascontiguousarray(faces[d], dtype=np.float64)
            if xf.shape != (g.n[d] + 1,) or not np.all(np.diff(xf) > 0):
                raise ValueError(f"faces[{d}] must hold n[{d}] + 1 increasing coordinates")
            if g.weno_order != 5 or g.weno_z:
                raise ValueError("non-uniform cells take WENO5 with Jiang-Shu weights")
            g._faces.append(xf)
            g.xf[d] = xf.ctypes.data
    if "inflow" in spec:
        nv = nvars(g.nf)
        a = np.asarray(spec["inflow"], dtype=np.float64).reshape(3, 2, nv)
        for d in range(3):
            for side in range(2):
                for v in range(nv):
                    g.inflow[d][side][v] = float(a[d, side, v])
    return g


def _shape(g: OrcGrid):
    return (nvars(g.nf), g.n[2], g.n[1], g.n[0])


def _state(g: OrcGrid, a, name: str = "state", copy: bool = False) -> np.ndarray:
    """a as a C-contiguous float64 array of the grid's state shape
    [nv, nz, ny, nx]; anything else raises (the C routines index the whole
    grid and would read or write past a smaller buffer)."""
    a = np.array(a, dtype=np.float64, order="C", copy=True) if copy else np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != _shape(g):
        raise ValueError(f"{name} has shape {a.shape}; the grid's state shape is {_shape(g)}")
    return a


def prim_to_cons(g: OrcGrid, w: np.ndarray) -> np.ndarray:
    w = _state(g, w, "w")
    q = np.empty_like(w)
    lib().orc_prim_to_cons(ctypes.byref(g), _dp(w), _dp(q))
    return q


def cons_to_prim(g: OrcGrid, q: np.ndarray) -> np.ndarray:
    q = _state(g, q, "q")
    w = np.empty_like(q)
    lib().orc_cons_to_prim(ctypes.byref(g), _dp(q), _dp(w))
    return w


def rhs(g: OrcGrid, q: np.ndarray) -> np.ndarray:
    q = _state(g, q, "q")
    out = np.empty_like(q)
    lib().orc_rhs(ctypes.byref(g), _dp(q), _dp(out))
    return out


def rhs_at(g: OrcGrid, q: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """RHS at linear cell indices ``cells``; returns [ncell, 7]."""
    q = _state(g, q, "q")
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    if cells.size and (cells.min() < 0 or cells.max() >= g.n[0] * g.n[1] * g.n[2]):
        raise ValueError("cell index outside the grid")
    out = np.empty((cells.size, nvars(g.nf)), dtype=np.float64)
    lib().orc_rhs_at(ctypes.byref(g), _dp(q), cells.size,
                     cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    return out


LEARNED_PER_VARIABLE, LEARNED_SHARED = 1, 2


def rhs_learned(g: OrcGrid, q: np.ndarray, theta, mode: int = LEARNED_PER_VARIABLE, plant: int = 0):
    """Right-hand side with learned WENO weights (fifth order) as the solver
    applies them: features of every edge's stencil (the left edge as the
    reversed stencil's right edge), the network with bfloat16 operands,
    omega = softmax(ln omega_JS + z), and the per-edge Jiang-Shu fallback.
    theta: the 1347 parameters (float32 values); mode 1 per variable, 2
    shared per edge.  Returns (rhs, fallback edges, near-threshold
    decisions), counting the two edges of every distinct face once.
    plant != 0 (tests only) builds in a deliberate mistake (see orc.c)."""
    if g.nf != 2:
        raise ValueError("the learned weights are defined for two fluids")
    if any(g.xf[d] for d in range(3)):
        raise ValueError("the learned weights are defined on uniform cells")
    q = _state(g, q, "q")
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32), dtype=np.float64)
    assert th.size == 1347
    out = np.empty_like(q)
    counts = np.zeros(2, dtype=np.int64)
    lib().orc_rhs_learned(ctypes.byref(g), _dp(q), _dp(th), int(mode), int(plant), _dp(out),
                          counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out, int(counts[0]), int(counts[1])


def rhs_learned_at(g: OrcGrid, q: np.ndarray, theta, cells: np.ndarray, mode: int = LEARNED_PER_VARIABLE):
    """The learned right-hand side of rhs_learned at linear cell indices
    ``cells``, cell by cell (equal to rhs_learned there); returns
    [ncell, 7]."""
    if g.nf != 2:
        raise ValueError("the learned weights are defined for two fluids")
    if any(g.xf[d] for d in range(3)):
        raise ValueError("the learned weights are defined on uniform cells")
    q = _state(g, q, "q")
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32), dtype=np.float64)
    assert th.size == 1347
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    if cells.size and (cells.min() < 0 or cells.max() >= g.n[0] * g.n[1] * g.n[2]):
        raise ValueError("cell index outside the grid")
    out = np.empty((cells.size, NV), dtype=np.float64)
    lib().orc_rhs_learned_at(ctypes.byref(g), _dp(q), _dp(th), int(mode), cells.size,
                             cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    return out


def mlp_omega(theta, X, base) -> np.ndarray:
    """Weights softmax(ln base + z(X)) of single samples, the network with
    bfloat16 operands as in rhs_learned.  X [n, 5], base [n, 3]."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32), dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 5)
    base = np.ascontiguousarray(base, dtype=np.float64).reshape(-1, 3)
    om = np.empty((X.shape[0], 3))
    lib().orc_mlp_omega(_dp(th), X.shape[0], _dp(X), _dp(base), _dp(om))
    return om


def gelu(a: float) -> float:
    """GELU as the learned weights' inference evaluates it (the polynomial
    form of the tanh form's remainder; see orc.c gelu_inference)."""
    return lib().orc_gelu(float(a))


def gelu_tanh(a: float) -> float:
    """The tanh form of GELU (the training form)."""
    return lib().orc_gelu_tanh(float(a))


def cfl_dt(g: OrcGrid, q: np.ndarray) -> float:
    q = _state(g, q, "q")
    return lib().orc_cfl_dt(ctypes.byref(g), _dp(q))


def rk3_combine(stage: int, qn: np.ndarray, qs: np.ndarray, L: np.ndarray, dt: float) -> np.ndarray:
    qn = np.ascontiguousarray(qn, dtype=np.float64)
    qs = np.ascontiguousarray(qs, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    out = np.empty_like(qs)
    lib().orc_rk3_combine(int(stage), qs.size, _dp(qn), _dp(qs), _dp(L), float(dt), _dp(out))
    return out


def rk3_step(g: OrcGrid, q: np.ndarray, dt: float = 0.0):
    """One SSP-RK3 step; returns (new q, dt used).  dt <= 0 selects the CFL dt."""
    q = _state(g, q, "q", copy=True)
    used = lib().orc_rk3_step(ctypes.byref(g), _dp(q), float(dt))
    return q, used


def run(g: OrcGrid, q: np.ndarray, nsteps: int, dts=None):
    """nsteps steps; returns (q, dts used).  ``dts`` replays a prescribed sequence."""
    q = _state(g, q, "q", copy=True)
    out = np.empty(max(nsteps, 1), dtype=np.float64)
    if dts is not None:
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        assert dts.size >= nsteps
    lib().orc_run(ctypes.byref(g), _dp(q), int(nsteps), _dp(dts) if dts is not None else None, _dp(out))
    return q, out[:nsteps]


def weno5(v, eps=1e-6):
    """(left edge, right edge) of the middle cell of a 5-value stencil."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    l = ctypes.c_double()
    r = ctypes.c_double()
    lib().orc_weno5(_dp(v), float(eps), ctypes.byref(l), ctypes.byref(r))
    return l.value, r.value


def weno3(v, eps=1e-6):
    """(left edge, right edge) of the middle cell of a 3-value stencil,
    WENO3 with Jiang-Shu weights."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    l = ctypes.c_double()
    r = ctypes.c_double()
    lib().orc_weno3(_dp(v), float(eps), ctypes.byref(l), ctypes.byref(r))
    return l.value, r.value


def weno5_nu(h, v, eps=1e-6):
    """(left edge, right edge) of the middle cell of five cells of widths h
    with averages v: WENO5 with Jiang-Shu weights on non-uniform cells."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    l = ctypes.c_double()
    r = ctypes.c_double()
    lib().orc_weno5_nu(_dp(h), _dp(v), float(eps), ctypes.byref(l), ctypes.byref(r))
    return l.value, r.value


def weno5_nu_betas(h, v):
    h = np.ascontiguousarray(h, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    b = np.empty(3)
    lib().orc_weno5_nu_betas(_dp(h), _dp(v), _dp(b))
    return b


def ideal_weights_nu(h):
    """(right-edge, left-edge) ideal weights of the middle of five cells of widths h."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    dr = np.empty(3)
    dl = np.empty(3)
    lib().orc_ideal_weights_nu(_dp(h), _dp(dr), _dp(dl))
    return dr, dl


def weno5_z(v, eps=1e-6):
    """(left edge, right edge) with WENO-Z weights (comparison form)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    l = ctypes.c_double()
    r = ctypes.c_double()
    lib().orc_weno5_z(_dp(v), float(eps), ctypes.byref(l), ctypes.byref(r))
    return l.value, r.value


def weno5_betas(v):
    """The three smoothness indicators of the middle cell of a 5-value stencil."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    b = np.empty(3, dtype=np.float64)
    lib().orc_weno5_betas(_dp(v), _dp(b))
    return b


def hllc(g: OrcGrid, wl, wr, d: int):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    F = np.empty(nvars(g.nf), dtype=np.float64)
    uf = ctypes.c_double()
    lib().orc_hllc(ctypes.byref(g), _dp(wl), _dp(wr), int(d), _dp(F), ctypes.byref(uf))
    return F, uf.value


def sound_speed(g: OrcGrid, w) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().orc_sound_speed(ctypes.byref(g), _dp(w))


def max_threads() -> int:
    return lib().orc_max_threads()


def team_size() -> int:
    """Threads the oracle's parallel regions actually run with."""
    return lib().orc_team_size()


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel regions (results do not
    depend on it)."""
    lib().orc_set_threads(int(n))
