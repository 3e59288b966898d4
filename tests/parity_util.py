"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI,
run the oracle, and compare per field with the relative max norm
    relLinf_k = max_i |x_i - y_i| / max_i |y_i|.
"""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-12  # FP64 path against the FP64 oracle, per conserved field


MOMENTUM = (2, 3, 4)  # two fluids


def _nf(nv: int) -> int:
    """Fluids of a state with nv variables (2 nf + 3)."""
    return (nv - 3) // 2


def _shared_momentum(scale: np.ndarray) -> np.ndarray:
    """The three momentum components share one scale, so the error norm does
    not depend on how the axes are oriented (a problem with v = w = 0 has
    max|rho v| = 0, which cannot serve as a scale)."""
    scale = scale.copy()
    m = _nf(scale.size)
    scale[m:m + 3] = scale[m:m + 3].max()
    return scale


def rel_linf(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """State error per field: max|x - y| / max|y|, momentum sharing one scale."""
    x = x.reshape(x.shape[0], -1)
    y = y.reshape(y.shape[0], -1)
    den = _shared_momentum(np.abs(y).max(axis=1))
    den = np.where(den > 0, den, 1.0)
    return np.abs(x - y).max(axis=1) / den


def inv_width(spec, d: int) -> float:
    """Largest 1 / (cell width) along direction d: 1 / dx, or on unequal
    cells (spec["faces"]) the reciprocal of the narrowest cell."""
    faces = spec.get("faces")
    if faces is not None and faces[d] is not None:
        return 1.0 / np.diff(np.asarray(faces[d], dtype=np.float64)).min()
    return 1.0 / spec["dx"][d]


def physical_flux_scale(q: np.ndarray, spec) -> np.ndarray:
    """Per field, max over cells of sum_d |F_k,d(q)| / dx_d with the model's
    physical flux F alone (the scale the FP64 right-hand-side bar was first
    written with; flux_scale adds the wave-speed term)."""
    g = oracle.make_grid(spec)
    nv = q.shape[0]
    m, e = _nf(nv), _nf(nv) + 3
    w = oracle.cons_to_prim(g, q).reshape(nv, -1)
    qq = q.reshape(nv, -1)
    p = w[e]
    tot = np.zeros_like(qq)
    for d in range(3):
        if spec["n"][d] <= 1:
            continue
        ud = w[m + d]
        F = np.abs(qq * ud)
        F[m + d] = np.abs(qq[m + d] * ud + p)
        F[e] = np.abs((qq[e] + p) * ud)
        tot += F * inv_width(spec, d)
    return _shared_momentum(tot.max(axis=1))


def flux_scale(q: np.ndarray, spec) -> np.ndarray:
    """Size of the terms a right-hand side is a difference of.  An HLLC flux
    is the physical flux of one side plus a wave speed times a jump of the
    state, so per field the terms are bounded by
        max over cells of sum_d |F_k,d(q)| / dx_d  +  lambda * max |q_k|,
    with the model's physical flux F (partial densities and alpha1 times u_d;
    momentum rho u u_d + p delta; energy (rho E + p) u_d) and lambda =
    max over cells of sum_d (|u_d| + c) / dx_d."""
    g = oracle.make_grid(spec)
    nv = q.shape[0]
    m, e = _nf(nv), _nf(nv) + 3
    w = oracle.cons_to_prim(g, q).reshape(nv, -1)
    qq = q.reshape(nv, -1)
    p = w[e]
    tot = np.zeros_like(qq)
    for d in range(3):
        if spec["n"][d] <= 1:
            continue
        ud = w[m + d]
        F = np.abs(qq * ud)
        F[m + d] = np.abs(qq[m + d] * ud + p)
        F[e] = np.abs((qq[e] + p) * ud)
        tot += F * inv_width(spec, d)
    dt = oracle.cfl_dt(g, q)
    lam = spec.get("cfl", 0.4) / dt if np.isfinite(dt) else 0.0
    return _shared_momentum(tot.max(axis=1) + lam * np.abs(qq).max(axis=1))


def rhs_rel_linf(x: np.ndarray, y: np.ndarray, q: np.ndarray, spec) -> np.ndarray:
    """Right-hand-side error per field, scaled by the size of the flux terms it
    is a difference of (flux_scale).  Where L_k vanishes in exact arithmetic
    (uniform alpha1, or uniform pressure for the transverse momentum) both
    sides hold rounding noise of those terms, so max|L_k| is no scale."""
    x = x.reshape(x.shape[0], -1)
    y = y.reshape(y.shape[0], -1)
    den = np.maximum(np.abs(y).max(axis=1), flux_scale(q, spec))
    den = np.where(den > 0, den, 1.0)  # no active direction: L == 0 exactly
    return np.abs(x - y).max(axis=1) / den


def rhs_rel_linf_physical(x: np.ndarray, y: np.ndarray, q: np.ndarray, spec) -> np.ndarray:
    """The same error scaled by max(max|L_k|, physical_flux_scale): the
    stricter scale without the wave-speed term."""
    x = x.reshape(x.shape[0], -1)
    y = y.reshape(y.shape[0], -1)
    den = np.maximum(np.abs(y).max(axis=1), physical_flux_scale(q, spec))
    den = np.where(den > 0, den, 1.0)
    return np.abs(x - y).max(axis=1) / den


def fp64_rhs_errors(x: np.ndarray, y: np.ndarray, q: np.ndarray, spec):
    """(error under flux_scale, error under the physical-flux scale alone):
    the FP64 path must meet the 1e-12 bar under both."""
    return rhs_rel_linf(x, y, q, spec), rhs_rel_linf_physical(x, y, q, spec)


def gpu_solver(spec, q0=None, w0=None, **kw):
    import torch

    from paper_2409_10729_amd import Solver

    s = Solver(spec, **kw)
    if w0 is not None:
        s.set_primitive(torch.from_numpy(np.ascontiguousarray(w0)).cuda())
    else:
        s.set_state(torch.from_numpy(np.ascontiguousarray(q0)).cuda())
    return s


def cross_cells(spec, cells: np.ndarray, reach: int = 3) -> np.ndarray:
    """All cells within `reach` along one active axis of any cell in `cells`
    (boundary index map applied: periodic wraps, transmissive clamps,
    reflective mirrors), as sorted unique linear indices."""
    n = spec["n"]
    i = cells % n[0]
    j = (cells // n[0]) % n[1]
    k = cells // (n[0] * n[1])
    out = [cells]
    pos = [i, j, k]
    for d in range(3):
        if n[d] <= 1:
            continue
        for o in range(-reach, reach + 1):
            if o == 0:
                continue
            p = pos[d] + o
            lo, hi = spec["bc"][d]
            if lo == 0:
                p = np.mod(p, n[d])
            else:
                p = np.where(p < 0, -1 - p if lo == 2 else 0, p)
                p = np.where(p >= n[d], 2 * n[d] - 1 - p if hi == 2 else n[d] - 1, p)
            q = list(pos)
            q[d] = p
            out.append((q[2] * n[1] + q[1]) * n[0] + q[0])
    return np.unique(np.concatenate(out))


def oracle_step_at(spec, q0: np.ndarray, cells: np.ndarray, dt: float) -> np.ndarray:
    """One SSP-RK3 step of the oracle evaluated only at `cells` (returns [7, ncell]).
    Each stage's state is formed on the cells the next stage's stencils reach."""
    g = oracle.make_grid(spec)
    Nc = q0[0].size
    qf = q0.reshape(q0.shape[0], Nc)
    S2 = cross_cells(spec, cells)
    S1 = cross_cells(spec, S2)
    L0 = oracle.rhs_at(g, q0, S1).T
    q1s = oracle.rk3_combine(1, qf[:, S1], qf[:, S1], L0, dt)
    Q1 = np.zeros_like(qf)
    Q1[:, S1] = q1s
    L1 = oracle.rhs_at(g, Q1.reshape(q0.shape), S2).T
    q2s = oracle.rk3_combine(2, qf[:, S2], Q1[:, S2], L1, dt)
    Q2 = np.zeros_like(qf)
    Q2[:, S2] = q2s
    del Q1
    L2 = oracle.rhs_at(g, Q2.reshape(q0.shape), cells).T
    return oracle.rk3_combine(3, qf[:, cells], Q2[:, cells], L2, dt)


def sample_cells(spec, count: int, seed: int, q0: np.ndarray | None = None) -> np.ndarray:
    """Random cells plus every corner/edge-adjacent boundary cell class and,
    if a state is given, the cells with the largest alpha1 and pressure-like
    gradients (interfaces and shocks)."""
    rng = np.random.default_rng(seed)
    n = spec["n"]
    N = n[0] * n[1] * n[2]
    cells = [rng.integers(0, N, size=count)]
    for d in range(3):
        for edge in (0, 1, 2, n[d] - 3, n[d] - 2, n[d] - 1):
            if 0 <= edge < n[d]:
                pos = [rng.integers(0, n[0], 16), rng.integers(0, n[1], 16), rng.integers(0, n[2], 16)]
                pos[d] = np.full(16, edge)
                cells.append((pos[2] * n[1] + pos[1]) * n[0] + pos[0])
    if q0 is not None:
        for v in (5, 6):
            f = q0[v].reshape(n[2], n[1], n[0])
            g = np.abs(np.diff(f, axis=2))
            top = np.argsort(g.ravel())[-count // 4:]
            kk, jj, ii = np.unravel_index(top, g.shape)
            cells.append((kk * n[1] + jj) * n[0] + ii)
    return np.unique(np.concatenate(cells)).astype(np.int64)


def learned_reference(spec, q0: np.ndarray, theta, mode: int):
    """The oracle's learned right-hand side for a GPU comparison, with what
    sizes the comparison's tolerance.

    The kernel forms the network's operands in float32 from the float32
    primitives and rounds them to bfloat16; a different rounding of an
    operand moves the weights, so the learned right-hand side is only as
    well defined as the quantisation's response to float32 rounding of its
    inputs.  That response is measured on the oracle itself: the same
    right-hand side of the state whose primitives are first rounded to
    float32 (sens, per field, relative to flux_scale; and the change of the
    fallback count).  Returns a dict: rhs, fallbacks, near (decisions near a
    threshold), sens [7], fallback_shift."""
    g = oracle.make_grid(spec)
    r, fb, near = oracle.rhs_learned(g, q0, theta, mode)
    w = oracle.cons_to_prim(g, q0)
    q32 = oracle.prim_to_cons(g, w.astype(np.float32).astype(np.float64))
    r32, fb32, _ = oracle.rhs_learned(g, q32, theta, mode)
    sc = flux_scale(q0, spec)
    sens = np.abs(r - r32).reshape(7, -1).max(axis=1) / np.where(sc > 0, sc, 1.0)
    return {"rhs": r, "fallbacks": fb, "near": near, "sens": sens, "fallback_shift": abs(fb - fb32)}


# Float32 arithmetic bar of the reconstruction and Riemann solve (the FP32
# form's right-hand side against the oracle, relative to flux_scale).
FP32_BAR = 1e-5


def learned_tolerance(ref) -> np.ndarray:
    """Per-field tolerance of a learned right-hand side against the oracle:
    the float32 bar plus four times the oracle's own quantisation response."""
    return FP32_BAR + 4.0 * ref["sens"]
