"""Unequal cell widths (Sec. III-A: a structured mesh refined locally by a
hyperbolic-tangent stretching) on the HIP path against the oracle, through
the C ABI.

A direction with unequal cells reads per-position coefficient tables (x:
the x row kernel, each lane with its own position's coefficients, or the
marching x sweep; y, z: the y/z sweeps), its flux differences divide by
each cell's width, and the CFL reduction reads each cell's widths (in
the last sweep of a step, or the standalone pass).
Covered: stretching along x, y or z alone (next to the fused x-y pass and
the row kernels of equal directions) and along all three; every boundary
type (ghost cells take the widths the boundary rule maps them to); short
segments (tables read at segment starts); the marching x sweep forced, for
rows longer than the row kernel takes and for an inflow side with shared
row buffers; the float form; three fluids; a multi-step shock tube refined
at its interface.  Bar: FP64 relative
1e-12 (both right-hand-side scales, and the state after a step); the time
step equal to the oracle's; the float form 1e-5 of the flux scale.
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import MFX_FP32_MIXED
from paper_2409_10729_amd import workloads as wl
from parity_util import TOL, fp64_rhs_errors, gpu_solver, oracle_step_at, rel_linf, rhs_rel_linf, sample_cells

pytestmark = pytest.mark.gpu

P_, T_, R_, I_ = wl.PERIODIC, wl.TRANSMISSIVE, wl.REFLECTIVE, wl.INFLOW


def _faces(n, which, seed):
    rng = np.random.default_rng(seed)
    out = []
    for d in range(3):
        if d in which:
            out.append(wl.tanh_faces(n[d], centre=rng.uniform(0.3, 0.7), depth=rng.uniform(0.4, 0.7),
                                     sharpness=rng.uniform(6.0, 12.0)))
        else:
            out.append(None)
    return out


def _inflow_states(seed, nf=2):
    rng = np.random.default_rng(seed)
    nv = 2 * nf + 3
    g1 = oracle.make_grid(wl.spec((1, 1, 1), ((P_, P_),) * 3))
    out = np.zeros((3, 2, nv))
    for d in range(3):
        for s in range(2):
            a1 = rng.uniform(0.0, 0.3)
            w = np.array([a1 * 1000.0, (1 - a1) * rng.uniform(1.0, 4.0), rng.uniform(-80, 80),
                          rng.uniform(-80, 80), rng.uniform(-80, 80), rng.uniform(0.8e5, 3e5), a1])
            out[d, s] = oracle.prim_to_cons(g1, w.reshape(7, 1, 1, 1)).reshape(7)
    return out


# (n, bc, stretched directions, seed)
CASES = [
    ((40, 24, 20), ((T_, T_), (P_, P_), (P_, P_)), (0,), 80),        # x rows with tables; y, z equal
    ((48, 36, 16), ((P_, P_), (T_, R_), (P_, P_)), (1,), 81),        # x rows (equal) + y with tables
    ((33, 20, 40), ((R_, T_), (P_, P_), (T_, T_)), (2,), 82),        # fused x-y pass + z with tables
    ((26, 22, 30), ((I_, T_), (P_, P_), (R_, I_)), (0, 1, 2), 83),   # all three, every boundary type
    ((30, 28, 26), ((P_, P_), (P_, P_), (P_, P_)), (0, 1, 2), 84),   # periodic: widths wrap around
    ((200, 1, 1), ((T_, T_), (P_, P_), (P_, P_)), (0,), 85),         # 1D
    ((64, 48, 1), ((R_, R_), (R_, R_), (P_, P_)), (1,), 86),         # x-y plane, walls
    ((5, 40, 7), ((R_, I_), (I_, R_), (T_, R_)), (0, 2), 87),        # short rows between walls
    ((600, 3, 2), ((T_, T_), (P_, P_), (P_, P_)), (0,), 88),         # rows too long: x march with tables
    ((400, 2, 3), ((I_, T_), (P_, P_), (P_, P_)), (0, 1), 89),       # float64: inflow, shared row buffers: march
]


def _report(name, err):
    print(f"{name}: relLinf per field = " + " ".join(f"{e:.2e}" for e in err), flush=True)


def _setup(n, bc, which, seed):
    P = wl.random_smooth(n=n, seed=seed, bc=bc)
    spec = dict(wl.stretched(P, _faces(n, which, seed))["spec"], inflow=_inflow_states(seed))
    g = oracle.make_grid(spec)
    return spec, g, oracle.prim_to_cons(g, P["w"])


@pytest.mark.parametrize("seg,xsweep", [(None, None), (8, None), (None, "march")])
@pytest.mark.parametrize("n,bc,which,seed", CASES)
def test_stretched_rhs_and_step_match_oracle(monkeypatch, n, bc, which, seed, seg, xsweep):
    if seg is not None:
        monkeypatch.setenv("MFX_SWEEP_SEG", str(seg))
    if xsweep is not None:
        monkeypatch.setenv("MFX_XSWEEP", xsweep)
    spec, g, q0 = _setup(n, bc, which, seed)
    print(f"case n={n} bc={bc} stretched={which} seed={seed} seg={seg} x sweep={xsweep}", flush=True)
    s = gpu_solver(spec, q0=q0)
    r_ref = oracle.rhs(g, q0)
    err, errp = fp64_rhs_errors(s.rhs().cpu().numpy(), r_ref, q0, spec)
    _report("stretched rhs", err)
    _report("stretched rhs (physical-flux scale)", errp)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)
    dt = s.rk3_step(sync=True)
    assert dt == pytest.approx(oracle.cfl_dt(g, q0), rel=1e-15)
    cells = sample_cells(spec, 300, seed=seed, q0=q0)
    ref = oracle_step_at(spec, q0, cells, dt)
    err = rel_linf(s.get_state().cpu().numpy().reshape(7, -1)[:, cells], ref)
    _report("stretched step", err)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("n,bc,which,seed", CASES[:4] + CASES[-1:])
def test_stretched_float_form_matches_oracle(n, bc, which, seed):
    spec, g, q0 = _setup(n, bc, which, seed)
    s32 = gpu_solver(spec, q0=q0, precision=MFX_FP32_MIXED)
    err32 = rhs_rel_linf(s32.rhs().cpu().numpy(), oracle.rhs(g, q0), q0, spec)
    _report("stretched rhs float form", err32)
    assert np.all(err32 <= 1e-5), err32


@pytest.mark.parametrize("n,bc,which,seed", [
    ((24, 20, 28), ((T_, T_), (P_, P_), (P_, P_)), (0,), 95),  # z reduces with the x widths
    ((20, 22, 24), ((R_, T_), (P_, P_), (T_, R_)), (0, 1, 2), 96),  # z reduces, every width unequal
    ((40, 36, 1), ((T_, T_), (P_, P_), (P_, P_)), (1,), 97),  # x rows, then the y sweep reduces
])
def test_cfl_in_last_sweep_matches_standalone(monkeypatch, n, bc, which, seed):
    """On unequal cells the CFL reduction inside the last sweep of a step
    reads each cell's widths as the standalone reduction does: the same
    time steps and states bit for bit, and the oracle's CFL time step."""
    spec, g, q0 = _setup(n, bc, which, seed)
    res = []
    for fuse in ("0", "1"):
        monkeypatch.setenv("MFX_FUSE_CFL", fuse)
        s = gpu_solver(spec, q0=q0)
        dts = [s.rk3_step(sync=True) for _ in range(4)]
        q = s.get_state().cpu().numpy()
        dts.append(s.rk3_step(sync=True))  # CFL time step of q, from the fourth step's reduction
        res.append((dts, q))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    assert res[1][0][-1] == pytest.approx(oracle.cfl_dt(g, res[1][1]), rel=1e-15)


def test_full_size_stretched_rhs_sampled():
    """256^3 shock droplet on cells stretched in all three directions
    (finest cells at the droplet), in the benchmark's launch configuration:
    the right-hand side and one CFL step on sampled cells."""
    P = wl.shock_droplet_stretched(n=256, seed=0)
    spec = P["spec"]
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, P["w"])
    del P
    s = gpu_solver(spec, q0=q0)
    r = s.rhs().cpu().numpy().reshape(7, -1)
    cells = sample_cells(spec, 3000, seed=5, q0=q0)
    err, errp = fp64_rhs_errors(r[:, cells], oracle.rhs_at(g, q0, cells).T, q0, spec)
    _report(f"stretched rhs 256^3 on {cells.size} cells", err)
    _report(f"stretched rhs 256^3 on {cells.size} cells (physical-flux scale)", errp)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)
    dt = s.rk3_step(sync=True)
    assert dt == pytest.approx(oracle.cfl_dt(g, q0), rel=1e-15)
    q = s.get_state().cpu().numpy().reshape(7, -1)
    s.destroy()
    cells = sample_cells(spec, 200, seed=6, q0=q0)
    err = rel_linf(q[:, cells], oracle_step_at(spec, q0, cells, dt))
    _report(f"stretched step 256^3 on {cells.size} cells", err)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("which", [(0,), (1, 2), (0, 1, 2)])
def test_stretched_three_fluids_match_oracle(which):
    n = (28, 20, 18)
    bc = ((T_, R_), (P_, P_), (I_, T_))
    P = wl.random_smooth_nf(n=n, seed=90, bc=bc, nf=3)
    spec = wl.stretched(P, _faces(n, which, 90))["spec"]
    nv = 9
    inflow = np.zeros((3, 2, nv))
    # one cell's primitives as an inflow state, converted on a one-cell grid
    one = dict(spec, n=(1, 1, 1), faces=None, bc=((P_, P_),) * 3)
    wz = P["w"][:, :1, :1, :1].copy()
    inflow[2, 0] = oracle.prim_to_cons(oracle.make_grid(one), wz).reshape(nv)
    spec = dict(spec, inflow=inflow)
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, P["w"])
    s = gpu_solver(spec, q0=q0)
    err, errp = fp64_rhs_errors(s.rhs().cpu().numpy(), oracle.rhs(g, q0), q0, spec)
    _report(f"stretched three fluids {which}", err)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)
    dt = s.rk3_step(sync=True)
    q1, dt_ref = oracle.rk3_step(g, q0)
    assert dt == pytest.approx(dt_ref, rel=1e-15)
    err = rel_linf(s.get_state().cpu().numpy(), q1)
    assert np.all(err <= TOL), err


def test_refined_shock_tube_run_matches_oracle():
    """The water/air shock tube on 400 cells refined three-fold around the
    interface: 60 steps with the automatic time step against the oracle's
    whole-grid run (every step's time step equal)."""
    n = 400
    P = wl.shock_tube(n=n)
    faces = wl.tanh_faces(n, centre=0.5, depth=0.66, sharpness=10.0)
    spec = wl.stretched(P, (faces, None, None))["spec"]
    g = oracle.make_grid(spec)
    # cell averages from the same primitive profile at the stretched centres
    xc = 0.5 * (faces[1:] + faces[:-1])
    w = np.where((xc < 0.5).reshape(1, 1, 1, n), P["w"][:, :, :, :1], P["w"][:, :, :, -1:])
    q = oracle.prim_to_cons(g, w)
    s = gpu_solver(spec, q0=q)
    for step in range(60):
        q, dt_ref = oracle.rk3_step(g, q)
        dt = s.rk3_step(sync=True)
        assert dt == pytest.approx(dt_ref, rel=1e-14), (step, dt, dt_ref)
    err = rel_linf(s.get_state().cpu().numpy(), q)
    _report("refined shock tube, 60 steps", err)
    assert np.all(err <= TOL), err
