"""Reflective (slip-wall) boundaries on the HIP path against the oracle,
through the C ABI.

Every kernel that builds ghost cells is covered: the y and z sweeps (global
loads), the fused x-y pass and the separate x-row kernel (ghost slots of
the row buffer), the marching x sweep (staged loads), and the x boundary
faces with and without their six anchor cells (rows of 6 or more cells, and
shorter ones).  Bar as for the other FP64 parity tests (relative 1e-12);
the float form against the same oracle at 1e-5 of the flux scale.
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import MFX_FP32_MIXED, MFX_WENO5_JS, MFX_WENO5_LEARNED
from paper_2409_10729_amd import workloads as wl
from parity_util import TOL, fp64_rhs_errors, gpu_solver, oracle_step_at, rel_linf, rhs_rel_linf, sample_cells

pytestmark = pytest.mark.gpu

P_, T_, R_ = wl.PERIODIC, wl.TRANSMISSIVE, wl.REFLECTIVE

CASES = [
    ((37, 29, 23), ((R_, R_), (R_, R_), (R_, R_)), 60),  # closed box: fused x-y pass, z
    ((5, 40, 33), ((R_, R_), (P_, P_), (R_, T_)), 61),   # rows under 6 cells: faces without anchors
    ((600, 3, 4), ((R_, R_), (R_, R_), (T_, R_)), 62),   # marching x sweep; 3 cells between walls
    ((420, 6, 3), ((R_, T_), (P_, P_), (R_, R_)), 63),   # long rows: aliased row buffers
    ((3, 70, 9), ((T_, R_), (R_, T_), (P_, P_)), 64),
    ((64, 48, 1), ((R_, R_), (R_, R_), (P_, P_)), 65),   # x-y plane: the fused pass is the last
]


def _report(name, err):
    print(f"{name}: relLinf per field = " + " ".join(f"{e:.2e}" for e in err), flush=True)


def _setup(n, bc, seed):
    P = wl.random_smooth(n=n, seed=seed, bc=bc)
    g = oracle.make_grid(P["spec"])
    return P, g, oracle.prim_to_cons(g, P["w"])


@pytest.mark.parametrize("mode", ["default", "separate_xy", "march"])
@pytest.mark.parametrize("n,bc,seed", CASES)
def test_reflective_rhs_and_step_match_oracle(monkeypatch, n, bc, seed, mode):
    if mode == "separate_xy":
        monkeypatch.setenv("MFX_FUSE_XY", "0")
    elif mode == "march":
        monkeypatch.setenv("MFX_XSWEEP", "march")
    P, g, q0 = _setup(n, bc, seed)
    spec = P["spec"]
    s = gpu_solver(spec, q0=q0)
    r_ref = oracle.rhs(g, q0)
    err, errp = fp64_rhs_errors(s.rhs().cpu().numpy(), r_ref, q0, spec)
    _report(f"reflective rhs {n} {mode}", err)
    _report(f"reflective rhs {n} {mode}" + " (physical-flux scale)", errp)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)
    dt = s.rk3_step(sync=True)
    assert dt == pytest.approx(oracle.cfl_dt(g, q0), rel=1e-15)
    cells = sample_cells(spec, 300, seed=seed, q0=q0)
    ref = oracle_step_at(spec, q0, cells, dt)
    err = rel_linf(s.get_state().cpu().numpy().reshape(7, -1)[:, cells], ref)
    _report(f"reflective step {n} {mode}", err)
    assert np.all(err <= TOL), err
    s32 = gpu_solver(spec, q0=q0, precision=MFX_FP32_MIXED)
    err32 = rhs_rel_linf(s32.rhs().cpu().numpy(), r_ref, q0, spec)
    assert np.all(err32 <= 1e-5), err32


def test_closed_box_run_matches_oracle_and_conserves():
    """A shock hitting a droplet inside a closed box, 8 steps against the
    oracle's whole-grid run; mass of each fluid and the total energy stay
    constant to rounding (no flux crosses a slip wall)."""
    P = wl.shock_droplet(n=(48, 40, 36), seed=1)
    spec = dict(P["spec"], bc=((R_, R_),) * 3)
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, P["w"])
    s = gpu_solver(spec, q0=q0)
    for _ in range(8):
        s.rk3_step()
    q = s.get_state().cpu().numpy()
    q_ref, _ = oracle.run(g, q0, 8)
    err = rel_linf(q, q_ref)
    _report("closed box shock droplet x8", err)
    assert np.all(err <= TOL), err
    for v in (0, 1, 5):
        m0, m1 = q0[v].sum(), q[v].sum()
        assert abs(m1 - m0) <= 1e-12 * np.abs(q0[v]).sum(), (v, m0, m1)


def test_learned_zero_output_layer_matches_js_with_walls():
    """The learned forms build ghost cells through the same loaders: with a
    zero output layer (Jiang-Shu weights through the learned kernels) the
    run tracks the Jiang-Shu float run in a box with reflective sides."""
    import torch

    from paper_2409_10729_amd import Solver, learned

    P = wl.shock_droplet(n=(40, 24, 20), seed=2)
    spec = dict(P["spec"], bc=((R_, T_), (R_, R_), (T_, R_)))

    def solver(weights, params=None):
        s = Solver(spec, precision=MFX_FP32_MIXED, weights=weights)
        if params is not None:
            s.set_mlp(torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda())
        s.set_primitive(torch.from_numpy(P["w"]).cuda())
        return s

    s_l = solver(MFX_WENO5_LEARNED, learned.init_params(1))
    s_j = solver(MFX_WENO5_JS)
    for _ in range(3):
        s_l.rk3_step(2e-7)
        s_j.rk3_step(2e-7)
    d = rel_linf(s_l.get_state().cpu().numpy(), s_j.get_state().cpu().numpy())
    print("learned (zero output layer) vs JS, reflective sides:", d, flush=True)
    assert np.all(d <= 1e-4)
