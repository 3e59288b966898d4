"""Three fluids on the HIP path against the oracle's nf-fluid model,
through the C ABI (mfx_grid_desc.num_fluids = 3; the state holds three
partial densities, the momentum, the energy and two volume fractions).

Bar: FP64 relative 1e-12 per field (right-hand sides under both the flux
scale and the physical-flux scale), the float form 1e-5 of the flux scale.
Covers the fused x-y pass, the x row kernel (alone, and with the row
buffers sharing storage), the marching x sweep (rows longer than the row
kernel takes, an inflow x side with shared row buffers), the y and z
sweeps, every boundary type, WENO5, WENO3 and WENO-Z weights, the CFL time
step, one step and short runs, the status word, the full-size droplet and
bubble workload on sampled cells, and the reduction to two fluids when one
fluid is absent.
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import MFX_FP32_MIXED, MFX_WENO5_JS, MFX_WENO5_Z
from paper_2409_10729_amd import workloads as wl
from parity_util import (TOL, flux_scale, fp64_rhs_errors, gpu_solver, oracle_step_at, physical_flux_scale, rel_linf,
                         rhs_rel_linf, sample_cells)

pytestmark = pytest.mark.gpu

P_, T_, R_, I_ = wl.PERIODIC, wl.TRANSMISSIVE, wl.REFLECTIVE, wl.INFLOW


def _report(name, err):
    print(f"{name}: relLinf per field = " + " ".join(f"{e:.2e}" for e in err), flush=True)


def _inflow3(seed):
    """Conserved three-fluid states [3][2][9] of random valid primitives."""
    rng = np.random.default_rng(seed)
    g1 = oracle.make_grid(wl.spec_fluids((1, 1, 1), ((P_, P_),) * 3, 3))
    out = np.zeros((3, 2, 9))
    for d in range(3):
        for s in range(2):
            a = rng.dirichlet((1.0, 3.0, 1.0))
            w = np.array([a[0] * 1000.0, a[1] * rng.uniform(1.0, 4.0), a[2] * 0.17, rng.uniform(-80, 80),
                          rng.uniform(-80, 80), rng.uniform(-80, 80), rng.uniform(0.8e5, 3e5), a[0], a[1]])
            out[d, s] = oracle.prim_to_cons(g1, w.reshape(9, 1, 1, 1)).reshape(9)
    return out


CASES = [
    ((37, 29, 23), ((T_, T_), (P_, P_), (T_, T_)), 80),
    ((48, 40, 36), ((P_, P_), (P_, P_), (P_, P_)), 81),
    ((1, 40, 33), ((P_, P_), (T_, T_), (P_, P_)), 82),
    ((600, 3, 4), ((T_, T_), (P_, P_), (P_, P_)), 83),
    ((64, 48, 1), ((T_, T_), (P_, P_), (P_, P_)), 84),
    ((257, 1, 1), ((T_, T_), (P_, P_), (P_, P_)), 85),
    ((2, 3, 2), ((P_, P_), (P_, P_), (T_, T_)), 86),
    ((37, 29, 23), ((I_, R_), (R_, I_), (T_, I_)), 87),  # every boundary type
    ((5, 40, 33), ((I_, I_), (P_, P_), (R_, T_)), 88),
    # 300 cells along x: float64 row buffers share storage (fused x-y pass,
    # reflective ends); with an inflow side float64 takes the march and
    # float32 the unshared rows
    ((300, 5, 3), ((R_, R_), (P_, P_), (T_, T_)), 90),
    ((300, 3, 2), ((I_, T_), (P_, P_), (P_, P_)), 91),
]


def _setup(n, bc, seed):
    P = wl.random_smooth_nf(n=n, seed=seed, bc=bc, nf=3)
    spec = dict(P["spec"], inflow=_inflow3(seed))
    g = oracle.make_grid(spec)
    return P, spec, g, oracle.prim_to_cons(g, P["w"])


@pytest.mark.parametrize("n,bc,seed", CASES)
def test_rhs_and_step_match_oracle(n, bc, seed):
    print(f"case n={n} bc={bc} seed={seed}", flush=True)
    P, spec, g, q0 = _setup(n, bc, seed)
    s = gpu_solver(spec, q0=q0)
    r = s.rhs().cpu().numpy()
    assert r.shape[0] == 9
    r_ref = oracle.rhs(g, q0)
    err, errp = fp64_rhs_errors(r, r_ref, q0, spec)
    _report(f"3-fluid rhs {n}", err)
    _report(f"3-fluid rhs {n} (physical-flux scale)", errp)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)
    if not any(k > 1 for k in n):
        return
    dt = s.rk3_step(sync=True)
    assert dt == pytest.approx(oracle.cfl_dt(g, q0), rel=1e-15)
    q = s.get_state().cpu().numpy()
    cells = sample_cells(spec, 300, seed=seed, q0=q0)
    ref = oracle_step_at(spec, q0, cells, dt)
    err = rel_linf(q.reshape(9, -1)[:, cells], ref)
    _report(f"3-fluid step {n}", err)
    assert np.all(err <= TOL), err
    s32 = gpu_solver(spec, q0=q0, precision=MFX_FP32_MIXED)
    err32 = rhs_rel_linf(s32.rhs().cpu().numpy(), r_ref, q0, spec)
    _report(f"3-fluid float rhs {n}", err32)
    assert np.all(err32 <= 1e-5), err32


@pytest.mark.parametrize("order,weights", [(3, MFX_WENO5_JS), (5, MFX_WENO5_Z)])
def test_other_schemes_match_oracle(order, weights):
    P, spec, g, q0 = _setup((37, 29, 23), ((T_, T_), (P_, P_), (R_, R_)), 89)
    spec = dict(spec, weno_order=order, weno_z=weights == MFX_WENO5_Z)
    g = oracle.make_grid(spec)
    s = gpu_solver(spec, q0=q0, weights=weights)
    err, errp = fp64_rhs_errors(s.rhs().cpu().numpy(), oracle.rhs(g, q0), q0, spec)
    _report(f"3-fluid order {order} weights {weights}", err)
    assert np.all(err <= TOL) and np.all(errp <= TOL), (err, errp)


def test_full_size_droplet_and_bubble_rhs_sampled():
    """256^3 droplet and bubble workload (three fluids): the GPU right-hand
    side, in the benchmark's launch configuration, on sampled cells.

    The physical-flux bar applies to every field whose physical flux is not
    negligible beside its wave-speed term.  The helium partial density is
    not such a field: the helium sits at rest in its bubble, so its
    physical-flux scale (about 0.04) is some 1e-7 of its flux scale (about
    2e5), while the HLLC wave-speed terms of its right-hand side, which the
    flux scale bounds, are rounded like any other."""
    P = wl.droplet_bubble(n=256, seed=0)
    g = oracle.make_grid(P["spec"])
    q0 = oracle.prim_to_cons(g, P["w"])
    del P["w"]
    s = gpu_solver(P["spec"], q0=q0)
    r = s.rhs().cpu().numpy().reshape(9, -1)
    s.destroy()
    cells = sample_cells(P["spec"], 3000, seed=4, q0=q0)
    ref = oracle.rhs_at(g, q0, cells).T
    err, errp = fp64_rhs_errors(r[:, cells], ref, q0, P["spec"])
    _report(f"3-fluid rhs 256^3 on {cells.size} cells", err)
    _report(f"3-fluid rhs 256^3 on {cells.size} cells (physical-flux scale)", errp)
    moving = physical_flux_scale(q0, P["spec"]) >= 1e-6 * flux_scale(q0, P["spec"])
    assert moving.sum() == 8 and not moving[2]  # all but the helium partial density
    assert np.all(err <= TOL) and np.all(errp[moving] <= TOL), (err, errp)


def test_droplet_and_bubble_run_matches_oracle():
    """Three fluids (water droplet and helium bubble in air, Mach-2 shock),
    6 CFL steps on a 48 x 40 x 36 grid against the oracle's run."""
    P = wl.droplet_bubble(n=(48, 40, 36), seed=1)
    g = oracle.make_grid(P["spec"])
    q0 = oracle.prim_to_cons(g, P["w"])
    s = gpu_solver(P["spec"], w0=P["w"])
    assert np.all(rel_linf(s.get_state().cpu().numpy(), q0) <= 1e-15)  # the GPU's own conversion
    for _ in range(6):
        s.rk3_step()
    q = s.get_state().cpu().numpy()
    q_ref, _ = oracle.run(g, q0, 6)
    err = rel_linf(q, q_ref)
    _report("droplet + bubble 48x40x36 x6", err)
    assert np.all(err <= TOL), err
    st = s.stats()
    assert st["error"] == 0 and st["step"] == 6


def test_absent_fluid_matches_the_two_fluid_path():
    """A three-fluid state whose middle fluid is absent (alpha = 0,
    alpha rho = 0) evolves as the two-fluid state of the other two fluids:
    the three-fluid kernels against the two-fluid kernels over 4 steps."""
    P2 = wl.shock_droplet(n=(40, 32, 24), seed=2)
    w2 = P2["w"]
    z = np.zeros_like(w2[0])
    w3 = np.stack([w2[0], z, w2[1], w2[2], w2[3], w2[4], w2[5], w2[6], z])
    s3 = dict(P2["spec"], gamma=(wl.WATER[0], wl.HELIUM[0], wl.AIR[0]), pinf=(wl.WATER[1], wl.HELIUM[1], wl.AIR[1]))
    a = gpu_solver(P2["spec"], w0=w2)
    b = gpu_solver(s3, w0=w3)
    for _ in range(4):
        dta = a.rk3_step(sync=True)
        dtb = b.rk3_step(sync=True)
        assert dta == dtb
    qa = a.get_state().cpu().numpy()
    qb = b.get_state().cpu().numpy()
    assert not qb[1].any() and not qb[8].any()
    err = rel_linf(np.stack([qb[0], qb[2], qb[3], qb[4], qb[5], qb[6], qb[7]]), qa)
    _report("absent fluid: three-fluid kernels vs two-fluid kernels", err)
    assert np.all(err <= 1e-13), err
