"""mfx_rhs_static (the right-hand side for callers that cannot allocate:
scratch in a static device array) against mfx_rhs on a context, through the
C ABI: two calls in a row on one GPU, the second on a smaller grid (the
array keeps the first call's contents), in float64 and in the float form,
with every boundary type, for two and for three fluids.  Same kernels and launch shapes, so the results
are bit for bit the same."""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import MFX_FP32_MIXED, MFX_FP64, MFX_WENO5_JS, MFX_WENO5_Z, rhs_static
from paper_2409_10729_amd import workloads as wl
from parity_util import gpu_solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P_, T_, R_, I_ = wl.PERIODIC, wl.TRANSMISSIVE, wl.REFLECTIVE, wl.INFLOW


def _inflow(seed):
    rng = np.random.default_rng(seed)
    g1 = oracle.make_grid(wl.spec((1, 1, 1), ((P_, P_),) * 3))
    out = np.zeros((3, 2, 7))
    for d in range(3):
        for s in range(2):
            a1 = rng.uniform(0.0, 0.3)
            w = np.array([a1 * 1000.0, (1 - a1) * 1.5, 20.0, -10.0, 5.0, 1.5e5, a1])
            out[d, s] = oracle.prim_to_cons(g1, w.reshape(7, 1, 1, 1)).reshape(7)
    return out


@pytest.mark.parametrize("precision,weights", [(MFX_FP64, MFX_WENO5_JS), (MFX_FP32_MIXED, MFX_WENO5_JS),
                                               (MFX_FP64, MFX_WENO5_Z)])
def test_static_rhs_equals_context_rhs(precision, weights):
    cases = [((96, 80, 72), ((T_, T_), (P_, P_), (P_, P_)), 1),      # larger first
             ((37, 29, 23), ((I_, R_), (T_, I_), (R_, T_)), 2)]      # then smaller, every boundary type
    for n, bc, seed in cases:
        print(f"static rhs: n={n} bc={bc} precision={precision} weights={weights}", flush=True)
        P = wl.random_smooth(n=n, seed=seed, bc=bc)
        spec = dict(P["spec"], inflow=_inflow(seed), weno_z=weights == MFX_WENO5_Z)
        g = oracle.make_grid(spec)
        q0 = oracle.prim_to_cons(g, P["w"])
        s = gpu_solver(spec, q0=q0, precision=precision, weights=weights)
        ref = s.rhs().cpu().numpy()
        qd = torch.from_numpy(q0).cuda()
        out = torch.full_like(qd, float("nan"))
        rhs_static(spec, qd, out, precision=precision, weights=weights)
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), np.abs(got - ref).max()


def _inflow3(seed):
    """Conserved three-fluid inflow states [3][2][9] of random valid primitives."""
    rng = np.random.default_rng(seed)
    g1 = oracle.make_grid(wl.spec_fluids((1, 1, 1), ((P_, P_),) * 3, 3))
    out = np.zeros((3, 2, 9))
    for d in range(3):
        for s in range(2):
            a = rng.dirichlet((1.0, 3.0, 1.0))
            w = np.array([a[0] * 1000.0, a[1] * 1.5, a[2] * 0.17, 20.0, -10.0, 5.0, 1.5e5, a[0], a[1]])
            out[d, s] = oracle.prim_to_cons(g1, w.reshape(9, 1, 1, 1)).reshape(9)
    return out


@pytest.mark.parametrize("precision", [MFX_FP64, MFX_FP32_MIXED])
def test_static_rhs_equals_context_rhs_three_fluids(precision):
    """Nine variables: the static scratch holds ten values per boundary face
    and nine partial right-hand-side fields."""
    cases = [((64, 48, 40), ((T_, T_), (P_, P_), (P_, P_)), 3),      # larger first
             ((37, 29, 23), ((I_, R_), (T_, I_), (R_, T_)), 4)]      # then smaller, every boundary type
    for n, bc, seed in cases:
        print(f"static rhs, three fluids: n={n} bc={bc} precision={precision}", flush=True)
        P = wl.random_smooth_nf(n=n, seed=seed, bc=bc, nf=3)
        spec = dict(P["spec"], inflow=_inflow3(seed))
        g = oracle.make_grid(spec)
        q0 = oracle.prim_to_cons(g, P["w"])
        s = gpu_solver(spec, q0=q0, precision=precision)
        ref = s.rhs().cpu().numpy()
        qd = torch.from_numpy(q0).cuda()
        out = torch.full_like(qd, float("nan"))
        rhs_static(spec, qd, out, precision=precision)
        got = out.cpu().numpy()
        assert got.shape[0] == 9
        assert np.array_equal(got, ref), np.abs(got - ref).max()
