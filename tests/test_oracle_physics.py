"""Pins for the oracle's discretisation as a whole.

  - the 1000-cell water|air shock tube against the exact two-material
    Riemann solution (error falls with resolution; star state recovered);
  - conservation of the five conserved fields on periodic grids;
  - preservation of uniform pressure and velocity across a material
    interface (the reason for reconstructing primitives with the
    alpha*div(u) source built from the HLLC face velocity);
  - a uniform volume fraction stays uniform in a compressing flow (pins the
    sign and form of the alpha*div(u) source);
  - the same 1D problem along x, y and z gives bitwise-equal results;
  - a periodic shift of the input shifts the output, bitwise;
  - the cell-by-cell RHS equals the whole-grid RHS, bitwise.
"""
import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
from paper_2409_10729_amd import workloads as wl


def _setup(P):
    g = oracle.make_grid(P["spec"])
    return g, oracle.prim_to_cons(g, P["w"])


@pytest.fixture(scope="module")
def c1_run():
    P = wl.shock_tube()
    g, q0 = _setup(P)
    q, dts = oracle.run(g, q0, 300)
    return P, g, q, dts


def test_shock_tube_time_step_and_time(c1_run):
    """First CFL step and final time of the 300-step run: dt0 = CFL dx / (c_water
    of the 1e9 Pa state), which the exact sound speed fixes."""
    P, g, q, dts = c1_run
    c_w = np.sqrt(4.4 * (1e9 + 6e8) / 1000.0)
    # the left cells are 1e-6 air; their mixture sound speed is within 1e-5 of pure water
    assert dts[0] == pytest.approx(0.4 * 1e-3 / c_w, rel=1e-5)
    assert dts.sum() == pytest.approx(4.52e-5, rel=0.01)


def _errors(n, t_end):
    P = wl.shock_tube(n=n)
    g, q0 = _setup(P)
    nsteps = int(round(300 * n / 1000))
    q, _ = oracle.run(g, q0, nsteps, dts=np.full(nsteps, t_end / nsteps))
    w = oracle.cons_to_prim(g, q).reshape(7, n)
    x = (np.arange(n) + 0.5) / n
    L = er.Side(1000.0, 0.0, 1e9, 4.4, 6e8)
    R = er.Side(50.0, 0.0, 1e5, 1.4, 0.0)
    rho_e, u_e, p_e, _ = er.sample(L, R, (x - 0.5) / t_end)
    rho = w[0] + w[1]
    return (np.abs(rho - rho_e).mean() / np.abs(rho_e).mean(),
            np.abs(w[2] - u_e).mean() / np.abs(u_e).max(),
            np.abs(w[5] - p_e).mean() / np.abs(p_e).mean())


def test_shock_tube_converges_to_exact(c1_run):
    t_end = c1_run[3].sum()
    e = np.array([_errors(n, t_end) for n in (250, 500, 1000)])
    assert np.all(e[-1] < 0.01), e
    assert np.all(e[1:] < e[:-1]), e
    order = np.log2(e[0] / e[2]) / 2
    assert np.all(order > 0.5), order


def test_shock_tube_star_state(c1_run):
    P, g, q, dts = c1_run
    w = oracle.cons_to_prim(g, q).reshape(7, -1)
    x = (np.arange(1000) + 0.5) / 1000
    W = er.wave_speeds(er.Side(1000.0, 0.0, 1e9, 4.4, 6e8), er.Side(50.0, 0.0, 1e5, 1.4, 0.0))
    t = dts.sum()
    # water side of the star region, away from the tail of the fan and the contact
    lo = 0.5 + W["L"]["tail"] * t + 0.01
    hi = 0.5 + W["u"] * t - 0.005
    m = (x > lo) & (x < hi)
    assert m.sum() >= 20
    assert np.abs(w[5][m] / W["p"] - 1).max() < 0.05
    assert np.abs(w[2][m] / W["u"] - 1).max() < 0.02
    assert np.abs((w[0] + w[1])[m] / W["L"]["rho_star"] - 1).max() < 0.01


@pytest.mark.parametrize("seed", [0, 1])
def test_periodic_conservation(seed):
    P = wl.random_smooth(n=(16, 12, 10), seed=seed)
    g, q0 = _setup(P)
    q, _ = oracle.run(g, q0, 5)
    for v in range(6):
        s0 = q0[v].sum(dtype=np.float64)
        s1 = q[v].sum(dtype=np.float64)
        scale = np.abs(q0[v]).sum()
        assert abs(s1 - s0) <= 1e-13 * scale, (v, s0, s1)
    # alpha1 is not a conserved quantity (it carries the alpha div(u) source)
    assert abs(q[6].sum() - q0[6].sum()) > 0


def test_interface_equilibrium():
    P = wl.advected_bubble(n=24, seed=3)
    g, q0 = _setup(P)
    q, _ = oracle.run(g, q0, 20)
    w = oracle.cons_to_prim(g, q)
    assert np.abs(w[5] / 1e5 - 1).max() < 1e-9
    for d, u0 in enumerate((1.0, 0.5, 0.25)):
        assert np.abs(w[2 + d] / u0 - 1).max() < 1e-9
    # the interface did move: alpha changed somewhere
    assert np.abs(q[6] - q0[6]).max() > 1e-8


def test_uniform_alpha_stays_uniform_under_compression():
    n = 64
    s = wl.spec((n, 1, 1), ((1, 1), (0, 0), (0, 0)))
    x = (np.arange(n) + 0.5) / n
    w = np.zeros((7, 1, 1, n))
    a1 = 0.3
    w[0] = a1 * 1000.0 * (1 + 0.1 * np.sin(2 * np.pi * x))
    w[1] = (1 - a1) * 1.2 * (1 + 0.2 * np.cos(2 * np.pi * x))
    w[2] = 40.0 * np.sin(2 * np.pi * x)
    w[5] = 1e5 * (1 + 5.0 * (x < 0.4))
    w[6] = a1
    g = oracle.make_grid(s)
    q0 = oracle.prim_to_cons(g, w)
    q, _ = oracle.run(g, q0, 30)
    assert np.abs(q[6] - a1).max() < 1e-13
    assert np.abs(q[2] - q0[2]).max() > 1.0  # the flow did something


def test_direction_symmetry():
    P = wl.shock_tube(n=64)
    w1 = P["w"].reshape(7, 64)
    outs = []
    for d in range(3):
        n = [1, 1, 1]
        n[d] = 64
        bc = [(0, 0)] * 3
        bc[d] = (1, 1)
        s = wl.spec(n, bc)
        w = np.zeros((7, n[2], n[1], n[0]))
        for v in range(7):
            w[v] = w1[v].reshape(n[2], n[1], n[0])
        if d != 0:
            w[[2, 2 + d]] = w[[2 + d, 2]]
        g = oracle.make_grid(s)
        q, dts = oracle.run(g, oracle.prim_to_cons(g, w), 20)
        q = q.reshape(7, 64).copy()
        if d != 0:
            q[[2, 2 + d]] = q[[2 + d, 2]]
        outs.append((q, dts))
    for q, dts in outs[1:]:
        assert np.array_equal(q, outs[0][0])
        assert np.array_equal(dts, outs[0][1])


def test_translation_invariance():
    P = wl.random_smooth(n=(12, 10, 8), seed=5)
    g, q0 = _setup(P)
    r0 = oracle.rhs(g, q0)
    for axis, k in ((3, 5), (2, 3), (1, 2)):
        r1 = oracle.rhs(g, np.roll(q0, k, axis=axis))
        assert np.array_equal(r1, np.roll(r0, k, axis=axis))


@pytest.mark.parametrize("bc", [((1, 1), (0, 0), (1, 0)), ((0, 0), (1, 1), (0, 0))])
def test_rhs_at_equals_rhs(bc):
    P = wl.random_smooth(n=(9, 7, 11), seed=2, bc=bc)
    g, q0 = _setup(P)
    r = oracle.rhs(g, q0)
    cells = np.arange(9 * 7 * 11)
    ra = oracle.rhs_at(g, q0, cells)
    assert np.array_equal(ra.T.reshape(r.shape), r)


def test_mirror_symmetry():
    """Reflecting x (and the x velocity) reflects the result (up to rounding)."""
    P = wl.random_smooth(n=(16, 6, 6), seed=7, bc=((1, 1), (0, 0), (0, 0)))
    g, q0 = _setup(P)
    q1, _ = oracle.run(g, q0, 3, dts=np.full(3, 1e-6))
    qm = q0[:, :, :, ::-1].copy()
    qm[2] *= -1
    q2, _ = oracle.run(g, qm, 3, dts=np.full(3, 1e-6))
    q2 = q2[:, :, :, ::-1].copy()
    q2[2] *= -1
    for v in range(7):
        assert np.abs(q2[v] - q1[v]).max() <= 1e-12 * np.abs(q1[v]).max()


def test_single_fluid_limit_is_euler():
    """alpha1 = 1 everywhere: a pure stiffened-gas Euler problem.  A Sod-like
    water tube checked against the exact single-material solution."""
    n = 400
    s = wl.spec((n, 1, 1), ((1, 1), (0, 0), (0, 0)))
    x = (np.arange(n) + 0.5) / n
    w = np.zeros((7, 1, 1, n))
    left = x < 0.5
    w[0] = np.where(left, 1000.0, 990.0)
    w[5] = np.where(left, 5e8, 1e5)
    w[6] = 1.0
    g = oracle.make_grid(s)
    q, dts = oracle.run(g, oracle.prim_to_cons(g, w), 100)
    wq = oracle.cons_to_prim(g, q).reshape(7, n)
    t = dts.sum()
    re, ue, pe, _ = er.sample(er.Side(1000.0, 0, 5e8, 4.4, 6e8), er.Side(990.0, 0, 1e5, 4.4, 6e8), (x - 0.5) / t)
    assert np.abs(wq[0] - re).mean() / re.mean() < 2e-3
    assert np.abs(wq[5] - pe).mean() / pe.mean() < 2e-2
    assert np.abs(wq[2] - ue).mean() / np.abs(ue).max() < 2e-2
