"""Pins for the oracle's building blocks: EOS, WENO5, HLLC, SSP-RK3.

Each check compares the oracle with something other than its own formula:
closed forms (polynomial exactness, the Jiang-Shu indicator as an integral of
the stencil polynomial's derivatives, the SSP-RK3 stability polynomial),
textbook special cases (pure-fluid sound speed, isolated contacts, supersonic
upwinding) or invariants (round trips, rotations).
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import workloads as wl

G = oracle.make_grid(wl.spec((1, 1, 1), ((0, 0),) * 3))  # one cell: per-cell conversions


def _w(a1=0.3, rho1=1000.0, rho2=1.2, u=(10.0, -3.0, 2.0), p=2e5):
    return np.array([a1 * rho1, (1 - a1) * rho2, u[0], u[1], u[2], p, a1], dtype=np.float64)


# ---------------------------------------------------------------- EOS

@pytest.mark.parametrize("a1", [1e-6, 0.3, 0.5, 1 - 1e-6])
def test_prim_cons_round_trip(a1):
    w = _w(a1=a1)
    q = np.empty(7)
    w2 = np.empty(7)
    lib = oracle.lib()
    import ctypes
    lib.orc_prim_to_cons_cell(ctypes.byref(G), oracle._dp(w), oracle._dp(q))
    lib.orc_cons_to_prim_cell(ctypes.byref(G), oracle._dp(q), oracle._dp(w2))
    np.testing.assert_allclose(w2, w, rtol=1e-9)  # p loses digits to pi_inf cancellation
    np.testing.assert_allclose(w2[[0, 1, 6]], w[[0, 1, 6]], rtol=0, atol=0)


@pytest.mark.parametrize("fluid", [0, 1])
def test_pure_fluid_sound_speed(fluid):
    """With alpha1 in {0,1} the mixture sound speed is sqrt(gamma (p + pi_inf) / rho)."""
    gam = (4.4, 1.4)[fluid]
    pinf = (6e8, 0.0)[fluid]
    a1 = 1.0 if fluid == 0 else 0.0
    rho = 900.0 if fluid == 0 else 2.0
    w = np.array([a1 * rho, (1 - a1) * rho, 0, 0, 0, 3e5, a1], dtype=np.float64)
    c = oracle.sound_speed(G, w)
    assert c == pytest.approx(np.sqrt(gam * (3e5 + pinf) / rho), rel=1e-14)


def test_energy_of_pure_fluid_matches_stiffened_gas():
    """rho E = (p + gamma pi)/(gamma - 1) + kinetic energy for a pure fluid (Sec. II-A)."""
    w = np.array([1000.0, 0.0, 3.0, 4.0, 0.0, 1e6, 1.0])
    q = oracle.prim_to_cons(G, w.reshape(7, 1, 1, 1)).ravel()
    expect = (1e6 + 4.4 * 6e8) / 3.4 + 0.5 * 1000.0 * 25.0
    assert q[5] == pytest.approx(expect, rel=1e-15)


# ---------------------------------------------------------------- WENO5

def _cell_avgs(coeffs, h, centres):
    """Exact cell averages of the polynomial sum c_k x^k over [x-h/2, x+h/2]."""
    P = np.polynomial.Polynomial(coeffs).integ()
    return np.array([(P(x + h / 2) - P(x - h / 2)) / h for x in centres])


@pytest.mark.parametrize("seed", range(5))
def test_weno_exact_for_quadratics(seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-2, 2, size=3)
    h = 0.1
    xs = np.arange(-2, 3) * h
    v = _cell_avgs(c, h, xs)
    left, right = oracle.weno5(v)
    P = np.polynomial.Polynomial(c)
    assert right == pytest.approx(P(h / 2), rel=1e-13, abs=1e-13)
    assert left == pytest.approx(P(-h / 2), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_weno_linear_weights_exact_for_quartics(seed):
    """With epsilon >> beta the weights are the linear ones, and the 5-cell
    reconstruction is exact for polynomials of degree 4 (pins d_k and which
    weight goes with which stencil and edge)."""
    rng = np.random.default_rng(100 + seed)
    c = rng.uniform(-2, 2, size=5)
    h = 0.1
    v = _cell_avgs(c, h, np.arange(-2, 3) * h)
    left, right = oracle.weno5(v, eps=1e30)
    P = np.polynomial.Polynomial(c)
    assert right == pytest.approx(P(h / 2), rel=1e-12, abs=1e-13)
    assert left == pytest.approx(P(-h / 2), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_weno_betas_are_derivative_integrals(seed):
    """beta_k = sum_{l=1,2} h^(2l-1) * integral over the cell of (d^l p_k/dx^l)^2,
    with p_k the quadratic whose cell averages match stencil k (Jiang & Shu
    1996).  p_k is built here by solving the 3x3 cell-average system."""
    rng = np.random.default_rng(200 + seed)
    h = rng.uniform(0.01, 1.0)
    v = rng.uniform(-3, 3, size=5)
    betas = oracle.weno5_betas(v)
    xs = np.arange(-2, 3) * h
    for k in range(3):
        idx = [k, k + 1, k + 2]
        # cell average of x^m over cell j
        A = np.array([[((xs[j] + h / 2) ** (m + 1) - (xs[j] - h / 2) ** (m + 1)) / ((m + 1) * h)
                       for m in range(3)] for j in idx])
        coef = np.linalg.solve(A, v[idx])
        P = np.polynomial.Polynomial(coef)
        d1, d2 = P.deriv(1), P.deriv(2)
        I1 = (d1 * d1).integ()
        I2 = (d2 * d2).integ()
        expect = h * (I1(h / 2) - I1(-h / 2)) + h ** 3 * (I2(h / 2) - I2(-h / 2))
        assert betas[k] == pytest.approx(expect, rel=1e-9, abs=1e-12)


def test_weno_constant_and_mirror():
    l, r = oracle.weno5([7.0] * 5)
    assert l == pytest.approx(7.0, rel=1e-15) and r == pytest.approx(7.0, rel=1e-15)
    rng = np.random.default_rng(3)
    for _ in range(20):
        v = rng.uniform(-1, 1, size=5)
        l, r = oracle.weno5(v)
        l2, r2 = oracle.weno5(v[::-1])
        assert l2 == pytest.approx(r, rel=1e-13, abs=1e-15)
        assert r2 == pytest.approx(l, rel=1e-13, abs=1e-15)


def test_weno_fifth_order_on_smooth_data():
    """Smooth data away from critical points: error ~ h^5."""
    f = np.polynomial.Polynomial([0.3, 1.0, -0.7, 0.4, 0.9, -0.5, 0.2])  # degree 6, f' != 0 near x0
    x0 = 0.37
    errs = []
    hs = [0.04, 0.02, 0.01, 0.005]
    F = f.integ()
    for h in hs:
        xs = x0 + np.arange(-2, 3) * h
        v = np.array([(F(x + h / 2) - F(x - h / 2)) / h for x in xs])
        l, r = oracle.weno5(v, eps=1e-40)
        errs.append(abs(r - f(x0 + h / 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.5), orders


def test_weno_essentially_non_oscillatory_at_step():
    for v in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 0, 0, 0], [0, 0, 0, 0, 1]):
        l, r = oracle.weno5(np.array(v, dtype=float) * 1e9)
        for x in (l, r):
            assert -1e9 * 1e-6 <= x <= 1e9 * (1 + 1e-6)


# ---------------------------------------------------------------- WENO3 (Jiang-Shu weights)

@pytest.mark.parametrize("seed", range(3))
def test_weno3_exact_for_linear_data(seed):
    """Each candidate reproduces linear data, so any convex weights do:
    cell averages a, a+s, a+2s have edge values a+s/2 and a+3s/2."""
    rng = np.random.default_rng(seed)
    for _ in range(10):
        a, sl = rng.uniform(-5, 5, size=2)
        l, r = oracle.weno3([a, a + sl, a + 2 * sl])
        assert l == pytest.approx(a + sl / 2, rel=1e-13, abs=1e-13)
        assert r == pytest.approx(a + 1.5 * sl, rel=1e-13, abs=1e-13)


def test_weno3_linear_weights_reproduce_a_symmetric_quadratic():
    """With equal indicators the weights are the linear ones (1/3, 2/3), and
    the reconstruction is the third-order one: exact for the point values of
    a parabola from its cell averages.  Cell averages of x^2 over unit cells
    centred on -1, 0, 1 are (13/12, 1/12, 13/12); x^2 at +-1/2 is 1/4."""
    l, r = oracle.weno3([13.0 / 12.0, 1.0 / 12.0, 13.0 / 12.0], eps=1e-6)
    assert l == pytest.approx(0.25, rel=1e-14) and r == pytest.approx(0.25, rel=1e-14)
    # scaled and shifted: a x^2 + c
    l, r = oracle.weno3([3 * 13 / 12 + 2, 3 / 12 + 2, 3 * 13 / 12 + 2], eps=1e-6)
    assert l == pytest.approx(0.75 + 2, rel=1e-14) and r == pytest.approx(0.75 + 2, rel=1e-14)


def test_weno3_constant_and_mirror():
    l, r = oracle.weno3([7.0] * 3)
    assert l == pytest.approx(7.0, rel=1e-15) and r == pytest.approx(7.0, rel=1e-15)
    rng = np.random.default_rng(4)
    for _ in range(20):
        v = rng.uniform(-1, 1, size=3)
        l, r = oracle.weno3(v)
        l2, r2 = oracle.weno3(v[::-1])
        assert l2 == r and r2 == l


def test_weno3_third_order_on_smooth_data():
    """Smooth data away from critical points, indicators far above eps:
    error ~ h^3 (the candidates are second order; the weights recover the
    third-order combination)."""
    f = np.polynomial.Polynomial([0.3, 1.0, -0.7, 0.4, 0.9, -0.5, 0.2])
    F = f.integ()
    x0 = 0.37
    errs = []
    for h in [0.04, 0.02, 0.01, 0.005]:
        xs = x0 + np.arange(-1, 2) * h
        v = np.array([(F(x + h / 2) - F(x - h / 2)) / h for x in xs])
        l, r = oracle.weno3(v, eps=1e-40)
        errs.append(abs(r - f(x0 + h / 2)) + abs(l - f(x0 - h / 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 2.7), orders


def test_weno3_essentially_non_oscillatory_at_step():
    """A jump on one side: the smooth stencil takes (almost) all the weight."""
    for v, (lo, hi) in (([0, 0, 1], (0, 0)), ([1, 1, 0], (1, 1)), ([0, 1, 1], (1, 1)), ([1, 0, 0], (0, 0))):
        l, r = oracle.weno3(np.array(v, dtype=float) * 1e9)
        expect_r = (lo if v[2] != v[1] else v[1]) * 1e9
        expect_l = (v[1] if v[0] != v[1] else v[1]) * 1e9
        assert r == pytest.approx(expect_r, abs=1e9 * 1e-6)
        assert l == pytest.approx(expect_l, abs=1e9 * 1e-6)
        for x in (l, r):
            assert -1e9 * 1e-6 <= x <= 1e9 * (1 + 1e-6)


def test_weno3_rhs_differs_from_weno5_and_matches_per_cell_path():
    P = wl.random_smooth(n=(20, 12, 8), seed=2)
    spec3 = dict(P["spec"], weno_order=3)
    g3, g5 = oracle.make_grid(spec3), oracle.make_grid(P["spec"])
    q = oracle.prim_to_cons(g5, P["w"])
    r3, r5 = oracle.rhs(g3, q), oracle.rhs(g5, q)
    assert not np.allclose(r3, r5, rtol=1e-6, atol=0)
    cells = np.arange(0, 20 * 12 * 8, 37, dtype=np.int64)
    at = oracle.rhs_at(g3, q, cells)
    assert np.array_equal(at, r3.reshape(7, -1)[:, cells].T)


# ---------------------------------------------------------------- WENO-Z (comparison form)

@pytest.mark.parametrize("seed", range(3))
def test_weno_z_exact_for_quadratics_and_quartics_with_linear_weights(seed):
    rng = np.random.default_rng(300 + seed)
    h = 0.1
    xs = np.arange(-2, 3) * h
    c = rng.uniform(-2, 2, size=3)
    l, r = oracle.weno5_z(_cell_avgs(c, h, xs))
    P = np.polynomial.Polynomial(c)
    assert r == pytest.approx(P(h / 2), rel=1e-13, abs=1e-13)
    assert l == pytest.approx(P(-h / 2), rel=1e-13, abs=1e-13)
    # tau5 = 0 (symmetric beta0 = beta2) makes the weights linear: quartics even in x exact
    c4 = np.array([rng.uniform(-2, 2), 0.0, rng.uniform(-2, 2), 0.0, rng.uniform(-2, 2)])
    l, r = oracle.weno5_z(_cell_avgs(c4, h, xs))
    P4 = np.polynomial.Polynomial(c4)
    assert r == pytest.approx(P4(h / 2), rel=1e-12, abs=1e-13)
    assert l == pytest.approx(P4(-h / 2), rel=1e-12, abs=1e-13)


def test_weno_z_keeps_fifth_order_at_a_critical_point():
    """At a first-order critical point (vanishing first derivative) WENO-Z
    keeps fifth order and its weights stay closer to the linear ones than
    the Jiang-Shu weights, so its error is the smaller (Borges et al. 2008)."""
    f = np.polynomial.Polynomial([0.2, 0.0, 1.0, 0.8, -0.6, 0.3])  # f'(0) = 0
    F = f.integ()
    eps = 1e-40
    err = {"z": [], "js": []}
    for h in (0.04, 0.02, 0.01, 0.005):
        xs = np.arange(-2, 3) * h
        v = np.array([(F(x + h / 2) - F(x - h / 2)) / h for x in xs])
        err["z"].append(abs(oracle.weno5_z(v, eps=eps)[1] - f(h / 2)))
        err["js"].append(abs(oracle.weno5(v, eps=eps)[1] - f(h / 2)))
    oz = np.log2(np.array(err["z"][:-1]) / np.array(err["z"][1:]))
    oj = np.log2(np.array(err["js"][:-1]) / np.array(err["js"][1:]))
    print("orders at the critical point: WENO-Z", oz, "Jiang-Shu", oj)
    assert np.all(oz > 4.5), oz
    assert np.all(np.array(err["z"]) < np.array(err["js"]))


def test_weno_z_non_oscillatory_at_step_and_mirror():
    for v in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 0, 0, 0], [0, 0, 0, 0, 1]):
        l, r = oracle.weno5_z(np.array(v, dtype=float) * 1e9)
        for x in (l, r):
            assert -1e9 * 1e-6 <= x <= 1e9 * (1 + 1e-6)
    rng = np.random.default_rng(9)
    for _ in range(20):
        v = rng.uniform(-1, 1, size=5)
        l, r = oracle.weno5_z(v)
        l2, r2 = oracle.weno5_z(v[::-1])
        assert l2 == pytest.approx(r, rel=1e-13, abs=1e-15)
        assert r2 == pytest.approx(l, rel=1e-13, abs=1e-15)


# ---------------------------------------------------------------- HLLC

def _phys_flux(w, d):
    """Flux of the five-equation model along direction d (Sec. II-A)."""
    q = oracle.prim_to_cons(G, w.reshape(7, 1, 1, 1)).ravel()
    un = w[2 + d]
    F = q * un
    F[2 + d] += w[5]
    F[5] = (q[5] + w[5]) * un
    return F


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_consistency(d):
    rng = np.random.default_rng(d)
    for _ in range(10):
        w = _w(a1=rng.uniform(0, 1), u=rng.uniform(-300, 300, 3), p=rng.uniform(1e4, 1e9))
        F, uf = oracle.hllc(G, w, w, d)
        np.testing.assert_allclose(F, _phys_flux(w, d), rtol=1e-12, atol=1e-9 * np.abs(F).max())
        assert uf == pytest.approx(w[2 + d], rel=1e-12, abs=1e-12)


def test_hllc_supersonic_upwinding():
    wl = _w(a1=1e-6, rho2=1.2, u=(2000.0, 5.0, 0.0), p=1e5)
    wr = _w(a1=1e-6, rho2=3.0, u=(1500.0, -5.0, 1.0), p=3e5)
    F, uf = oracle.hllc(G, wl, wr, 0)
    np.testing.assert_allclose(F, _phys_flux(wl, 0), rtol=1e-13)
    assert uf == pytest.approx(wl[2], rel=1e-14)
    wl2 = _w(a1=1e-6, u=(-1500.0, 0, 0))
    wr2 = _w(a1=1e-6, u=(-2000.0, 0, 0), p=1.5e5)
    F, uf = oracle.hllc(G, wl2, wr2, 0)
    np.testing.assert_allclose(F, _phys_flux(wr2, 0), rtol=1e-13)
    assert uf == pytest.approx(wr2[2], rel=1e-14)


@pytest.mark.parametrize("U", [0.0, 35.0, -20.0])
def test_hllc_resolves_isolated_contact(U):
    """Equal pressure and normal velocity on both sides of a material
    interface: the HLLC flux is the upwind physical flux (a contact moving at
    U), and the face velocity is exactly U."""
    wl = _w(a1=1 - 1e-6, u=(U, 1.0, -2.0), p=1e5)
    wr = _w(a1=1e-6, u=(U, 4.0, 3.0), p=1e5)
    F, uf = oracle.hllc(G, wl, wr, 0)
    up = wl if U >= 0 else wr
    np.testing.assert_allclose(F, _phys_flux(up, 0), rtol=1e-12, atol=1e-6)
    assert uf == pytest.approx(U, abs=1e-9)
    if U == 0.0:
        assert F[0] == 0.0 and F[1] == 0.0 and F[6] == 0.0 and F[5] == 0.0
        assert F[2] == pytest.approx(1e5, rel=1e-14)


def test_hllc_rotation():
    rng = np.random.default_rng(11)
    wl = _w(a1=0.2, u=rng.uniform(-100, 100, 3), p=3e5)
    wr = _w(a1=0.7, rho1=990.0, u=rng.uniform(-100, 100, 3), p=1e5)
    Fx, ux = oracle.hllc(G, wl, wr, 0)
    for d in (1, 2):
        perm = [2, 3, 4]
        perm[0], perm[d] = perm[d], perm[0]
        wl2, wr2 = wl.copy(), wr.copy()
        wl2[[2, 3, 4]] = wl[perm]
        wr2[[2, 3, 4]] = wr[perm]
        Fd, ud = oracle.hllc(G, wl2, wr2, d)
        Fd_back = Fd.copy()
        Fd_back[[2, 3, 4]] = Fd[perm]
        np.testing.assert_allclose(Fd_back, Fx, rtol=1e-13, atol=1e-9)
        assert ud == pytest.approx(ux, rel=1e-14)


def test_hllc_star_velocity_in_subsonic_case():
    """In a star region the face velocity equals xi_K * S*, and the mass flux
    of each phase equals alpha_i rho_i of the upwind side times the face
    velocity (the alpha-consistency that keeps uniform alpha constant)."""
    wl = _w(a1=0.4, u=(30.0, 0, 0), p=5e6)
    wr = _w(a1=0.4, u=(-10.0, 0, 0), p=1e5)
    F, uf = oracle.hllc(G, wl, wr, 0)
    assert F[6] == pytest.approx(0.4 * uf, rel=1e-13)


# ---------------------------------------------------------------- SSP-RK3

@pytest.mark.parametrize("z", [-0.1, -0.5, -1.2, 0.3, -2.5])
def test_rk3_stability_polynomial(z):
    """For dq/dt = lambda q, one SSP-RK3 step multiplies q by 1 + z + z^2/2 + z^3/6."""
    lam, dt = z / 0.7, 0.7
    q = np.array([1.0, -2.0, 3.5])
    q1 = oracle.rk3_combine(1, q, q, lam * q, dt)
    q2 = oracle.rk3_combine(2, q, q1, lam * q1, dt)
    q3 = oracle.rk3_combine(3, q, q2, lam * q2, dt)
    np.testing.assert_allclose(q3, q * (1 + z + z * z / 2 + z ** 3 / 6), rtol=1e-14)


def test_wrappers_reject_a_state_of_another_shape():
    """The oracle's C routines index the whole grid: a state array of any
    other shape is refused before the call instead of read or written past
    its end."""
    spec = wl.random_smooth(n=(6, 5, 4), seed=3, bc=((1, 1), (0, 0), (0, 0)))["spec"]
    g = oracle.make_grid(spec)
    small = np.ones((7, 1, 1, 1))
    for f in (oracle.prim_to_cons, oracle.cons_to_prim, oracle.rhs, oracle.cfl_dt, oracle.rk3_step):
        with pytest.raises(ValueError):
            f(g, small)
    with pytest.raises(ValueError):
        oracle.run(g, small, 1)
    q = np.ones((7, 4, 5, 6))
    with pytest.raises(ValueError):
        oracle.rhs_at(g, q, np.array([6 * 5 * 4]))
