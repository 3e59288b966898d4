"""Pins of the oracle on non-uniform cells (Sec. III-A: structured mesh with
local refinement by a hyperbolic tangent): WENO5 with Jiang-Shu weights on
cells of unequal widths, flux differences over each cell's width.

What fixes it without an implementation to compare with:
  * equal widths reproduce the uniform WENO5 (and the uniform right-hand
    side) to rounding;
  * the three candidates reproduce any quadratic from its cell averages on
    any widths, whatever the weights; with the weights at their ideal values
    (eps large) any quartic is reproduced: this fixes the ideal weights;
  * the indicators of a linear profile are (h s)^2 and of x^2 the closed form
    h int (2x)^2 + h^3 int 4 over the cell;
  * volume-weighted conservation on a periodic stretched grid; uniform
    pressure and velocity across an interface stay uniform; x-mirror
    symmetry on a symmetric stretching; fifth-order convergence of the
    reconstruction under refinement of a fixed stretching.
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import workloads as wl
from parity_util import flux_scale

RNG = np.random.default_rng(0)


def _averages(coef, edges):
    """Averages of the polynomial sum coef[m] x^m over the cells edges[i]..edges[i+1]."""
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        P = sum(c * (b ** (m + 1) - a ** (m + 1)) / (m + 1) for m, c in enumerate(coef))
        out.append(P / (b - a))
    return np.array(out)


def _random_cells():
    h = RNG.uniform(0.5, 2.0, size=5)
    edges = np.concatenate([[0.0], np.cumsum(h)]) - h[:2].sum() - 0.5 * h[2]
    return h, edges


def test_equal_widths_reproduce_uniform_weno5():
    for _ in range(50):
        v = RNG.normal(size=5) * RNG.uniform(0.01, 100)
        h = np.full(5, RNG.uniform(0.1, 10))
        a, b = oracle.weno5_nu(h, v), oracle.weno5(v)
        assert abs(a[0] - b[0]) <= 1e-13 * np.abs(v).max() and abs(a[1] - b[1]) <= 1e-13 * np.abs(v).max()


def test_quadratics_are_exact_on_any_widths():
    for _ in range(50):
        h, e = _random_cells()
        coef = RNG.normal(size=3)
        left, right = oracle.weno5_nu(h, _averages(coef, e))
        xl, xr = e[2], e[3]
        assert left == pytest.approx(np.polyval(coef[::-1], xl), abs=1e-11)
        assert right == pytest.approx(np.polyval(coef[::-1], xr), abs=1e-11)


def test_ideal_weights_reproduce_quartics():
    for _ in range(50):
        h, e = _random_cells()
        coef = RNG.normal(size=5)
        left, right = oracle.weno5_nu(h, _averages(coef, e), eps=1e30)
        assert left == pytest.approx(np.polyval(coef[::-1], e[2]), abs=1e-10)
        assert right == pytest.approx(np.polyval(coef[::-1], e[3]), abs=1e-10)
        dr, dl = oracle.ideal_weights_nu(h)
        assert dr.sum() == pytest.approx(1.0, abs=1e-14) and dl.sum() == pytest.approx(1.0, abs=1e-14)


def test_indicators_closed_forms():
    for _ in range(20):
        h, e = _random_cells()
        s = RNG.normal()
        b = oracle.weno5_nu_betas(h, _averages([0.3, s], e))
        np.testing.assert_allclose(b, (h[2] * s) ** 2, rtol=1e-11)
        b = oracle.weno5_nu_betas(h, _averages([0.0, 0.0, 1.0], e))
        xa, xb, hc = e[2], e[3], h[2]
        closed = hc * 4.0 * (xb ** 3 - xa ** 3) / 3.0 + hc ** 3 * 4.0 * hc
        np.testing.assert_allclose(b, closed, rtol=1e-11)


def _q0(P):
    g = oracle.make_grid(P["spec"])
    return g, oracle.prim_to_cons(g, P["w"])


def test_uniform_faces_give_the_uniform_rhs():
    P = wl.random_smooth(n=(24, 20, 16), seed=2, bc=((1, 1), (0, 0), (2, 2)))
    g, q = _q0(P)
    S = wl.stretched(P, [np.linspace(0, 1, 25), np.linspace(0, 1, 21), np.linspace(0, 1, 17)])
    r0, r1 = oracle.rhs(g, q), oracle.rhs(oracle.make_grid(S["spec"]), q)
    err = np.abs(r0 - r1).reshape(7, -1).max(axis=1) / flux_scale(q, P["spec"])
    assert np.all(err <= 1e-13), err


def test_volume_weighted_conservation_on_a_periodic_stretched_grid():
    P = wl.random_smooth(n=(24, 20, 16), seed=3)
    g0, q = _q0(P)
    f = [wl.tanh_faces(24, 0.4, 0.6, 10.0), wl.tanh_faces(20, 0.6, 0.5, 6.0), None]
    S = wl.stretched(P, f)
    r = oracle.rhs(oracle.make_grid(S["spec"]), q)
    hx, hy = np.diff(f[0]), np.diff(f[1])
    vol = hx[None, None, :] * hy[None, :, None] * (1.0 / 16)
    scale = flux_scale(q, P["spec"])
    for v in range(6):
        tot = (r[v] * vol).sum()
        assert abs(tot) <= 1e-14 * scale[v], v
    # and the widths matter: the unweighted sum does not vanish
    assert abs(r[0].sum()) > 1e-8 * scale[0]


def test_equilibrium_on_a_stretched_grid():
    n = 32
    spec = wl.spec((n, n, 1), ((0, 0), (0, 0), (0, 0)))
    f = wl.tanh_faces(n, 0.5, 0.7, 8.0)
    xc = 0.5 * (f[1:] + f[:-1])
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.45) ** 2)
    a1 = wl.ALPHA_EPS + (1 - 2 * wl.ALPHA_EPS) * 0.5 * (1 - np.tanh((r - 0.2) / 0.02))
    w = wl._pack(a1, 1000.0, 1.2, 3.0, -2.0, 0.0, 1.0e5).reshape(7, 1, n, n)
    S = dict(spec, faces=(f, f, None))
    g = oracle.make_grid(S)
    q, _ = oracle.run(g, oracle.prim_to_cons(g, w), 20)
    wp = oracle.cons_to_prim(g, q)
    assert np.abs(wp[5] / 1e5 - 1).max() <= 1e-9
    assert np.abs(wp[2] - 3.0).max() <= 1e-8 and np.abs(wp[3] + 2.0).max() <= 1e-8


def test_mirror_symmetry_on_a_symmetric_stretching():
    P = wl.random_smooth(n=(40, 6, 5), seed=7, bc=((1, 1), (0, 0), (0, 0)))
    f = wl.tanh_faces(40, 0.5, 0.6, 8.0)
    assert np.allclose(f, 1.0 - f[::-1], atol=1e-15)
    S = wl.stretched(P, [f, None, None])
    g = oracle.make_grid(S["spec"])
    q = oracle.prim_to_cons(g, P["w"])
    m = q[:, :, :, ::-1].copy()
    m[2] = -m[2]
    r = oracle.rhs(g, q)
    rm = oracle.rhs(g, m)[:, :, :, ::-1].copy()
    rm[2] = -rm[2]
    err = np.abs(rm - r).reshape(7, -1).max(axis=1) / flux_scale(q, P["spec"])
    assert np.all(err <= 1e-12), err


def test_fifth_order_under_refinement():
    """Face values of a smooth profile reconstructed from its exact cell
    averages on a refined tanh-stretched grid: the error falls at about
    fifth order."""
    errs = []
    for n in (40, 80, 160):
        f = wl.tanh_faces(n, 0.5, 0.6, 6.0)
        cellavg = (np.cos(2 * np.pi * f[:-1]) - np.cos(2 * np.pi * f[1:])) / (2 * np.pi * np.diff(f))
        e = 0.0
        for c in range(2, n - 2):
            left, right = oracle.weno5_nu(np.diff(f)[c - 2:c + 3], cellavg[c - 2:c + 3])
            e = max(e, abs(right - np.sin(2 * np.pi * f[c + 1])), abs(left - np.sin(2 * np.pi * f[c])))
        errs.append(e)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("errors", errs, "orders", order, flush=True)
    assert np.all(order >= 4.3)
