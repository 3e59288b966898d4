"""Pins of the oracle's model with more than two fluids (Sec. II-A states
the two-component Allaire system with a continuity and a volume-fraction
equation per component; the same system for nf components, with mixture
rules linear in every volume fraction).

What fixes it without an implementation to compare with:
  * an absent fluid (alpha = 0, alpha rho = 0) changes nothing: the
    three-fluid right-hand side and steps equal the two-fluid ones of the
    remaining fluids bit for bit, and the absent fluid's variables stay 0;
  * relabelling two fluids permutes the result (to rounding of the mixture
    sums);
  * a pure fluid's sound speed is gamma (p + pi_inf) / rho, for each fluid;
  * conservation of every partial density, momentum and energy on a
    periodic grid; uniform pressure and velocity across three-fluid
    interfaces stay uniform (equilibrium);
  * the same 1D problem along x, y or z gives the same result.
"""
import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import workloads as wl


def _q0(P):
    g = oracle.make_grid(P["spec"])
    return g, oracle.prim_to_cons(g, P["w"])


def _absent_middle(P2):
    """Three-fluid copy of a two-fluid problem (fluids: its fluid 1, an
    absent helium fluid, its fluid 2)."""
    w2 = P2["w"]
    z = np.zeros_like(w2[0])
    w3 = np.stack([w2[0], z, w2[1], w2[2], w2[3], w2[4], w2[5], w2[6], z])
    s = dict(P2["spec"], gamma=(P2["spec"]["gamma"][0], wl.HELIUM[0], P2["spec"]["gamma"][1]),
             pinf=(P2["spec"]["pinf"][0], wl.HELIUM[1], P2["spec"]["pinf"][1]))
    if "inflow" in s:
        i2 = np.asarray(s["inflow"]).reshape(3, 2, 7)
        zi = np.zeros((3, 2, 1))
        s["inflow"] = np.concatenate([i2[..., :1], zi, i2[..., 1:], zi], axis=2)
    return dict(P2, spec=s, w=w3)


def _three_to_two(x3):
    return np.stack([x3[0], x3[2], x3[3], x3[4], x3[5], x3[6], x3[7]])


@pytest.mark.parametrize("maker", [lambda: wl.random_smooth(n=(20, 16, 12), seed=3, bc=((1, 1), (0, 0), (2, 2))),
                                   lambda: wl.shock_droplet(n=(24, 20, 16), seed=1),
                                   lambda: wl.shock_tube(n=200)])
def test_absent_fluid_reduces_to_two_fluids(maker):
    P2 = maker()
    P3 = _absent_middle(P2)
    g2, q2 = _q0(P2)
    g3, q3 = _q0(P3)
    assert np.array_equal(_three_to_two(q3), q2) and not q3[1].any() and not q3[8].any()
    r2, r3 = oracle.rhs(g2, q2), oracle.rhs(g3, q3)
    assert np.array_equal(_three_to_two(r3), r2)
    assert np.all(r3[1] == 0.0) and np.all(r3[8] == 0.0)
    a2, dt2 = oracle.run(g2, q2, 3)
    a3, dt3 = oracle.run(g3, q3, 3)
    assert np.array_equal(dt2, dt3) and np.array_equal(_three_to_two(a3), a2)


def test_relabelling_permutes_the_result():
    P = wl.random_smooth_nf(n=(20, 16, 12), seed=5, bc=((1, 1), (0, 0), (0, 0)))
    g, q = _q0(P)
    r = oracle.rhs(g, q)
    # swap fluids 1 and 2: partial densities 0 <-> 1, volume fractions 7 <-> 8
    perm = [1, 0, 2, 3, 4, 5, 6, 8, 7]
    s2 = dict(P["spec"], gamma=tuple(P["spec"]["gamma"][i] for i in (1, 0, 2)),
              pinf=tuple(P["spec"]["pinf"][i] for i in (1, 0, 2)))
    g2 = oracle.make_grid(s2)
    r2 = oracle.rhs(g2, np.ascontiguousarray(q[perm]))[np.argsort(perm)]
    scale = np.abs(r).reshape(9, -1).max(axis=1)
    assert np.all(np.abs(r2 - r).reshape(9, -1).max(axis=1) <= 1e-12 * scale)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_pure_fluid_sound_speed(k):
    spec = wl.spec_fluids((1, 1, 1), ((0, 0),) * 3, 3)
    g = oracle.make_grid(spec)
    rho, p = (1000.0, 1.2, 0.17)[k], 3.0e5
    w = np.zeros(9)
    w[k] = rho
    w[6] = p
    w[7], w[8] = (1.0 if k == 0 else 0.0), (1.0 if k == 1 else 0.0)
    gam, pinf = wl.FLUIDS[k]
    assert oracle.sound_speed(g, w) == pytest.approx(np.sqrt(gam * (p + pinf) / rho), rel=1e-14)


def test_conservation_on_a_periodic_grid():
    P = wl.random_smooth_nf(n=(20, 16, 12), seed=6)
    g, q = _q0(P)
    r = oracle.rhs(g, q).reshape(9, -1)
    q2 = oracle.rk3_step(g, q)[0].reshape(9, -1)
    qf = q.reshape(9, -1)
    for v in range(7):  # three partial densities, momentum, energy
        scale = np.abs(r[v]).max() * r.shape[1]
        assert abs(r[v].sum()) <= 1e-13 * scale, v
        assert abs(q2[v].sum() - qf[v].sum()) <= 1e-13 * np.abs(qf[v]).sum(), v


def test_equilibrium_across_three_fluid_interfaces():
    """A water droplet and a helium bubble in air, all moving at one
    velocity at one pressure: pressure and velocity stay uniform."""
    n = 32
    spec = wl.spec_fluids((n, n, n), ((0, 0),) * 3, 3)
    Z, Y, X = np.meshgrid(*[(np.arange(n) + 0.5) / n] * 3, indexing="ij")
    rw = np.sqrt((X - 0.35) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    rh = np.sqrt((X - 0.7) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    eps = wl.ALPHA_EPS
    aw = eps + (1 - 3 * eps) * 0.5 * (1 - np.tanh((rw - 0.2) / (1.5 / n)))
    ah = eps + (1 - 3 * eps) * 0.5 * (1 - np.tanh((rh - 0.15) / (1.5 / n)))
    aa = 1.0 - aw - ah
    u0 = (2.0, -1.0, 0.5)
    w = wl._pack_nf([aw, aa, ah], [1000.0, 1.2, 0.17], u0[0], u0[1], u0[2], 1.0e5)
    g = oracle.make_grid(spec)
    q, _ = oracle.run(g, oracle.prim_to_cons(g, w), 20)
    wp = oracle.cons_to_prim(g, q)
    assert np.abs(wp[6] / 1.0e5 - 1).max() <= 1e-9
    for d in range(3):
        assert np.abs(wp[3 + d] - u0[d]).max() <= 1e-9 * abs(u0[d]) * 50


def test_direction_symmetry():
    P = wl.random_smooth_nf(n=(40, 1, 1), seed=7, bc=((1, 1), (0, 0), (0, 0)))
    g, q = _q0(P)
    rx = oracle.rhs(g, q)
    for d in (1, 2):
        n = [1, 1, 1]
        n[d] = 40
        bc = [(0, 0)] * 3
        bc[d] = (1, 1)
        spec = dict(P["spec"], n=tuple(n), bc=tuple(bc), dx=(P["spec"]["dx"][0],) * 3)
        qd = np.moveaxis(q, 3, 3 - d).copy()
        qd[[3, 3 + d]] = qd[[3 + d, 3]]
        rd = oracle.rhs(oracle.make_grid(spec), qd)
        rd[[3, 3 + d]] = rd[[3 + d, 3]]
        assert np.array_equal(np.moveaxis(rd, 3 - d, 3), rx)


def test_four_fluids_run():
    P = wl.random_smooth_nf(n=(16, 12, 10), seed=8, nf=4)
    g, q = _q0(P)
    assert q.shape[0] == 11
    q1, _ = oracle.run(g, q, 2)
    assert np.all(np.isfinite(q1))


def test_uniform_volume_fractions_stay_uniform_under_compression():
    """alpha_i is advected (d alpha_i / dt + u . grad alpha_i = 0): with
    uniform volume fractions and a compressing velocity field every
    volume-fraction right-hand side vanishes (each needs its alpha_i div(u)
    source with the sign of the model), while the partial densities change."""
    n = 48
    spec = wl.spec_fluids((n, 1, 1), ((0, 0),) * 3, 3)
    x = (np.arange(n) + 0.5) / n
    u = 100.0 * np.sin(2 * np.pi * x)
    w = wl._pack_nf([np.full(n, 0.3), np.full(n, 0.5), np.full(n, 0.2)], [1000.0, 1.2, 0.17], u, 0.0, 0.0, 1.0e5)
    g = oracle.make_grid(spec)
    q = oracle.prim_to_cons(g, w.reshape(9, 1, 1, n))
    r = oracle.rhs(g, q).reshape(9, -1)
    scale = 0.5 * np.abs(np.diff(u)).max() * n
    assert np.abs(r[7]).max() <= 1e-12 * scale and np.abs(r[8]).max() <= 1e-12 * scale
    assert np.abs(r[0]).max() > 1.0
