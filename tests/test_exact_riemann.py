"""Pins for the exact two-material Riemann solver (oracle side).

The solver is checked against things other than itself: Toro's printed
star-region values (golden fixture), the Rankine-Hugoniot jump conditions
across each computed shock, the isentrope through each computed rarefaction,
the p -> p + pi_inf shift that maps a single stiffened gas onto an ideal gas,
and bisection against Newton.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.exact_riemann import Side, sample, star_state, wave_speeds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toro_exact_riemann.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_toro_table_values(case):
    L = Side(*case["left"], 1.4)
    R = Side(*case["right"], 1.4)
    p, u = star_state(L, R)
    # the table prints 5-6 significant digits
    assert p == pytest.approx(case["p_star"], rel=2e-5, abs=1e-5)
    assert u == pytest.approx(case["u_star"], rel=2e-5, abs=1e-5)


WATER_AIR = (Side(1000.0, 0.0, 1.0e9, 4.4, 6.0e8), Side(50.0, 0.0, 1.0e5, 1.4, 0.0))


@pytest.mark.parametrize("L,R", [WATER_AIR,
                                 (Side(1.2, 0.0, 1e5, 1.4), Side(1000.0, 0.0, 1e5, 4.4, 6e8)),
                                 (Side(1000.0, 300.0, 2e8, 4.4, 6e8), Side(1.2, -50.0, 1e5, 1.4))])
def test_bisection_matches_newton(L, R):
    pb, ub = star_state(L, R, method="bisect")
    pn, un = star_state(L, R, method="newton")
    assert pb == pytest.approx(pn, rel=1e-12)
    assert ub == pytest.approx(un, rel=1e-10, abs=1e-9)


def _check_jumps(s: Side, info, ps, us):
    g, pi = s.gamma, s.pinf
    if info["type"] == "shock":
        S = info["S"]
        rs = info["rho_star"]
        # mass and momentum fluxes through the moving shock
        m0, m1 = s.rho * (s.u - S), rs * (us - S)
        assert m0 == pytest.approx(m1, rel=1e-10)
        assert s.rho * (s.u - S) ** 2 + s.p == pytest.approx(rs * (us - S) ** 2 + ps, rel=1e-10)
        # energy: total enthalpy flux, stiffened-gas internal energy (p + g pi)/((g-1) rho)
        e0 = (s.p + g * pi) / ((g - 1.0) * s.rho)
        e1 = (ps + g * pi) / ((g - 1.0) * rs)
        E0 = s.rho * (e0 + 0.5 * (s.u - S) ** 2)
        E1 = rs * (e1 + 0.5 * (us - S) ** 2)
        assert (E0 + s.p) * (s.u - S) == pytest.approx((E1 + ps) * (us - S), rel=1e-9)
    else:
        rs = info["rho_star"]
        # isentrope (p + pi)/rho^gamma and Riemann invariant across the fan
        assert (ps + pi) / rs ** g == pytest.approx((s.p + pi) / s.rho ** g, rel=1e-10)
        cs = math.sqrt(g * (ps + pi) / rs)
        sign = 1.0 if info["head"] < s.u else -1.0  # left fan: u + 2c/(g-1) constant
        assert s.u + sign * 2 * s.c / (g - 1) == pytest.approx(us + sign * 2 * cs / (g - 1), rel=1e-10)


@pytest.mark.parametrize("L,R", [WATER_AIR,
                                 (Side(1.0, 0.0, 1.0, 1.4), Side(0.125, 0.0, 0.1, 1.4)),
                                 (Side(3.2, 426.96, 4.5e5, 1.4), Side(1000.0, 0.0, 1e5, 4.4, 6e8)),
                                 (Side(1.0, -2.0, 0.4, 1.4), Side(1.0, 2.0, 0.4, 1.4))])
def test_jump_conditions(L, R):
    W = wave_speeds(L, R)
    _check_jumps(L, W["L"], W["p"], W["u"])
    _check_jumps(R, W["R"], W["p"], W["u"])


def test_stiffened_shift_equals_ideal_gas():
    pi = 6.0e8
    L = Side(1000.0, 10.0, 1.0e9, 4.4, pi)
    R = Side(990.0, -5.0, 1.0e5, 4.4, pi)
    Li = Side(1000.0, 10.0, 1.0e9 + pi, 4.4, 0.0)
    Ri = Side(990.0, -5.0, 1.0e5 + pi, 4.4, 0.0)
    p, u = star_state(L, R)
    pi_, ui = star_state(Li, Ri)
    assert p + pi == pytest.approx(pi_, rel=1e-12)
    assert u == pytest.approx(ui, rel=1e-10)
    xi = np.linspace(-3000, 3000, 101)
    r1, u1, p1, _ = sample(L, R, xi)
    r2, u2, p2, _ = sample(Li, Ri, xi)
    np.testing.assert_allclose(r1, r2, rtol=1e-11)
    np.testing.assert_allclose(p1 + pi, p2, rtol=1e-11)


def test_water_air_values_match_hand_estimate():
    """Order-of-magnitude values for the 1000-cell water|air tube computed by
    hand from Toro's relations; the solver must agree to the hand precision."""
    W = wave_speeds(*WATER_AIR)
    assert W["p"] == pytest.approx(1.40e7, rel=0.02)
    assert W["u"] == pytest.approx(483.0, rel=0.01)
    assert W["L"]["rho_star"] == pytest.approx(804.0, rel=0.01)
    assert W["R"]["rho_star"] == pytest.approx(288.0, rel=0.01)
    assert W["L"]["head"] == pytest.approx(-2653.0, rel=0.01)
    assert W["R"]["S"] == pytest.approx(580.0, rel=0.02)


def test_sample_continuity_across_fan():
    L, R = WATER_AIR
    W = wave_speeds(L, R)
    eps = 1e-9
    for xi in (W["L"]["head"], W["L"]["tail"]):
        a = sample(L, R, np.array([xi - eps, xi + eps]))
        assert a[0][0] == pytest.approx(a[0][1], rel=1e-6)
        assert a[2][0] == pytest.approx(a[2][1], rel=1e-6)
