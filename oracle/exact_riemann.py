"""Exact solution of the 1D Riemann problem between two stiffened gases.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Each side K has its own (gamma_K, pi_K).  With pbar = p + pi_K the stiffened
gas behaves as an ideal gas in pbar, so Toro's exact solver (Toro 2009,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4: pressure
functions, star-region velocity, wave-structure sampling) applies side by
side with p -> p + pi_K and c_K = sqrt(gamma_K (p_K + pi_K) / rho_K).  The
star pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, found by
bisection (robust) and refined/cross-checked by Newton.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Side:
    rho: float
    u: float
    p: float
    gamma: float
    pinf: float = 0.0

    @property
    def c(self) -> float:
        return math.sqrt(self.gamma * (self.p + self.pinf) / self.rho)


def _f(s: Side, p: float):
    """Pressure function f_K(p) and its derivative (Toro eqs. 4.6-4.7, 4.37)."""
    g = s.gamma
    pb, pkb = p + s.pinf, s.p + s.pinf
    if p > s.p:  # shock
        A = 2.0 / ((g + 1.0) * s.rho)
        B = (g - 1.0) / (g + 1.0) * pkb
        sq = math.sqrt(A / (pb + B))
        return (p - s.p) * sq, sq * (1.0 - 0.5 * (p - s.p) / (pb + B))
    # rarefaction
    c = s.c
    r = pb / pkb
    e = (g - 1.0) / (2.0 * g)
    if r <= 0.0:  # vacuum limit p + pi_K -> 0
        return -2.0 * c / (g - 1.0), math.inf
    return 2.0 * c / (g - 1.0) * (r ** e - 1.0), (1.0 / (s.rho * c)) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(L: Side, R: Side, tol: float = 1e-15, method: str = "bisect"):
    """(p*, u*) of the Riemann problem; method 'bisect' or 'newton'."""
    du = R.u - L.u
    lo = max(-L.pinf, -R.pinf)  # p + pi_K > 0 on both sides

    def F(p):
        return _f(L, p)[0] + _f(R, p)[0] + du

    if method == "bisect":
        a = lo
        b = max(L.p, R.p, 1.0)
        while F(b) < 0.0:
            b *= 2.0
        if F(a) > 0.0:
            raise ValueError("vacuum generated; no positive star pressure")
        for _ in range(400):
            m = 0.5 * (a + b)
            if F(m) > 0.0:
                b = m
            else:
                a = m
            if b - a <= tol * max(abs(m), 1e-300):
                break
        p = 0.5 * (a + b)
    elif method == "newton":
        # two-rarefaction style initial guess in pbar, then Newton
        p = max(0.5 * (L.p + R.p), lo * 0.5 + 1e-12)
        for _ in range(200):
            fl, dl = _f(L, p)
            fr, dr = _f(R, p)
            step = (fl + fr + du) / (dl + dr)
            pn = p - step
            if pn <= lo:
                pn = 0.5 * (p + lo)
            if abs(pn - p) <= tol * max(abs(pn), 1e-300):
                p = pn
                break
            p = pn
    else:
        raise ValueError(method)
    u = 0.5 * (L.u + R.u) + 0.5 * (_f(R, p)[0] - _f(L, p)[0])
    return p, u


def wave_speeds(L: Side, R: Side):
    """Characteristic speeds of the solution: dict with the star state, the
    shock speeds or rarefaction head/tail on each side, and star densities."""
    ps, us = star_state(L, R)
    out = {"p": ps, "u": us}
    for name, s, sign in (("L", L, -1.0), ("R", R, 1.0)):
        g = s.gamma
        ratio = (ps + s.pinf) / (s.p + s.pinf)
        if ps > s.p:
            S = s.u + sign * s.c * math.sqrt((g + 1.0) / (2.0 * g) * ratio + (g - 1.0) / (2.0 * g))
            gm = (g - 1.0) / (g + 1.0)
            rho_star = s.rho * (ratio + gm) / (gm * ratio + 1.0)
            out[name] = {"type": "shock", "S": S, "rho_star": rho_star}
        else:
            rho_star = s.rho * ratio ** (1.0 / g)
            c_star = s.c * ratio ** ((g - 1.0) / (2.0 * g))
            out[name] = {"type": "rarefaction", "head": s.u + sign * s.c,
                         "tail": us + sign * c_star, "rho_star": rho_star}
    return out


def sample(L: Side, R: Side, xi: np.ndarray):
    """(rho, u, p, side) at similarity coordinates xi = (x - x0)/t.
    side is 0 where the material is the left one and 1 for the right one."""
    xi = np.asarray(xi, dtype=np.float64)
    W = wave_speeds(L, R)
    ps, us = W["p"], W["u"]
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    side = (xi >= us).astype(np.int8)
    for k, x in np.ndenumerate(xi):
        if x < us:
            s, info, sign = L, W["L"], -1.0
        else:
            s, info, sign = R, W["R"], 1.0
        g = s.gamma
        if info["type"] == "shock":
            beyond = (x < info["S"]) if sign < 0 else (x > info["S"])
            if beyond:
                rho[k], u[k], p[k] = s.rho, s.u, s.p
            else:
                rho[k], u[k], p[k] = info["rho_star"], us, ps
        else:
            head, tail = info["head"], info["tail"]
            outside = (x < head) if sign < 0 else (x > head)
            inside_star = (x > tail) if sign < 0 else (x < tail)
            if outside:
                rho[k], u[k], p[k] = s.rho, s.u, s.p
            elif inside_star:
                rho[k], u[k], p[k] = info["rho_star"], us, ps
            else:
                # inside the fan (Toro eq. 4.56 / 4.63 with pbar)
                c = s.c
                base = 2.0 / (g + 1.0) - sign * (g - 1.0) / ((g + 1.0) * c) * (s.u - x)
                rho[k] = s.rho * base ** (2.0 / (g - 1.0))
                u[k] = 2.0 / (g + 1.0) * (-sign * c + (g - 1.0) / 2.0 * s.u + x)
                p[k] = (s.p + s.pinf) * base ** (2.0 * g / (g - 1.0)) - s.pinf
    return rho, u, p, side
