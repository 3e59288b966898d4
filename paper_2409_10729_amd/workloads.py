"""Seeded synthetic problems shaped like the paper's two-phase workloads.

This module only draws initial conditions in PRIMITIVE variables
(alpha1*rho1, alpha2*rho2, u, v, w, p, alpha1), stored [7][nz][ny][nx] in
float64, plus the grid description.  It holds none of the solver's
arithmetic (no equation of state, no reconstruction, no fluxes): both the
GPU library and the CPU oracle convert these fields to conserved variables
with their own code.

Fluid 1 is water-like (gamma 4.4, pi_inf 6e8), fluid 2 air-like (gamma 1.4,
pi_inf 0).  Domain [0,1]^d, uniform spacing 1/n, cell centres (i + 1/2)/n.
Random numbers come from numpy's PCG64 ``default_rng(seed)``.

Workloads (the paper's demonstrations, Sec. V, are 2B-cell shock-droplet and
shock-bubble-cloud runs; these are single-GPU blocks of the same physics):
  shock_tube      1D water|air tube, 1000 cells, transmissive
  advected_bubble 3D periodic air bubble in water, uniform velocity
  shock_droplet   3D Mach-2 air shock on a water droplet with 1% density noise
  shock_droplet_stretched
                  the same on a grid refined around the droplet (tanh)
  bubble_cloud    3D Mach-1.5 water shock on several air bubbles
  droplet_cloud   3D Mach-2 air shock on many log-uniform droplets
  random_smooth   small random valid states for RHS parity
  advected_slab, shock_tube_family
                  1D families for training and evaluating the learned weights
  random_smooth_nf, droplet_bubble
                  the same for more than two fluids (variables: nf partial
                  densities, u, v, w, p, volume fractions 1 .. nf-1)
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC, TRANSMISSIVE, REFLECTIVE, INFLOW = 0, 1, 2, 3
WATER = (4.4, 6.0e8)
AIR = (1.4, 0.0)
HELIUM = (5.0 / 3.0, 0.0)
SF6 = (1.1, 0.0)
FLUIDS = (WATER, AIR, HELIUM, SF6)  # fluid i of an nf-fluid problem is FLUIDS[i]
ALPHA_EPS = 1.0e-6


def spec(n, bc, cfl=0.4, eps=1e-6):
    n = tuple(int(v) for v in n)
    return {
        "n": n,
        "dx": tuple(1.0 / v for v in n),
        "lo": (0.0, 0.0, 0.0),
        "bc": tuple(tuple(int(b) for b in pair) for pair in bc),
        "gamma": (WATER[0], AIR[0]),
        "pinf": (WATER[1], AIR[1]),
        "eps": float(eps),
        "cfl": float(cfl),
    }


def spec_fluids(n, bc, nf, cfl=0.4, eps=1e-6):
    """Grid description of an nf-fluid problem (fluids FLUIDS[:nf])."""
    s = spec(n, bc, cfl, eps)
    s["gamma"] = tuple(f[0] for f in FLUIDS[:nf])
    s["pinf"] = tuple(f[1] for f in FLUIDS[:nf])
    return s


def _pack_nf(alphas, rhos, u, v, w, p):
    """Primitives of the nf-fluid model: alpha_i rho_i (i = 1..nf), u, v, w,
    p, alpha_1 .. alpha_{nf-1}; the alphas are the nf volume fractions."""
    nf = len(alphas)
    shape = np.broadcast(*alphas, *rhos, u, v, w, p).shape
    out = np.empty((2 * nf + 3,) + shape, dtype=np.float64)
    for i in range(nf):
        out[i] = alphas[i] * rhos[i]
    out[nf], out[nf + 1], out[nf + 2], out[nf + 3] = u, v, w, p
    for i in range(nf - 1):
        out[nf + 4 + i] = alphas[i]
    return out


def _centres(n):
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    return np.meshgrid(z, y, x, indexing="ij")  # Z, Y, X each [nz, ny, nx]


def _pack(a1, rho1, rho2, u, v, w, p):
    a1 = np.asarray(a1, dtype=np.float64)
    shape = a1.shape
    out = np.empty((7,) + shape, dtype=np.float64)
    out[0] = a1 * rho1
    out[1] = (1.0 - a1) * rho2
    out[2] = u
    out[3] = v
    out[4] = w
    out[5] = p
    out[6] = a1
    return out


def _smooth_indicator(dist, radius, width):
    """1 inside the sphere, 0 outside, tanh transition of the given width."""
    return 0.5 * (1.0 - np.tanh((dist - radius) / width))


def shock_tube(n=1000, x0=0.5, p_left=1.0e9, p_right=1.0e5, rho_w=1000.0, rho_a=50.0):
    """Water (left, alpha1 = 1-1e-6) against air (right, alpha1 = 1e-6), both at rest."""
    s = spec((n, 1, 1), ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    x = (np.arange(n) + 0.5) / n
    left = x < x0
    a1 = np.where(left, 1.0 - ALPHA_EPS, ALPHA_EPS)
    p = np.where(left, p_left, p_right)
    w = _pack(a1, rho_w, rho_a, 0.0, 0.0, 0.0, p)
    return {"name": "shock_tube", "spec": s, "w": w.reshape(7, 1, 1, n)}


def advected_bubble(n=128, seed=0, velocity=(1.0, 0.5, 0.25), p0=1.0e5):
    """Air bubble (radius U(0.1,0.2), centre U(0,1)^3) in water; periodic;
    interface alpha1 = e + (1-2e) * 0.5 (1 + tanh((r-R)/(1.5 dx)))."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.1, 0.2)
    c = rng.uniform(0.0, 1.0, size=3)
    s = spec(n3, ((PERIODIC, PERIODIC),) * 3)
    Z, Y, X = _centres(n3)
    d = [X - c[0], Y - c[1], Z - c[2]]
    d = [a - np.round(a) for a in d]  # minimum image on the unit torus
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    width = 1.5 / max(n3)
    a1 = ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * 0.5 * (1.0 + np.tanh((r - R) / width))
    w = _pack(a1, 1000.0, 1.2, velocity[0], velocity[1], velocity[2], p0)
    return {"name": "advected_bubble", "spec": s, "w": w, "meta": {"R": R, "centre": c.tolist()}}


def advected_slab(n=256, seed=0, u_range=(100.0, 400.0), p0=1.0e5):
    """1D periodic water slab in air (centre U(0.3,0.7), half-width
    U(0.1,0.2), tanh interfaces over 1.5 cells) moving at a uniform speed
    U(u_range).  Returns the problem and `face_prims(t)`: the translated
    profile evaluated at the n+1 faces at time t, [7][n+1] (the exact
    solution of pure advection, used as training and error reference)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7)
    R = rng.uniform(0.1, 0.2)
    u = rng.uniform(*u_range)
    width = 1.5 / n
    s = spec((n, 1, 1), ((PERIODIC, PERIODIC),) * 3)

    def profile(x):
        d = x - c
        d = d - np.round(d)
        return ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * 0.5 * (1.0 - np.tanh((np.abs(d) - R) / width))

    x = (np.arange(n) + 0.5) / n
    a1 = profile(x)
    w = _pack(a1, 1000.0, 1.2, u, 0.0, 0.0, p0).reshape(7, 1, 1, n)

    def face_prims(t):
        xf = np.arange(n + 1) / n - u * t
        return _pack(profile(xf), 1000.0, 1.2, u, 0.0, 0.0, p0)

    def alpha_cell_avg(t, sub=32):
        """Cell averages of the translated alpha1 profile (midpoint rule, `sub` points per cell)."""
        xs = (np.arange(n)[:, None] + (np.arange(sub)[None, :] + 0.5) / sub) / n - u * t
        return profile(xs).mean(axis=1)

    return {"name": "advected_slab", "spec": s, "w": w, "face_prims": face_prims, "alpha_cell_avg": alpha_cell_avg,
            "meta": {"u": u, "c": c, "R": R}}


def shock_tube_family(n=500, seed=0):
    """Water|air tube of the shock_tube kind with a seeded interface position
    U(0.3,0.7) and left pressure log-uniform in [1e8, 1e9]."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.3, 0.7)
    pl = float(np.exp(rng.uniform(np.log(1e8), np.log(1e9))))
    P = shock_tube(n=n, x0=x0, p_left=pl)
    P["meta"] = {"x0": x0, "p_left": pl}
    return P


def _ideal_gas_shock(M, rho1, p1, gamma):
    """Post-shock (rho, p, u) behind a shock of Mach M into gas at rest
    (normal-shock relations)."""
    c1 = math.sqrt(gamma * p1 / rho1)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (M * M - 1.0))
    rho2 = rho1 * (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    u2 = M * c1 * (1.0 - rho1 / rho2)
    return rho2, p2, u2


def _stiff_shock(M, rho1, p1, gamma, pinf):
    """Same relations written in p + pi_inf (stiffened gas)."""
    c1 = math.sqrt(gamma * (p1 + pinf) / rho1)
    pb2 = (p1 + pinf) * (1.0 + 2.0 * gamma / (gamma + 1.0) * (M * M - 1.0))
    rho2 = rho1 * (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    u2 = M * c1 * (1.0 - rho1 / rho2)
    return rho2, pb2 - pinf, u2


def _noise(rng, shape, amp=0.01):
    return 1.0 + amp * np.clip(rng.standard_normal(shape), -3.0, 3.0)


def shock_droplet(n=256, seed=0, mach=2.0, radius=0.15, noise=0.01):
    """Mach-2 air shock (ideal-gas normal-shock state) 4 cells upstream of a
    water droplet (radius 0.15, centre (0.5,0.5,0.5) + U(-0.05,0.05)^3);
    x transmissive, y/z periodic; 1% Gaussian multiplicative density noise
    (clipped at 3 sigma) on both partial densities."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    c = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    s = spec(n3, ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    Z, Y, X = _centres(n3)
    h = 1.0 / n3[0]
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    water = _smooth_indicator(r, radius, 1.5 * h)
    a1 = ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * water
    rho_a1, p_a1 = 1.2, 1.0e5
    rho_a2, p_a2, u_a2 = _ideal_gas_shock(mach, rho_a1, p_a1, AIR[0])
    xs = c[0] - radius - 4.0 * h
    post = X < xs
    rho_air = np.where(post, rho_a2, rho_a1)
    p = np.where(post, p_a2, p_a1)
    u = np.where(post, u_a2, 0.0)
    w = _pack(a1, 1000.0, rho_air, u, 0.0, 0.0, p)
    f = _noise(rng, a1.shape, noise)
    w[0] *= f
    w[1] *= f
    return {"name": "shock_droplet", "spec": s, "w": w,
            "meta": {"centre": c.tolist(), "radius": radius, "shock_x": xs}}


def shock_droplet_walls(n=256, seed=0, mach=2.0, radius=0.15, noise=0.01):
    """The shock droplet in a closed channel: the x-lower side is an inflow
    held at the post-shock air state (the shock keeps being driven), the
    x-upper side transmissive, walls (reflective) in y and z; the same
    initial state as shock_droplet.  The inflow state comes as primitives
    (inflow_prim [3][2][7], zero for the other sides); each consumer
    converts it to the conserved ghost state with its own EOS code."""
    P = shock_droplet(n=n, seed=seed, mach=mach, radius=radius, noise=noise)
    s = dict(P["spec"])
    s["bc"] = ((INFLOW, TRANSMISSIVE), (REFLECTIVE, REFLECTIVE), (REFLECTIVE, REFLECTIVE))
    rho_a2, p_a2, u_a2 = _ideal_gas_shock(mach, 1.2, 1.0e5, AIR[0])
    prim = np.zeros((3, 2, 7))
    prim[0, 0] = [ALPHA_EPS * 1000.0, (1.0 - ALPHA_EPS) * rho_a2, u_a2, 0.0, 0.0, p_a2, ALPHA_EPS]
    return {"name": "shock_droplet_walls", "spec": s, "w": P["w"], "inflow_prim": prim, "meta": P["meta"]}


def _sphere_union(n3, centres, radii, width):
    """max over spheres of _smooth_indicator(distance to centre, R, width) on
    the cell centres.  Each sphere is evaluated only on the index box within
    R + 20 widths of its centre: beyond that tanh rounds to 1 and the
    indicator is exactly 0, so the result equals the whole-grid evaluation
    bit for bit."""
    nx, ny, nz = n3
    out = np.zeros((nz, ny, nx))
    for c, R in zip(centres, radii):
        m = R + 20.0 * width
        sl = []
        for ax, nn in zip((2, 1, 0), (nz, ny, nx)):
            lo = max(0, int(np.floor((c[ax] - m) * nn - 0.5)))
            hi = min(nn, int(np.ceil((c[ax] + m) * nn + 0.5)) + 1)
            sl.append(slice(lo, hi))
        z = (np.arange(sl[0].start, sl[0].stop) + 0.5) / nz
        y = (np.arange(sl[1].start, sl[1].stop) + 0.5) / ny
        x = (np.arange(sl[2].start, sl[2].stop) + 0.5) / nx
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        sub = out[sl[0], sl[1], sl[2]]
        np.maximum(sub, _smooth_indicator(r, R, width), out=sub)
    return out


def _place_spheres(rng, count, rmin, rmax, gap, log_uniform, xmin=0.15, tries=20000):
    centres, radii = [], []
    for _ in range(tries):
        if len(radii) == count:
            break
        r = math.exp(rng.uniform(math.log(rmin), math.log(rmax))) if log_uniform else rng.uniform(rmin, rmax)
        c = np.array([rng.uniform(xmin + r, 1.0 - r - gap), rng.uniform(r, 1.0 - r), rng.uniform(r, 1.0 - r)])
        if all(np.linalg.norm(c - c2) >= r + r2 + gap for c2, r2 in zip(centres, radii)):
            centres.append(c)
            radii.append(r)
    return centres, radii


def bubble_cloud(n=192, seed=0, mach=1.5):
    """Water at rest (rho 1000, p 1e5) with U{4..16} non-overlapping air
    bubbles of radius U(0.05,0.15) (gap >= 4 cells); Mach-1.5 water shock
    (stiffened-gas normal-shock state) 4 cells upstream of the first bubble."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    h = 1.0 / n3[0]
    nb = int(rng.integers(4, 17))
    centres, radii = _place_spheres(rng, nb, 0.05, 0.15, 4.0 * h, False)
    s = spec(n3, ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    Z, Y, X = _centres(n3)
    air = np.zeros(X.shape)
    for c, R in zip(centres, radii):
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        air = np.maximum(air, _smooth_indicator(r, R, 1.5 * h))
    a1 = ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * (1.0 - air)
    rho2, p2, u2 = _stiff_shock(mach, 1000.0, 1.0e5, WATER[0], WATER[1])
    xs = min(c[0] - R for c, R in zip(centres, radii)) - 4.0 * h
    post = X < xs
    rho_w = np.where(post, rho2, 1000.0)
    p = np.where(post, p2, 1.0e5)
    u = np.where(post, u2, 0.0)
    w = _pack(a1, rho_w, 1.2, u, 0.0, 0.0, p)
    return {"name": "bubble_cloud", "spec": s, "w": w,
            "meta": {"bubbles": len(radii), "shock_x": xs}}


def droplet_cloud(n=384, seed=0, count=32, mach=2.0, noise=0.01):
    """Shock-droplet physics with ``count`` non-overlapping water droplets of
    log-uniform radius in [0.02, 0.1]."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    h = 1.0 / n3[0]
    centres, radii = _place_spheres(rng, count, 0.02, 0.1, 4.0 * h, True, xmin=0.2)
    s = spec(n3, ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    Z, Y, X = _centres(n3)
    water = _sphere_union(n3, centres, radii, 1.5 * h)
    a1 = ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * water
    rho_a2, p_a2, u_a2 = _ideal_gas_shock(mach, 1.2, 1.0e5, AIR[0])
    xs = min(c[0] - R for c, R in zip(centres, radii)) - 4.0 * h
    post = X < xs
    rho_air = np.where(post, rho_a2, 1.2)
    p = np.where(post, p_a2, 1.0e5)
    u = np.where(post, u_a2, 0.0)
    w = _pack(a1, 1000.0, rho_air, u, 0.0, 0.0, p)
    f = _noise(rng, a1.shape, noise)
    w[0] *= f
    w[1] *= f
    return {"name": "droplet_cloud", "spec": s, "w": w,
            "meta": {"droplets": len(radii), "shock_x": xs}}


def random_smooth(n=(24, 20, 16), seed=0, bc=None, jumps=True):
    """Random valid state: smooth Fourier-mode fields plus (optionally) a
    material interface and a pressure jump, for RHS parity on small grids.
    bc defaults to periodic in every direction."""
    n3 = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    if bc is None:
        bc = ((PERIODIC, PERIODIC),) * 3
    s = spec(n3, bc)
    Z, Y, X = _centres(n3)

    def field(amp):
        f = np.zeros(X.shape)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            f += rng.uniform(-1, 1) * np.sin(2 * math.pi * k[0] * X + ph[0]) * \
                np.sin(2 * math.pi * k[1] * Y + ph[1]) * np.sin(2 * math.pi * k[2] * Z + ph[2])
        return amp * f / 3.0

    a1 = 0.5 + field(0.45)
    p = 1.0e5 * (1.0 + field(0.5))
    rho1 = 1000.0 * (1.0 + field(0.05))
    rho2 = 1.2 * (1.0 + field(0.3))
    u, v, w_ = field(50.0), field(50.0), field(50.0)
    if jumps:
        cx = rng.uniform(0.3, 0.7)
        inside = X < cx
        a1 = np.where(inside, 1.0 - ALPHA_EPS, a1)
        p = np.where(Y < rng.uniform(0.3, 0.7), p * 20.0, p)
    w = _pack(a1, rho1, rho2, u, v, w_, p)
    return {"name": "random_smooth", "spec": s, "w": w}


def random_smooth_nf(n=(24, 20, 16), seed=0, bc=None, nf=3, jumps=True):
    """Random valid nf-fluid state: smooth Fourier-mode volume fractions
    (each in about [0.05, 0.8], summing to 1), phase densities, velocity and
    pressure, plus (optionally) a region of nearly pure fluid 1 and a 20x
    pressure jump.  bc defaults to periodic."""
    n3 = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    if bc is None:
        bc = ((PERIODIC, PERIODIC),) * 3
    s = spec_fluids(n3, bc, nf)
    Z, Y, X = _centres(n3)

    def field(amp):
        f = np.zeros(X.shape)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            f += rng.uniform(-1, 1) * np.sin(2 * math.pi * k[0] * X + ph[0]) * \
                np.sin(2 * math.pi * k[1] * Y + ph[1]) * np.sin(2 * math.pi * k[2] * Z + ph[2])
        return amp * f / 3.0

    raw = [1.0 + field(0.8) for _ in range(nf)]
    tot = sum(raw)
    alphas = [r / tot for r in raw]
    base = (1000.0, 1.2, 0.17, 6.0)
    rhos = [base[i] * (1.0 + field(0.2)) for i in range(nf)]
    u, v, w_ = field(50.0), field(50.0), field(50.0)
    p = 1.0e5 * (1.0 + field(0.5))
    if jumps:
        inside = X < rng.uniform(0.3, 0.7)
        alphas = [np.where(inside, 1.0 - (nf - 1) * ALPHA_EPS if i == 0 else ALPHA_EPS, a)
                  for i, a in enumerate(alphas)]
        p = np.where(Y < rng.uniform(0.3, 0.7), p * 20.0, p)
    return {"name": f"random_smooth_{nf}f", "spec": s, "w": _pack_nf(alphas, rhos, u, v, w_, p)}


def droplet_bubble(n=256, seed=0, mach=2.0, radius=0.15, bubble=0.08, noise=0.01):
    """Three fluids: the shock_droplet problem (Mach-2 air shock 4 cells
    upstream of a water droplet of radius 0.15, 1% density noise) with a
    helium bubble (radius 0.08) in the air beside the droplet, at a seeded
    centre.  Fluids: water, air, helium; x transmissive, y/z periodic."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    c = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    cb = np.array([c[0] + rng.uniform(-0.05, 0.05), c[1] + radius + bubble + 0.06, c[2] + rng.uniform(-0.05, 0.05)])
    s = spec_fluids(n3, ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)), 3)
    Z, Y, X = _centres(n3)
    h = 1.0 / n3[0]
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    rb = np.sqrt((X - cb[0]) ** 2 + (Y - cb[1]) ** 2 + (Z - cb[2]) ** 2)
    water = _smooth_indicator(r, radius, 1.5 * h)
    helium = _smooth_indicator(rb, bubble, 1.5 * h) * (1.0 - water)
    a_w = ALPHA_EPS + (1.0 - 3.0 * ALPHA_EPS) * water
    a_h = ALPHA_EPS + (1.0 - 3.0 * ALPHA_EPS) * helium
    a_a = 1.0 - a_w - a_h
    rho_a1, p_a1 = 1.2, 1.0e5
    rho_a2, p_a2, u_a2 = _ideal_gas_shock(mach, rho_a1, p_a1, AIR[0])
    xs = min(c[0] - radius, cb[0] - bubble) - 4.0 * h
    post = X < xs
    rho_air = np.where(post, rho_a2, rho_a1)
    p = np.where(post, p_a2, p_a1)
    u = np.where(post, u_a2, 0.0)
    w = _pack_nf([a_w, a_a, a_h], [1000.0, rho_air, 0.17], u, 0.0, 0.0, p)
    f = _noise(rng, a_w.shape, noise)
    for i in range(3):
        w[i] *= f
    return {"name": "droplet_bubble", "spec": s, "w": w,
            "meta": {"centre": c.tolist(), "bubble_centre": cb.tolist(), "shock_x": xs}}


def tanh_faces(n, centre=0.5, depth=0.5, sharpness=8.0, lo=0.0, hi=1.0):
    """Face coordinates (n + 1) of a structured direction refined locally by a
    hyperbolic tangent: the map x(s) = s - (depth / sharpness) tanh(sharpness
    (s - centre)) of the uniform coordinate s in [0, 1], rescaled onto
    [lo, hi], has dx/ds = 1 - depth sech^2(sharpness (s - centre)), so cells
    near `centre` are finer by up to the factor 1 - depth (0 <= depth < 1)
    and the widths vary smoothly.  depth = 0 gives uniform cells."""
    if not 0.0 <= depth < 1.0:
        raise ValueError("depth must lie in [0, 1)")
    s = np.arange(n + 1) / n
    x = s - (depth / sharpness) * np.tanh(sharpness * (s - centre))
    x = (x - x[0]) / (x[-1] - x[0])
    out = lo + (hi - lo) * x
    out[0], out[-1] = lo, hi
    return out


def shock_droplet_stretched(n=256, seed=0, mach=2.0, radius=0.15, noise=0.01, depth=0.5, sharpness=8.0):
    """The shock_droplet problem on a grid refined around the droplet in all
    three directions: faces from tanh_faces centred on the droplet centre
    (cells there finer by up to 1 - depth), the fields evaluated at the
    stretched cell centres, the shock 4 of the finest cells upstream of the
    droplet; x transmissive, y/z periodic."""
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    c = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    faces = [tanh_faces(n3[d], centre=c[d], depth=depth, sharpness=sharpness) for d in range(3)]
    s = spec(n3, ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    s["faces"] = tuple(faces)
    xc, yc, zc = (0.5 * (f[1:] + f[:-1]) for f in faces)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    h = float(min(np.diff(f).min() for f in faces))
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    water = _smooth_indicator(r, radius, 1.5 * h)
    a1 = ALPHA_EPS + (1.0 - 2.0 * ALPHA_EPS) * water
    rho_a1, p_a1 = 1.2, 1.0e5
    rho_a2, p_a2, u_a2 = _ideal_gas_shock(mach, rho_a1, p_a1, AIR[0])
    xs = c[0] - radius - 4.0 * h
    post = X < xs
    rho_air = np.where(post, rho_a2, rho_a1)
    p = np.where(post, p_a2, p_a1)
    u = np.where(post, u_a2, 0.0)
    w = _pack(a1, 1000.0, rho_air, u, 0.0, 0.0, p)
    f = _noise(rng, a1.shape, noise)
    w[0] *= f
    w[1] *= f
    return {"name": "shock_droplet_stretched", "spec": s, "w": w,
            "meta": {"centre": c.tolist(), "radius": radius, "shock_x": xs, "finest_width": h}}


def stretched(P, faces):
    """The problem P on a non-uniform grid: spec["faces"] = faces (per
    direction an array of n + 1 face coordinates, or None for uniform
    cells); the field values are kept cell by cell."""
    return dict(P, spec=dict(P["spec"], faces=tuple(faces)))
