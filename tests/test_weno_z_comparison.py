"""WENO-Z against the paper's Jiang-Shu WENO5 on the held-out problems the
learned forms are judged on (the 1000-cell water/air tube after 300 CFL
steps, L1 of density + velocity + pressure against the exact solution; the
advected slab of seed 7777 after 200 steps, L1 of alpha1 against the exact
cell averages), both run by the FP64 oracle.  WENO-Z is a comparison form
for the learned weights: the GPU tests of the learned forms assert their own
gains against Jiang-Shu on the same problems."""
import numpy as np

import oracle
from oracle import exact_riemann as er
from paper_2409_10729_amd import workloads as wl


def _l1(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())


def _tube(weno_z):
    P = wl.shock_tube()
    g = oracle.make_grid(P["spec"], weno_z=weno_z)
    q = oracle.prim_to_cons(g, P["w"])
    t = 0.0
    for _ in range(300):
        q, dt = oracle.rk3_step(g, q)
        t += dt
    w = oracle.cons_to_prim(g, q).reshape(7, -1)
    x = (np.arange(1000) + 0.5) / 1000
    re, ue, pe, _ = er.sample(er.Side(1000.0, 0, 1e9, 4.4, 6e8), er.Side(50.0, 0, 1e5, 1.4, 0.0), (x - 0.5) / t)
    return _l1(w[0] + w[1], re) + float(np.abs(w[2] - ue).mean() / np.abs(ue).max()) + _l1(w[5], pe)


def _slab(weno_z):
    P = wl.advected_slab(n=256, seed=7777)
    g = oracle.make_grid(P["spec"], weno_z=weno_z)
    q = oracle.prim_to_cons(g, P["w"])
    t = 0.0
    for _ in range(200):
        q, dt = oracle.rk3_step(g, q)
        t += dt
    return _l1(q.reshape(7, -1)[6], P["alpha_cell_avg"](t))


def test_weno_z_against_jiang_shu_on_the_gain_problems():
    res = {name: (_tube(z), _slab(z)) for name, z in (("jiang-shu", False), ("weno-z", True))}
    print("L1 (tube rho+u+p, slab alpha1):", res, flush=True)
    assert res["weno-z"][0] < res["jiang-shu"][0] and res["weno-z"][1] < res["jiang-shu"][1]
