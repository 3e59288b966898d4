"""The learned WENO weights as the sweeps apply them, against the oracle's
learned right-hand side (oracle.rhs_learned), element by element.

Each case runs the solver's right-hand side in a learned mode
(MFX_WENO5_LEARNED: one network evaluation per variable and edge;
MFX_WENO5_LEARNED_EDGE: one per edge on pooled features, its logits
correcting each variable's own Jiang-Shu weights) through the C ABI
and compares it with the oracle on the same state and network:
  * per field, max |gpu - oracle| over the flux scale <= the tolerance
    parity_util.learned_tolerance derives: the float32 bar (1e-5) plus four
    times the oracle's own response to float32 rounding of its inputs (the
    network's operands are quantised to bfloat16, so a rounding difference
    of an operand can move a weight; the oracle measures how far);
  * at most 1% of the cells above the float32 bar;
  * the fallback count (edges a face uses, each distinct face once) within
    2 + 1% of the oracle's plus four times its own rounding response.
Networks: a random one (every edge corrected), the committed trained ones,
and a steered one whose weights sit on the most upwind candidate (many
edges fail the admissibility test and fall back).  Kernels: the x row
kernel with its boundary faces, the marching x sweep (forced, and for rows
longer than 512), the y and z sweeps; periodic, transmissive, reflective
and inflow sides.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2409_10729_amd import MFX_FP32_MIXED, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE
from paper_2409_10729_amd import workloads as wl
from parity_util import FP32_BAR, flux_scale, gpu_solver, learned_reference, learned_tolerance, sample_cells

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2409_10729_amd", "data")
PER_VAR, SHARED = oracle.LEARNED_PER_VARIABLE, oracle.LEARNED_SHARED
WEIGHTS = {PER_VAR: MFX_WENO5_LEARNED, SHARED: MFX_WENO5_LEARNED_EDGE}


def _walls(n, seed):
    P = wl.shock_droplet_walls(n=n, seed=seed)
    g1 = oracle.make_grid(dict(P["spec"], n=(1, 1, 1), bc=((0, 0),) * 3))
    inflow = np.array([[oracle.prim_to_cons(g1, np.asarray(w7).reshape(7, 1, 1, 1)).reshape(7) for w7 in pair]
                       for pair in P["inflow_prim"]])
    return dict(P, spec=dict(P["spec"], inflow=inflow))


PROBLEMS = {
    "smooth": lambda: wl.random_smooth(n=(24, 20, 16), seed=1, bc=((1, 1), (0, 0), (0, 0))),
    "droplet": lambda: wl.shock_droplet(n=(40, 24, 20), seed=2),
    "tube": lambda: wl.shock_tube(n=200),
    # rows longer than the row kernel takes (marching x sweep); a smooth state:
    # the shock droplet on 5 x 4 cells across would be a sharp 3D interface
    # whose face states leave the physical range in the oracle as well
    "long_rows": lambda: wl.random_smooth(n=(600, 5, 4), seed=3, bc=((1, 1), (0, 0), (0, 0))),
    "walls": lambda: _walls((36, 20, 18), 4),
    "cloud": lambda: wl.bubble_cloud(n=(40, 24, 20), seed=1),
}


def _steered():
    p = omlp.unpack(omlp.init_params(12))
    p["b3"] = np.array([40.0, -40.0, -40.0])
    return omlp.pack(p)


def _network(name):
    if name == "random":
        return omlp.init_params(4, out_scale=0.5)
    if name == "steered":
        return _steered()
    return np.load(os.path.join(DATA, name + ".npy"), allow_pickle=False)


CASES = [
    ("smooth", PER_VAR, "random", "rows"),
    ("smooth", SHARED, "random", "rows"),
    ("droplet", PER_VAR, "mlp_weno5", "rows"),
    ("droplet", SHARED, "mlp_weno5_edge", "rows"),
    ("droplet", PER_VAR, "steered", "rows"),
    ("droplet", SHARED, "steered", "rows"),
    ("droplet", PER_VAR, "random", "march"),
    ("droplet", SHARED, "random", "march"),
    ("tube", PER_VAR, "random", "rows"),
    ("tube", SHARED, "steered", "rows"),
    ("long_rows", PER_VAR, "random", "rows"),
    ("walls", PER_VAR, "random", "rows"),
    ("walls", SHARED, "mlp_weno5_edge", "rows"),
    ("cloud", SHARED, "random", "rows"),
    ("cloud", PER_VAR, "mlp_weno5", "rows"),
]


@pytest.mark.parametrize("problem,mode,net,xpass", CASES)
def test_learned_rhs_matches_oracle(problem, mode, net, xpass, monkeypatch):
    if xpass == "march":
        monkeypatch.setenv("MFX_XSWEEP", "march")
    P = PROBLEMS[problem]()
    spec = P["spec"]
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, P["w"])
    theta = np.asarray(_network(net), dtype=np.float32)
    print(f"case {problem} mode {mode} net {net} x pass {xpass} n={spec['n']}", flush=True)
    s = gpu_solver(spec, q0=q0, precision=MFX_FP32_MIXED, weights=WEIGHTS[mode])
    s.set_mlp(torch.from_numpy(theta).cuda())
    r = s.rhs().cpu().numpy()
    st = s.stats()
    ref = learned_reference(spec, q0, theta, mode)
    den = np.maximum(np.abs(ref["rhs"]).reshape(7, -1).max(axis=1), flux_scale(q0, spec))
    cell_err = np.abs(r - ref["rhs"]).reshape(7, -1) / den[:, None]
    err = cell_err.max(axis=1)
    tol = learned_tolerance(ref)
    above = float(np.mean(cell_err.max(axis=0) > FP32_BAR))
    fb_tol = 2 + 0.01 * ref["fallbacks"] + 4 * ref["fallback_shift"]
    print("  error per field " + " ".join(f"{e:.1e}" for e in err), flush=True)
    print("  tolerance       " + " ".join(f"{t:.1e}" for t in tol), flush=True)
    print(f"  cells above the float32 bar {above:.4f}; fallback edges gpu {st['fallback_faces']} oracle "
          f"{ref['fallbacks']} (near a threshold {ref['near']}, rounding response {ref['fallback_shift']})",
          flush=True)
    assert st["error"] == 0
    assert np.all(err <= tol), (err, tol)
    assert above <= 0.01
    assert abs(st["fallback_faces"] - ref["fallbacks"]) <= fb_tol


FULL = [
    # the learned configuration (multi-bubble, 192^3) and the benchmark's problem (256^3)
    ("bubble_cloud", 192, PER_VAR, "mlp_weno5"),
    ("bubble_cloud", 192, SHARED, "mlp_weno5_edge"),
    ("shock_droplet", 256, PER_VAR, "mlp_weno5"),
    ("shock_droplet", 256, SHARED, "mlp_weno5_edge"),
]


@pytest.mark.parametrize("workload,n,mode,net", FULL)
def test_full_size_learned_rhs_sampled(workload, n, mode, net):
    """The learned right-hand side at full size, in the launch configuration
    the benchmark times, against the oracle's cell-by-cell learned
    right-hand side on sampled cells (random cells, every boundary-adjacent
    cell class, the steepest interfaces and shocks).  Tolerance as above,
    with the oracle's float32-rounding response measured on the same cells."""
    P = getattr(wl, workload)(n=n, seed=0)
    spec = P["spec"]
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, P["w"])
    theta = np.asarray(_network(net), dtype=np.float32)
    print(f"full size {workload} {n}^3 mode {mode} net {net}", flush=True)
    s = gpu_solver(spec, q0=q0, precision=MFX_FP32_MIXED, weights=WEIGHTS[mode])
    s.set_mlp(torch.from_numpy(theta).cuda())
    r = s.rhs().cpu().numpy().reshape(7, -1)
    assert s.stats()["error"] == 0
    s.destroy()
    cells = sample_cells(spec, 300, seed=n, q0=q0)
    ref = oracle.rhs_learned_at(g, q0, theta, cells, mode).T
    w = oracle.cons_to_prim(g, q0)
    q32 = oracle.prim_to_cons(g, w.astype(np.float32).astype(np.float64))
    del w
    ref32 = oracle.rhs_learned_at(g, q32, theta, cells, mode).T
    del q32
    sc = flux_scale(q0, spec)
    sens = np.abs(ref - ref32).max(axis=1) / np.where(sc > 0, sc, 1.0)
    tol = FP32_BAR + 4.0 * sens
    den = np.maximum(np.abs(ref).max(axis=1), sc)
    cell_err = np.abs(r[:, cells] - ref) / den[:, None]
    err = cell_err.max(axis=1)
    above = float(np.mean(cell_err.max(axis=0) > FP32_BAR))
    print(f"  {cells.size} cells; error per field " + " ".join(f"{e:.1e}" for e in err), flush=True)
    print("  tolerance " + " ".join(f"{t:.1e}" for t in tol) + f"; cells above the float32 bar {above:.4f}",
          flush=True)
    assert np.all(err <= tol), (err, tol)
    assert above <= 0.01
