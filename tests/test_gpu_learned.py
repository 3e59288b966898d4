"""Learned WENO weights on the GPU against the FP64 oracle (oracle/mlp.py)
and against exact solutions.

  * features, Jiang-Shu weights and normalised candidates of the data
    preparation kernel;
  * the float32 forward and the bfloat16 matrix-core forward (compared with
    the oracle evaluated on bfloat16-rounded operands);
  * loss and gradient of the training kernels (relative L2 per tensor
    <= 1e-4), deterministic across calls; one Adam step;
  * a network with NaN parameters makes every edge fall back to Jiang-Shu
    (tests the fallback plumbing); a zero output layer reproduces the
    Jiang-Shu run (tests the residual form);
  * the solution-error fine-tuning optimiser on a closed-form objective;
  * gain: with the committed parameters the learned form's L1 error against
    the exact solution is below the Jiang-Shu form's on held-out problems
    (the standard tube is outside the training seeds, the slab seeds too).
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
from oracle import mlp as omlp
from paper_2409_10729_amd import MFX_FP32_MIXED, MFX_WENO5_JS, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE
from paper_2409_10729_amd import workloads as wl
from parity_util import rel_linf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stencils(n, seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(n, 5)) * rng.uniform(0.01, 1e3, size=(n, 1)) + rng.normal(size=(n, 1)) * 10
    V[::3, 3:] += rng.uniform(1, 1e4, size=(len(V[::3]), 1))
    return V


def _prep(V, T):
    from paper_2409_10729_amd import learned

    st = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    tg = torch.from_numpy(np.ascontiguousarray(T)).cuda()
    return learned.features(st, tg)


def test_features_match_oracle():
    V = _stencils(3000, 0)
    T = V[:, 2] + 0.1 * (V[:, 3] - V[:, 2])
    feat, cand, tn, ojs = (x.cpu().numpy().astype(np.float64) for x in _prep(V, T))
    np.testing.assert_allclose(feat, omlp.features(V), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(ojs, omlp.js_weights_right(V), rtol=1e-6, atol=1e-7)
    sc = V.max(1) - V.min(1)
    c_ref = (omlp.candidates_right(V) - V[:, 2:3]) / sc[:, None]
    np.testing.assert_allclose(cand, c_ref, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(tn, (T - V[:, 2]) / sc, rtol=1e-6, atol=1e-6)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def test_forward_f32_matches_oracle():
    from paper_2409_10729_amd import learned

    theta = omlp.init_params(11, out_scale=0.5)
    V = _stencils(4096, 1)
    X, OJS = _f32(omlp.features(V)), _f32(omlp.js_weights_right(V))
    om = learned.forward(torch.from_numpy(_f32(theta)).cuda(), torch.from_numpy(X).cuda(),
                         torch.from_numpy(OJS).cuda()).cpu().numpy()
    ref, _ = omlp.forward(_f32(theta).astype(np.float64), X.astype(np.float64), OJS.astype(np.float64))
    np.testing.assert_allclose(om, ref, rtol=0, atol=2e-6)


@pytest.mark.parametrize("n", [64, 1000, 4099])
def test_forward_mfma_matches_bf16_oracle(n):
    from paper_2409_10729_amd import learned

    theta = omlp.init_params(12, out_scale=0.5)
    V = _stencils(n, 2)
    X, OJS = _f32(omlp.features(V)), _f32(omlp.js_weights_right(V))
    om = learned.forward(torch.from_numpy(_f32(theta)).cuda(), torch.from_numpy(X).cuda(),
                         torch.from_numpy(OJS).cuda(), packed=True).cpu().numpy()
    with np.errstate(divide="ignore"):
        ref = omlp.forward_bf16(theta, X.astype(np.float64), OJS.astype(np.float64))
    err = np.abs(om - ref).max()
    print(f"mfma forward n={n}: max |omega - bf16 oracle| = {err:.2e}", flush=True)
    assert err <= 5e-3
    np.testing.assert_allclose(om.sum(1), 1.0, atol=1e-5)


def _train_batch(n, seed):
    V = _stencils(n, seed)
    T = V[:, 2] + 0.3 * (V[:, 3] - V[:, 2]) * np.random.default_rng(seed).uniform(0, 1, n)
    return V, T


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_loss_grad_matches_oracle(lam):
    from paper_2409_10729_amd import learned

    V, T = _train_batch(2000, 3)
    feat, cand, tn, ojs = _prep(V, T)
    theta = omlp.init_params(5, out_scale=0.5).astype(np.float32)
    loss, grad, _ = learned.loss_grad(torch.from_numpy(theta).cuda(), feat, cand, tn, ojs, lam)
    L_ref, g_ref = omlp.loss_grad(theta.astype(np.float64), feat.cpu().numpy().astype(np.float64),
                                  cand.cpu().numpy().astype(np.float64), tn.cpu().numpy().astype(np.float64),
                                  ojs.cpu().numpy().astype(np.float64), lam)
    g = grad.cpu().numpy().astype(np.float64)
    assert float(loss.item()) == pytest.approx(L_ref, rel=1e-5)
    o = 0
    for name, size in (("W1", 160), ("b1", 32), ("W2", 1024), ("b2", 32), ("W3", 96), ("b3", 3)):
        e = np.linalg.norm(g[o:o + size] - g_ref[o:o + size]) / np.linalg.norm(g_ref[o:o + size])
        print(f"grad {name}: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-4, name
        o += size


def test_loss_grad_deterministic():
    from paper_2409_10729_amd import learned

    V, T = _train_batch(70000, 4)
    data = _prep(V, T)
    theta = torch.from_numpy(omlp.init_params(6, out_scale=0.5).astype(np.float32)).cuda()
    a = learned.loss_grad(theta, *data, 0.02)
    b = learned.loss_grad(theta, *data, 0.02)
    assert torch.equal(a[1], b[1]) and torch.equal(a[0], b[0])


def test_adam_step():
    from paper_2409_10729_amd import _native

    rng = np.random.default_rng(0)
    p0 = rng.normal(size=1347).astype(np.float32)
    g = rng.normal(size=1347).astype(np.float32)
    P, m, v, G = (torch.from_numpy(x).cuda() for x in (p0.copy(), np.zeros(1347, np.float32),
                                                        np.zeros(1347, np.float32), g))
    _native.check_mlp(_native.lib().mfx_mlp_adam(ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                                 ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(G.data_ptr()), 1,
                                                 ctypes.c_float(1e-2), None))
    torch.cuda.synchronize()
    # first Adam step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    ref = p0 - 1e-2 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(P.cpu().numpy(), ref, rtol=1e-5, atol=1e-7)


def test_short_training_lowers_loss():
    from paper_2409_10729_amd import learned

    data = learned.build_dataset([0, 1], [1000, 1001], log=lambda *_: None)[:4]
    params, hist = learned.train(data, epochs=3, batch=16384, log=lambda *_: None)
    print("validation losses", hist, flush=True)
    assert hist[-1] < hist[0]
    assert np.all(np.isfinite(params.cpu().numpy()))


def _solver(P, weights, params=None):
    from paper_2409_10729_amd import Solver

    s = Solver(P["spec"], precision=MFX_FP32_MIXED, weights=weights)
    if params is not None:
        s.set_mlp(torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda())
    s.set_primitive(torch.from_numpy(P["w"]).cuda())
    return s


def test_finetune_minimises_a_quadratic():
    """The evolution-strategies estimate plus Adam drives a known quadratic
    in the output-layer parameters down (the solver objective is replaced
    by a closed-form one, so this checks the optimiser alone)."""
    from paper_2409_10729_amd import learned

    lo, hi = learned.OUT_LAYER
    target = torch.from_numpy(np.random.default_rng(3).normal(0, 0.3, hi - lo).astype(np.float32)).cuda()

    def objective(p):
        return float(((p[lo:hi] - target) ** 2).sum().item())

    p0 = torch.from_numpy(learned.init_params(0)).cuda()
    best, hist = learned.finetune(p0, objective, iters=40, pairs=8, sigma=0.05, lr=0.02, log=lambda *_: None)
    print("quadratic objective", hist[0], "->", min(hist), flush=True)
    assert min(hist) < 0.3 * hist[0]
    assert torch.equal(best[:lo], p0[:lo])  # only the output layer moves


def test_zero_output_layer_reproduces_js_run():
    """A network whose output layer is zero gives the Jiang-Shu weights
    (through the log/exp form), so the learned run tracks the JS run to
    float32 rounding."""
    from paper_2409_10729_amd import learned

    P = wl.shock_droplet(n=(40, 24, 20), seed=2)
    zero = learned.init_params(1)
    s_l = _solver(P, MFX_WENO5_LEARNED, zero)
    s_j = _solver(P, MFX_WENO5_JS)
    for _ in range(3):
        s_l.rk3_step(2e-7)
        s_j.rk3_step(2e-7)
    d = rel_linf(s_l.get_state().cpu().numpy(), s_j.get_state().cpu().numpy())
    print("zero output layer vs JS:", d, flush=True)
    assert np.all(d <= 1e-4)


def test_uniform_state_skips_the_network():
    """A uniform state makes every stencil constant, so every wave skips the
    network and every edge takes the cell value (any convex weights give
    it): with a network of NaNs nothing falls back and the right-hand side
    of both learned forms vanishes to float rounding, as the Jiang-Shu float
    form's does (the two x-boundary faces of a row come from a separate
    kernel, whose multiply-adds the compiler may fuse differently, so exact
    zeros are not guaranteed in float)."""
    n = (40, 24, 20)
    P = wl.random_smooth(n=n, seed=1, bc=((0, 0), (0, 0), (0, 0)))
    w = np.empty_like(P["w"])
    for v, val in enumerate((998.0, 0.0012, 12.0, -3.0, 0.5, 2.0e5, 0.999)):
        w[v] = val
    P = dict(P, w=w)
    scale = 998.0 * (12.0 ** 2) * n[0] + 2.0e5 * n[0]  # momentum flux over dx
    nan_net = np.full(omlp.N_PARAMS, np.nan, dtype=np.float32)
    r_j = _solver(P, MFX_WENO5_JS).rhs().cpu().numpy()
    assert np.abs(r_j).max() <= 1e-6 * scale
    for weights in (MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE):
        s = _solver(P, weights, nan_net)
        r_l = s.rhs().cpu().numpy()
        st = s.stats()
        print(f"uniform state, weights {weights}: max |rhs| = {np.abs(r_l).max():.3e}, "
              f"fallback edges {st['fallback_faces']}", flush=True)
        assert st["fallback_faces"] == 0 and st["error"] == 0
        assert np.all(np.isfinite(r_l))
        assert np.abs(r_l).max() <= 1e-6 * scale


@pytest.mark.parametrize("nx", [72, 600])
def test_learned_x_sweep_variants_agree(monkeypatch, nx):
    """Learned form: the whole-row and the marching x sweep take the same
    decisions and agree to float rounding (600-cell rows use the marching
    sweep in both settings)."""
    P = wl.shock_droplet(n=(nx, 20, 16), seed=3)
    params = omlp.init_params(4, out_scale=0.5)
    out = {}
    for mode in ("rows", "march"):
        monkeypatch.setenv("MFX_XSWEEP", mode)
        s = _solver(P, MFX_WENO5_LEARNED, params)
        for _ in range(2):
            s.rk3_step(2e-7)
        out[mode] = (s.get_state().cpu().numpy(), s.stats())
    d = rel_linf(out["rows"][0], out["march"][0])
    print(f"learned x variants nx={nx}:", d, out["rows"][1]["fallback_faces"], out["march"][1]["fallback_faces"],
          flush=True)
    assert np.all(d <= 1e-4)
    assert out["rows"][1]["error"] == 0 and out["march"][1]["error"] == 0


def test_learned_needs_a_network():
    from paper_2409_10729_amd import MfxError

    P = wl.shock_tube(n=64)
    s = _solver(P, MFX_WENO5_LEARNED)
    with pytest.raises(MfxError):
        s.rk3_step(1e-8)


@pytest.mark.parametrize("maker", [lambda: wl.shock_tube(n=200), lambda: wl.shock_droplet(n=(40, 24, 20), seed=1)])
def test_nan_network_falls_back_everywhere(maker):
    P = maker()
    nan = np.full(1347, np.nan, dtype=np.float32)
    s_l = _solver(P, MFX_WENO5_LEARNED, nan)
    s_j = _solver(P, MFX_WENO5_JS)
    for _ in range(3):
        s_l.rk3_step(2e-7)
        s_j.rk3_step(2e-7)
    ql = s_l.get_state().cpu().numpy()
    qj = s_j.get_state().cpu().numpy()
    st = s_l.stats()
    assert st["fallback_faces"] > 0 and st["error"] == 0
    d = rel_linf(ql, qj)
    print("nan network vs JS:", d, "fallback edges", st["fallback_faces"], flush=True)
    assert np.all(d <= 1e-6)


TRAINED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2409_10729_amd", "data",
                       "mlp_weno5.npy")


def _l1(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())


@pytest.mark.skipif(not os.path.exists(TRAINED), reason="no trained network committed")
def test_gain_shock_tube():
    """1000-cell water|air tube, 300 CFL steps: L1 error of density, velocity
    and pressure against the exact two-material Riemann solution."""
    params = np.load(TRAINED, allow_pickle=False)
    P = wl.shock_tube()
    g = oracle.make_grid(P["spec"])
    errs = {}
    for name, weights, prm in (("js", MFX_WENO5_JS, None), ("learned", MFX_WENO5_LEARNED, params)):
        s = _solver(P, weights, prm)
        t = sum(s.rk3_step(sync=True) for _ in range(300))
        w = oracle.cons_to_prim(g, s.get_state().cpu().numpy()).reshape(7, -1)
        x = (np.arange(1000) + 0.5) / 1000
        re, ue, pe, _ = er.sample(er.Side(1000.0, 0, 1e9, 4.4, 6e8), er.Side(50.0, 0, 1e5, 1.4, 0.0), (x - 0.5) / t)
        errs[name] = (_l1(w[0] + w[1], re), np.abs(w[2] - ue).mean() / np.abs(ue).max(), _l1(w[5], pe))
        if name == "learned":
            print("fallback edges", s.stats()["fallback_faces"], flush=True)
    print("shock tube L1 (rho, u, p):", errs, flush=True)
    js, ln = np.array(errs["js"]), np.array(errs["learned"])
    assert np.sum(ln) < np.sum(js)


@pytest.mark.skipif(not os.path.exists(TRAINED), reason="no trained network committed")
def test_gain_advected_slab():
    """Held-out advected slab (seed outside the training range): L1 error of
    alpha1 against the exact translated profile after 200 steps."""
    params = np.load(TRAINED, allow_pickle=False)
    P = wl.advected_slab(n=256, seed=7777)
    errs = {}
    for name, weights, prm in (("js", MFX_WENO5_JS, None), ("learned", MFX_WENO5_LEARNED, params)):
        s = _solver(P, weights, prm)
        t = sum(s.rk3_step(sync=True) for _ in range(200))
        q = s.get_state().cpu().numpy().reshape(7, -1)
        errs[name] = _l1(q[6], P["alpha_cell_avg"](t))
    print("advected slab alpha1 L1:", errs, flush=True)
    assert errs["learned"] < errs["js"]


# ---- shared (per-edge) form

def _edge_set(ncell, seed):
    """A 1D sample set in the layout of mfx_mlp_sample_stencils:
    stencil (side*7 + v)*ncell + i, with flat variables and far targets mixed in."""
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(2, 7, ncell, 5)) * rng.uniform(0.01, 100.0, size=(2, 7, ncell, 1))
    V[:, 3, ::3, :] = 4.0  # flat
    V[:, 5, 1::5, 3:] += 50.0  # jumps
    T = V[..., 2] + (V[..., 3] - V[..., 2]) * rng.uniform(-0.5, 0.8, size=V.shape[:3])
    T[:, 6, ::7] += 1e4  # far off: dropped per variable
    return V, T


def _edge_oracle(V, T, tmax=2.0):
    ncell = V.shape[2]
    S = np.transpose(V, (0, 2, 1, 3)).reshape(2 * ncell, 7, 5)  # sample j = side*ncell + i
    Tj = np.transpose(T, (0, 2, 1)).reshape(2 * ncell, 7)
    f, B = omlp.edge_inputs(S)
    sc = S.max(axis=2) - S.min(axis=2)
    inv = np.where(sc > 0, 1.0 / np.where(sc > 0, sc, 1.0), 0.0)
    C = (omlp.candidates_right(S) - S[:, :, 2:3]) * inv[:, :, None]
    t = (Tj - S[:, :, 2]) * inv
    off = ~(np.abs(t) <= tmax)
    C[off] = 0.0
    t[off] = 0.0
    return f, C, t, B


def test_edge_features_match_oracle():
    from paper_2409_10729_amd import learned

    V, T = _edge_set(500, 0)
    st = torch.from_numpy(np.ascontiguousarray(V.reshape(-1, 5))).cuda()
    tg = torch.from_numpy(np.ascontiguousarray(T.reshape(-1))).cuda()
    feat, cand, tn, base = (x.cpu().numpy().astype(np.float64) for x in learned.features_edge(st, tg))
    f, C, t, B = _edge_oracle(V, T)
    np.testing.assert_allclose(feat, f, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(base, B, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(cand, C, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(tn, t, rtol=1e-6, atol=1e-6)
    assert np.count_nonzero(C[:, 3]) < C[:, 3].size and np.count_nonzero(t[:, 6] == 0) > 0


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_edge_loss_grad_matches_oracle(lam):
    from paper_2409_10729_amd import learned

    V, T = _edge_set(700, 1)
    st = torch.from_numpy(np.ascontiguousarray(V.reshape(-1, 5))).cuda()
    tg = torch.from_numpy(np.ascontiguousarray(T.reshape(-1))).cuda()
    feat, cand, tn, base = learned.features_edge(st, tg)
    theta = omlp.init_params(7, out_scale=0.5).astype(np.float32)
    loss, grad, _ = learned.loss_grad(torch.from_numpy(theta).cuda(), feat, cand, tn, base, lam)
    L_ref, g_ref = omlp.loss_grad(theta.astype(np.float64), *(x.cpu().numpy().astype(np.float64)
                                                                for x in (feat, cand, tn, base)), lam)
    assert float(loss.item()) == pytest.approx(L_ref, rel=1e-5)
    g = grad.cpu().numpy().astype(np.float64)
    o = 0
    for name, size in (("W1", 160), ("b1", 32), ("W2", 1024), ("b2", 32), ("W3", 96), ("b3", 3)):
        e = np.linalg.norm(g[o:o + size] - g_ref[o:o + size]) / np.linalg.norm(g_ref[o:o + size])
        print(f"edge grad {name}: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-4, name
        o += size


def test_edge_form_nan_network_falls_back_and_uniform_state_skips():
    P = wl.shock_droplet(n=(40, 24, 20), seed=1)
    nan = np.full(1347, np.nan, dtype=np.float32)
    s_e = _solver(P, MFX_WENO5_LEARNED_EDGE, nan)
    s_j = _solver(P, MFX_WENO5_JS)
    for _ in range(3):
        s_e.rk3_step(2e-7)
        s_j.rk3_step(2e-7)
    st = s_e.stats()
    d = rel_linf(s_e.get_state().cpu().numpy(), s_j.get_state().cpu().numpy())
    print("edge form, nan network vs JS:", d, "fallback edges", st["fallback_faces"], flush=True)
    assert st["fallback_faces"] > 0 and st["error"] == 0 and np.all(d <= 1e-6)
    # (the uniform state, where the network is skipped, for both forms:
    # test_uniform_state_skips_the_network)


EDGE_TRAINED = os.path.join(os.path.dirname(TRAINED), "mlp_weno5_edge.npy")


@pytest.mark.skipif(not os.path.exists(EDGE_TRAINED), reason="no trained shared network committed")
def test_edge_gain_shock_tube():
    """Shared form on the held-out 1000-cell tube: L1 of density, velocity and
    pressure against the exact solution below the Jiang-Shu form's."""
    params = np.load(EDGE_TRAINED, allow_pickle=False)
    P = wl.shock_tube()
    g = oracle.make_grid(P["spec"])
    errs = {}
    for name, weights, prm in (("js", MFX_WENO5_JS, None), ("edge", MFX_WENO5_LEARNED_EDGE, params)):
        s = _solver(P, weights, prm)
        t = sum(s.rk3_step(sync=True) for _ in range(300))
        w = oracle.cons_to_prim(g, s.get_state().cpu().numpy()).reshape(7, -1)
        x = (np.arange(1000) + 0.5) / 1000
        re, ue, pe, _ = er.sample(er.Side(1000.0, 0, 1e9, 4.4, 6e8), er.Side(50.0, 0, 1e5, 1.4, 0.0), (x - 0.5) / t)
        errs[name] = (_l1(w[0] + w[1], re), np.abs(w[2] - ue).mean() / np.abs(ue).max(), _l1(w[5], pe))
    print("edge form, shock tube L1 (rho, u, p):", errs, flush=True)
    assert np.sum(errs["edge"]) < np.sum(errs["js"])


@pytest.mark.skipif(not os.path.exists(EDGE_TRAINED), reason="no trained shared network committed")
def test_edge_gain_advected_slab():
    params = np.load(EDGE_TRAINED, allow_pickle=False)
    P = wl.advected_slab(n=256, seed=7777)
    errs = {}
    for name, weights, prm in (("js", MFX_WENO5_JS, None), ("edge", MFX_WENO5_LEARNED_EDGE, params)):
        s = _solver(P, weights, prm)
        t = sum(s.rk3_step(sync=True) for _ in range(200))
        q = s.get_state().cpu().numpy().reshape(7, -1)
        errs[name] = _l1(q[6], P["alpha_cell_avg"](t))
    print("edge form, advected slab alpha1 L1:", errs, flush=True)
    assert errs["edge"] < errs["js"]
