"""Pins for the learned-weights oracle (oracle/mlp.py): the backward pass
against central finite differences, closed-form special cases (zero output
layer gives uniform weights, softmax rows sum to one), the feature map's
invariances, and its smoothness indicators against the C oracle's."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import mlp


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(n, 5)) * rng.uniform(0.1, 3.0, size=(n, 1))
    V[::4, 3:] += 5.0  # a few steps
    X = mlp.features(V)
    C = mlp.candidates_right(V)
    c2 = V[:, 2:3]
    sc = V.max(axis=1, keepdims=True) - V.min(axis=1, keepdims=True)
    Cn = (C - c2) / sc
    T = rng.normal(size=n) * 0.3
    OJS = mlp.js_weights_right(V)
    return X, Cn, T, OJS


@pytest.mark.parametrize("lam", [0.0, 0.1])
def test_backward_matches_finite_differences(lam):
    X, C, T, OJS = _data()
    theta = mlp.init_params(3, out_scale=0.3)
    L, g = mlp.loss_grad(theta, X, C, T, OJS, lam)
    assert L == pytest.approx(mlp.loss(theta, X, C, T, OJS, lam), rel=1e-14)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (mlp.loss(tp, X, C, T, OJS, lam) - mlp.loss(tm, X, C, T, OJS, lam)) / (2 * h)
    o = 0
    for name, size in (("W1", 160), ("b1", 32), ("W2", 1024), ("b2", 32), ("W3", 96), ("b3", 3)):
        a, b = g[o:o + size], fd[o:o + size]
        o += size
        assert np.linalg.norm(a - b) <= 1e-6 * max(np.linalg.norm(b), 1e-12), name


def test_zero_output_layer_gives_js_weights():
    X, _, _, OJS = _data()
    om, _ = mlp.forward(mlp.init_params(1), X, OJS)
    np.testing.assert_allclose(om, OJS, rtol=1e-12, atol=1e-300)


def test_uniform_logits_give_uniform_weights():
    """Equal Jiang-Shu weights and a zero output layer: omega = (1/3,1/3,1/3)."""
    X, _, _, _ = _data()
    om, _ = mlp.forward(mlp.init_params(1), X, np.full((X.shape[0], 3), 0.25))
    assert np.array_equal(om, np.full_like(om, 1.0 / 3.0))


def test_softmax_rows_are_convex():
    X, _, _, OJS = _data(200, 5)
    om, _ = mlp.forward(mlp.init_params(7, out_scale=1.0), X, OJS)
    assert np.all(om > 0)
    np.testing.assert_allclose(om.sum(axis=1), 1.0, rtol=1e-15)


def test_gelu_limits():
    x = np.array([-40.0, -10.0, 0.0, 10.0, 40.0])
    g = mlp.gelu(x)
    assert g[2] == 0.0 and g[3] == pytest.approx(10.0) and g[4] == 40.0
    assert abs(g[0]) < 1e-300 and abs(g[1]) < 1e-20


def test_features_scale_shift_and_mirror():
    rng = np.random.default_rng(4)
    V = rng.normal(size=(50, 5)) * 100.0
    X = mlp.features(V, eps=1e-40)
    X2 = mlp.features(7.5 * V + 3.0, eps=1e-40)
    np.testing.assert_allclose(X2, X, rtol=1e-9, atol=1e-12)
    Xm = mlp.features(V[:, ::-1], eps=1e-40)
    np.testing.assert_allclose(Xm, X[:, [2, 1, 0, 3, 4]], rtol=1e-9, atol=1e-12)
    assert np.all((X >= 0) & (X <= 1))


def test_betas_agree_with_c_oracle():
    rng = np.random.default_rng(9)
    for _ in range(20):
        v = rng.normal(size=5) * rng.uniform(0.01, 1e4)
        np.testing.assert_allclose(mlp.betas(v), oracle.weno5_betas(v), rtol=1e-13, atol=1e-300)


def test_js_weights_reproduce_weno_right_edge():
    rng = np.random.default_rng(10)
    for _ in range(20):
        v = rng.normal(size=5)
        om = mlp.js_weights_right(v)
        val = (om * mlp.candidates_right(v)).sum()
        assert val == pytest.approx(oracle.weno5(v)[1], rel=1e-13, abs=1e-14)


def test_bf16_round():
    # bfloat16 spacing at 1 is 2^-7: 1 + 2^-8 is a tie (to even: 1), 1 + 2^-8 + 2^-10 rounds up
    x = np.array([1.0, 1.0 + 2 ** -8 + 2 ** -10, 1.0 + 2 ** -8, -3.5, 1e-3])
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0078125 and r[2] == 1.0
    assert r[3] == -3.5
    assert abs(r[4] - 1e-3) / 1e-3 < 2 ** -8


# ---- shared (per-edge) form

def _edge_data(n=30, nv=7, seed=0):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(n, nv, 5)) * rng.uniform(0.1, 3.0, size=(n, nv, 1))
    V[::3, 2, 3:] += 5.0
    V[1::4, 4, :] = 1.5  # flat variables
    f, B = mlp.edge_inputs(V)
    C = mlp.candidates_right(V)
    sc = V.max(axis=2, keepdims=True) - V.min(axis=2, keepdims=True)
    Cn = np.where(sc > 0, (C - V[:, :, 2:3]) / np.where(sc > 0, sc, 1.0), 0.0)
    T = rng.normal(size=(n, nv)) * 0.3
    return f, Cn, T, B


def test_edge_inputs_of_identical_variables_are_the_single_variable_ones():
    rng = np.random.default_rng(4)
    V1 = rng.normal(size=(50, 5)) * 2.0
    f, B = mlp.edge_inputs(np.repeat(V1[:, None, :], 7, axis=1))
    np.testing.assert_array_equal(f, mlp.features(V1))
    for v in range(7):
        np.testing.assert_allclose(B[:, v], mlp.js_weights_right(V1), rtol=1e-15)


def test_edge_inputs_pool_features_by_max_and_keep_each_baseline():
    """Features are the componentwise maxima; each variable keeps its own
    Jiang-Shu weights as the baseline; flat variables contribute zero
    features and the linear weights (1/10, 6/10, 3/10)."""
    rng = np.random.default_rng(5)
    V = rng.normal(size=(40, 3, 5))
    V[:, 1, :] = 7.0  # flat
    f, B = mlp.edge_inputs(V)
    X = np.stack([mlp.features(V[:, v]) for v in range(3)], axis=1)
    W = np.stack([mlp.js_weights_right(V[:, v]) for v in range(3)], axis=1)
    assert np.array_equal(X[:, 1], np.zeros((40, 5)))
    np.testing.assert_allclose(W[:, 1], np.broadcast_to([0.1, 0.6, 0.3], (40, 3)), rtol=1e-12)
    np.testing.assert_array_equal(f, np.maximum(np.maximum(X[:, 0], X[:, 1]), X[:, 2]))
    np.testing.assert_array_equal(B, W)
    # mirrored edge: the reversed stencils swap beta0 and beta2
    fm, _ = mlp.edge_inputs(V[:, :, ::-1])
    np.testing.assert_allclose(fm, f[:, [2, 1, 0, 3, 4]], rtol=1e-15)


def test_shared_logits_correct_each_variable():
    """Shared form: a zero output layer gives every variable its own
    Jiang-Shu weights; logits from the last bias b alone give each variable
    softmax(log omega_JS,v + b)."""
    rng = np.random.default_rng(6)
    V = rng.normal(size=(30, 7, 5)) * rng.uniform(0.1, 10.0, size=(30, 7, 1))
    f, B = mlp.edge_inputs(V)
    om, _ = mlp.forward(mlp.init_params(2), f, B)
    np.testing.assert_allclose(om, B, rtol=1e-14)
    p = mlp.unpack(mlp.init_params(2))
    p["b3"] = np.array([0.7, -0.2, 0.4])
    om, _ = mlp.forward(mlp.pack(p), f, B)
    e = B * np.exp(p["b3"])
    np.testing.assert_allclose(om, e / e.sum(axis=2, keepdims=True), rtol=1e-14)


def test_single_variable_loss_is_the_one_variable_case():
    X, C, T, OJS = _data()
    theta = mlp.init_params(3, out_scale=0.3)
    a = mlp.loss_grad(theta, X, C, T, OJS, 0.05)
    b = mlp.loss_grad(theta, X, C[:, None, :], T[:, None], OJS, 0.05)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("lam", [0.0, 0.1])
def test_shared_backward_matches_finite_differences(lam):
    X, C, T, OJS = _edge_data()
    theta = mlp.init_params(6, out_scale=0.3)
    L, g = mlp.loss_grad(theta, X, C, T, OJS, lam)
    assert L == pytest.approx(mlp.loss(theta, X, C, T, OJS, lam), rel=1e-14)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (mlp.loss(tp, X, C, T, OJS, lam) - mlp.loss(tm, X, C, T, OJS, lam)) / (2 * h)
    o = 0
    for name, size in (("W1", 160), ("b1", 32), ("W2", 1024), ("b2", 32), ("W3", 96), ("b3", 3)):
        a, b = g[o:o + size], fd[o:o + size]
        o += size
        assert np.linalg.norm(a - b) <= 1e-6 * max(np.linalg.norm(b), 1e-12), name


def test_calibration_scales_the_correction(tmp_path):
    """learned.calibrate scales the output layer; in the residual form the
    logits that correct log(omega_JS) scale by the same factor, so the
    calibrated weights are softmax(log omega_JS + s z)."""
    import shutil

    from paper_2409_10729_amd import learned

    src = learned.DEFAULT_PARAMS
    if not os.path.exists(src):
        pytest.skip("no trained network committed")
    dst = tmp_path / "net.npy"
    shutil.copy(src, dst)
    theta = np.load(dst).astype(np.float64)
    learned.calibrate(str(dst), 0.8, "test")
    theta_s = np.load(dst).astype(np.float64)
    rng = np.random.default_rng(5)
    V = rng.normal(size=(64, 5)) * rng.uniform(0.01, 10.0, size=(64, 1))
    X = np.stack([mlp.features(v) for v in V])
    ojs = np.stack([mlp.js_weights_right(v) for v in V])
    w1 = mlp.forward(theta, X, ojs)[0]
    w_s = mlp.forward(theta_s, X, ojs)[0]
    # z = log(omega) - log(omega_JS) up to a per-row constant
    z1 = np.log(w1) - np.log(ojs)
    zs = np.log(w_s) - np.log(ojs)
    z1 -= z1.mean(axis=1, keepdims=True)
    zs -= zs.mean(axis=1, keepdims=True)
    np.testing.assert_allclose(zs, 0.8 * z1, rtol=1e-5, atol=1e-6)
    meta = json.load(open(tmp_path / "net.json"))
    assert meta["calibration"][-1]["correction_scale"] == 0.8
