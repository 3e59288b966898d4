"""Pins of the oracle's learned-weights right-hand side (oracle.rhs_learned:
the learned WENO weights as the solver applies them -- per-edge features,
the left edge as the reversed stencil's right edge, the network with
bfloat16 operands, omega = softmax(ln omega_JS + z), the shared per-edge
pooling and the per-edge Jiang-Shu fallback).

What fixes each part without an implementation to compare with:
  * GELU: the training form (tanh form) approximates x Phi(x) to 5e-4
    (Hendrycks & Gimpel's approximation; wrong constants miss by 3e-3 or
    more); the inference form (positive part minus a polynomial remainder)
    stays within 1.2e-4 of the tanh form evaluated here with math.tanh, at
    interior points and over [-20, 20] (a wrong coefficient or clamp misses
    by 1e-3 or more); both satisfy GELU(x) - GELU(-x) = x;
  * the network: the C evaluation equals the numpy one of oracle.mlp (whose
    backward pass is pinned by finite differences); a zero output layer
    returns the baseline; logits from the last bias alone give the closed
    softmax;
  * a zero output layer reproduces the Jiang-Shu right-hand side in both
    forms; a network whose logits are its last bias alone (no dependence on
    the features) gives the same right-hand side in both forms, since the
    shared logits correct each variable's own Jiang-Shu weights; on a state
    whose seven primitives are affine images of one profile (identical
    features and weights in every variable) the two forms agree for any
    network;
  * a network of NaNs makes every edge fall back: the Jiang-Shu right-hand
    side bit for bit, with the closed-form count of edges;
  * mirror symmetry (the left edge is the reversed stencil's right edge),
    conservation on periodic grids, direction symmetry;
  * planted mistakes (in the oracle, on the CPU) move the result by far more
    than the GPU comparison's tolerance on its test problems.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2409_10729_amd import workloads as wl
from parity_util import flux_scale, learned_reference, learned_tolerance

PER_VAR, SHARED = oracle.LEARNED_PER_VARIABLE, oracle.LEARNED_SHARED


def _q0(P):
    g = oracle.make_grid(P["spec"])
    return g, oracle.prim_to_cons(g, P["w"])


def _rel(a, b, spec, q0):
    return np.abs(a - b).reshape(7, -1).max(axis=1) / flux_scale(q0, spec)


def _gelu_tanh_here(v):
    return 0.5 * v * (1.0 + math.tanh(math.sqrt(2.0 / math.pi) * (v + 0.044715 * v ** 3)))


def test_gelu_approximates_x_phi():
    x = np.linspace(-8, 8, 4001)
    exact = np.array([v * 0.5 * (1.0 + math.erf(v / math.sqrt(2.0))) for v in x])
    g = np.array([oracle.gelu_tanh(v) for v in x])
    assert np.abs(g - exact).max() <= 5e-4
    np.testing.assert_allclose(g - np.array([oracle.gelu_tanh(-v) for v in x]), x, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g, omlp.gelu(x), rtol=0, atol=1e-14)
    np.testing.assert_allclose(g, [_gelu_tanh_here(v) for v in x], rtol=0, atol=1e-15)
    for v in (-1.0, -0.5, 0.5, 1.0):
        assert abs(oracle.gelu_tanh(v) - v * 0.5 * (1.0 + math.erf(v / math.sqrt(2.0)))) <= 5e-4


def test_inference_gelu_tracks_the_tanh_form():
    """The inference GELU against the tanh form computed here: within
    1.2e-4 everywhere (about 1/30 of a bfloat16 step at 1), the odd-part
    identity exactly, the positive part beyond the clamp, and the numpy and
    C evaluations alike."""
    x = np.concatenate([np.linspace(-20, 20, 16001), [-3.75, 3.75, -1.0, -0.5, 0.5, 1.0, 0.0]])
    g = np.array([oracle.gelu(v) for v in x])
    ref = np.array([_gelu_tanh_here(v) for v in x])
    assert np.abs(g - ref).max() <= 1.2e-4
    for v in (-1.0, -0.5, 0.5, 1.0):
        assert abs(oracle.gelu(v) - _gelu_tanh_here(v)) <= 1.2e-4
        assert abs(oracle.gelu(v) - v * 0.5 * (1.0 + math.erf(v / math.sqrt(2.0)))) <= 6e-4
    np.testing.assert_allclose(g - np.array([oracle.gelu(-v) for v in x]), x, rtol=0, atol=1e-14)
    assert oracle.gelu(0.0) == 0.0
    # beyond the clamp: x minus a constant for x > 3.75, the same constant below -3.75
    tail = oracle.gelu(10.0) - 10.0
    assert abs(tail) <= 1.2e-4
    assert oracle.gelu(25.0) - 25.0 == pytest.approx(tail, abs=1e-14)
    assert oracle.gelu(-10.0) == pytest.approx(tail, abs=1e-15)
    np.testing.assert_allclose(omlp.gelu_inference(x), g, rtol=0, atol=1e-15)


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(n, 5)) * rng.uniform(0.01, 1e3, size=(n, 1))
    return omlp.features(V), omlp.js_weights_right(V)


def test_c_network_equals_numpy_network():
    X, OJS = _samples(3000, 0)
    for seed in (1, 2):
        theta = omlp.init_params(seed, out_scale=0.7).astype(np.float32)
        a = oracle.mlp_omega(theta, X, OJS)
        b = omlp.forward_bf16(theta, X, OJS)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
        np.testing.assert_allclose(a.sum(1), 1.0, atol=1e-14)


def test_network_closed_forms():
    X, OJS = _samples(500, 3)
    zero = omlp.init_params(4)  # output layer zero
    np.testing.assert_allclose(oracle.mlp_omega(zero, X, OJS), OJS, rtol=1e-13, atol=0)
    p = omlp.unpack(zero)
    p["b3"] = np.array([1.5, -0.5, 0.25])
    th = omlp.pack(p).astype(np.float32)
    e = OJS * np.exp(p["b3"].astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(oracle.mlp_omega(th, X, OJS), e / e.sum(1, keepdims=True), rtol=1e-13, atol=0)


PROBLEMS = {
    "smooth": lambda: wl.random_smooth(n=(24, 20, 16), seed=1, bc=((1, 1), (0, 0), (0, 0))),
    "droplet": lambda: wl.shock_droplet(n=(40, 24, 20), seed=2),
    "tube": lambda: wl.shock_tube(n=200),
}


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_zero_output_layer_is_jiang_shu(name, mode):
    P = PROBLEMS[name]()
    g, q0 = _q0(P)
    r, fb, _ = oracle.rhs_learned(g, q0, omlp.init_params(5), mode)
    assert np.all(_rel(r, oracle.rhs(g, q0), P["spec"], q0) <= 1e-13)


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_feature_free_logits_agree_in_both_forms(name):
    """Logits from the last bias alone are the same on every edge and
    variable, so the shared form (its logits applied to each variable's own
    Jiang-Shu weights) equals the per-variable form."""
    P = PROBLEMS[name]()
    g, q0 = _q0(P)
    p = omlp.unpack(omlp.init_params(13))
    p["b3"] = np.array([0.6, -0.3, 0.2])
    th = omlp.pack(p).astype(np.float32)
    r1, fb1, _ = oracle.rhs_learned(g, q0, th, PER_VAR)
    r2, fb2, _ = oracle.rhs_learned(g, q0, th, SHARED)
    assert np.all(_rel(r2, r1, P["spec"], q0) <= 1e-13) and fb1 == fb2
    if name != "tube":  # (the tube's edges are flat or at a bare jump, where the bias barely acts)
        assert _rel(r1, oracle.rhs(g, q0), P["spec"], q0).max() > 1e-6  # the bias moves the result


def _affine_state(n=96):
    """1D state whose seven primitives are affine images of one profile f
    (a smoothed step plus a wave): every variable has the same normalised
    features and the same Jiang-Shu weights."""
    x = (np.arange(n) + 0.5) / n
    f = 0.5 * (1.0 + np.tanh((x - 0.4) / 0.03)) + 0.2 * np.sin(2 * np.pi * x)
    a1 = 0.2 + 0.6 * f
    w = np.stack([200 + 600 * f, 1.0 + 0.5 * f, 10 + 20 * f, 5 + 3 * f, -2 + f, 1e5 * (1.0 + f), a1])
    spec = wl.spec((n, 1, 1), ((1, 1), (0, 0), (0, 0)))
    spec = dict(spec, eps=1e-40)  # no absolute epsilon: the weights are scale free
    return spec, w.reshape(7, 1, 1, n)


def test_shared_form_on_an_affine_state_is_the_per_variable_form():
    spec, w = _affine_state()
    g = oracle.make_grid(spec)
    q0 = oracle.prim_to_cons(g, w)
    th = omlp.init_params(6, out_scale=0.5)
    r, _, _ = oracle.rhs_learned(g, q0, th, SHARED)
    r1, _, _ = oracle.rhs_learned(g, q0, th, PER_VAR)
    assert np.all(_rel(r, r1, spec, q0) <= 1e-12)
    # and the network moves it (the form is live)
    assert _rel(r, oracle.rhs(g, q0), spec, q0).max() > 1e-6


def _edges(spec):
    n = spec["n"]
    N = n[0] * n[1] * n[2]
    tot = 0
    for d in range(3):
        if n[d] > 1:
            faces = n[d] if spec["bc"][d][0] == 0 else n[d] + 1
            tot += 2 * faces * (N // n[d])
    return tot


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_nan_network_falls_back_on_every_edge(name, mode):
    P = PROBLEMS[name]()
    g, q0 = _q0(P)
    r, fb, near = oracle.rhs_learned(g, q0, np.full(1347, np.nan), mode)
    assert np.array_equal(r, oracle.rhs(g, q0))
    assert fb == _edges(P["spec"]) and near == 0


def _mirror_x(q):
    m = q[:, :, :, ::-1].copy()
    m[2] = -m[2]
    return m


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
@pytest.mark.parametrize("plant", [0, 1])
def test_mirror_symmetry(mode, plant):
    """The x-mirror image of a state has the x-mirror image of its learned
    right-hand side: the left edge is the reversed stencil's right edge.
    Feeding the left edge the unreversed stencil's features (plant 1)
    breaks it."""
    P = wl.random_smooth(n=(40, 6, 5), seed=7, bc=((1, 1), (0, 0), (0, 0)))
    g, q0 = _q0(P)
    th = omlp.init_params(8, out_scale=0.5)
    r, _, _ = oracle.rhs_learned(g, q0, th, mode, plant)
    rm, _, _ = oracle.rhs_learned(g, _mirror_x(q0), th, mode, plant)
    err = _rel(_mirror_x(rm), r, P["spec"], q0)
    if plant == 0:
        assert np.all(err <= 1e-12), err
    else:
        assert err.max() > 1e-4, err


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
def test_conservation_on_a_periodic_grid(mode):
    P = wl.random_smooth(n=(20, 16, 12), seed=9)
    g, q0 = _q0(P)
    r, _, _ = oracle.rhs_learned(g, q0, omlp.init_params(10, out_scale=0.5), mode)
    sc = flux_scale(q0, P["spec"])
    tot = np.abs(r.reshape(7, -1).sum(axis=1)[:6]) / (sc[:6] * r[0].size)
    assert np.all(tot <= 1e-14), tot


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
def test_direction_symmetry(mode):
    """The same 1D problem along x, y or z gives the same right-hand side."""
    P = wl.shock_tube(n=64)
    g, q0 = _q0(P)
    th = omlp.init_params(11, out_scale=0.5)
    rx, fx, _ = oracle.rhs_learned(g, q0, th, mode)
    for d in (1, 2):
        n = [1, 1, 1]
        n[d] = 64
        bc = [(0, 0)] * 3
        bc[d] = P["spec"]["bc"][0]
        spec = dict(P["spec"], n=tuple(n), bc=tuple(bc), dx=(P["spec"]["dx"][0],) * 3)
        q = np.moveaxis(q0, 3, 3 - d).copy()
        q[[2, 2 + d]] = q[[2 + d, 2]]
        gd = oracle.make_grid(spec)
        rd, fd, _ = oracle.rhs_learned(gd, q, th, mode)
        rd[[2, 2 + d]] = rd[[2 + d, 2]]
        assert np.array_equal(np.moveaxis(rd, 3 - d, 3), rx) and fd == fx


def steered_params():
    """A network whose logits are its last bias alone, (40, -40, -40): the
    weights sit near (1, 0, 0), the most upwind candidate, which overshoots
    at jumps -- many edges fail the admissibility test and fall back."""
    p = omlp.unpack(omlp.init_params(12))
    p["b3"] = np.array([40.0, -40.0, -40.0])
    return omlp.pack(p).astype(np.float32)


def test_steered_network_falls_back_at_the_contact():
    P = PROBLEMS["tube"]()
    g, q0 = _q0(P)
    r, fb, near = oracle.rhs_learned(g, q0, steered_params(), PER_VAR)
    assert fb > 0
    print("steered network, tube: fallback edges", fb, "near", near, flush=True)


# planted mistake -> (mode, problem, network) where the GPU comparison would see it
PLANTS = {
    1: (PER_VAR, "droplet", "random"),   # left edge with the unreversed stencil's features
    2: (PER_VAR, "smooth", "zero"),      # left and right edges exchanged
    3: (PER_VAR, "droplet", "steered"),  # fallback per variable, not per edge
    4: (SHARED, "droplet", "random"),    # shared logits on one pooled baseline, not each variable's own
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistakes_exceed_the_gpu_tolerance(plant):
    from paper_2409_10729_amd import learned

    mode, name, net = PLANTS[plant]
    P = PROBLEMS[name]()
    g, q0 = _q0(P)
    th = {"random": omlp.init_params(4, out_scale=0.5), "zero": omlp.init_params(4),
          "trained": learned.load_params(learned.DEFAULT_PARAMS), "steered": steered_params()}[net]
    ref = learned_reference(P["spec"], q0, th, mode)
    bad, _, _ = oracle.rhs_learned(g, q0, th, mode, plant)
    err = _rel(bad, ref["rhs"], P["spec"], q0)
    tol = learned_tolerance(ref)
    print(f"plant {plant}: error/tolerance per field", np.round(err / tol, 1), flush=True)
    assert (err / tol).max() > 10.0


@pytest.mark.parametrize("mode", [PER_VAR, SHARED])
@pytest.mark.parametrize("name", ["smooth", "droplet", "walls"])
def test_cell_by_cell_learned_rhs_equals_the_whole_grid(name, mode):
    """rhs_learned_at (one cell at a time, the boundary rule applied to each
    stencil index) equals rhs_learned (padded grid, pencils) bit for bit at
    every cell, including those next to reflective and inflow sides."""
    if name == "walls":
        P = wl.shock_droplet_walls(n=(20, 12, 10), seed=5)
        g1 = oracle.make_grid(dict(P["spec"], n=(1, 1, 1), bc=((0, 0),) * 3))
        inflow = np.array([[oracle.prim_to_cons(g1, np.asarray(w7).reshape(7, 1, 1, 1)).reshape(7)
                            for w7 in pair] for pair in P["inflow_prim"]])
        P = dict(P, spec=dict(P["spec"], inflow=inflow))
    else:
        P = PROBLEMS[name]()
    g, q0 = _q0(P)
    th = omlp.init_params(14, out_scale=0.5)
    r, _, _ = oracle.rhs_learned(g, q0, th, mode)
    cells = np.arange(q0[0].size)
    ra = oracle.rhs_learned_at(g, q0, th, cells, mode)
    assert np.array_equal(ra.T, r.reshape(7, -1))
