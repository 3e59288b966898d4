"""FP64 oracle for the learned WENO weights: features, MLP forward and
backward, loss.

TEST INFRASTRUCTURE ONLY (part of the oracle).

What it computes (the learned-weights form; the paper's WENO5 is Sec. II-B,
Shu 2006; the network is this project's addition):
  features of a 5-cell stencil v0..v4 reconstructed at its right edge, with
  the Jiang-Shu indicators beta_k and S = beta0 + beta1 + beta2 + eps:
      x = (beta0/S, beta1/S, beta2/S, |beta0 - beta2|/S, D^2/(S + D^2)),
      D = v0 - 4 v1 + 6 v2 - 4 v3 + v4;
  network 5 -> 32 (GELU) -> 32 (GELU) -> 3 logits z, added to the
  Jiang-Shu log-weights: omega = softmax(log omega_JS + z) (a zero output
  layer gives the Jiang-Shu weights exactly);
  value = sum_k omega_k p_k with the three third-order candidates p_k;
  loss  = mean((value' - target')^2) + lam * mean(sum_k (omega_k - omega_JS,k)^2),
  where primes are stencil-normalised: (. - v2) / scale.
GELU: training uses its tanh form (gelu, gelu_grad); the bfloat16 inference
forward uses gelu_inference, max(x, 0) minus a degree-7 polynomial fit of the
tanh form's remainder (within 1.2e-4 of the tanh form).
Parameters, flat float vector of 1347: W1[32][5], b1[32], W2[32][32], b2[32],
W3[3][32], b3[3].

Shared (per-edge) form: one evaluation serves all variables of an edge.  Its
input is the componentwise maximum over the variables of their features; its
logits z correct every variable's own Jiang-Shu weights,
omega_v = softmax(log omega_JS,v + z), so a zero output layer gives each
variable its Jiang-Shu weights exactly; the loss averages the squared
normalised error and the regulariser over the variables.  A left edge is the
right edge of the reversed stencils.
"""
from __future__ import annotations

import numpy as np

H = 32
N_PARAMS = H * 5 + H + H * H + H + 3 * H + 3  # 1347
GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    o = 0
    out = {}
    for name, shape in (("W1", (H, 5)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (3, H)), ("b3", (3,))):
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def betas(v):
    """Jiang-Shu smoothness indicators, v: [..., 5]."""
    v = np.asarray(v, dtype=np.float64)
    a, b, c, d, e = (v[..., i] for i in range(5))
    b0 = 13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    return np.stack([b0, b1, b2], axis=-1)


def candidates_right(v):
    """Third-order candidate values at the right edge of the middle cell."""
    v = np.asarray(v, dtype=np.float64)
    a, b, c, d, e = (v[..., i] for i in range(5))
    return np.stack([(2 * a - 7 * b + 11 * c) / 6.0, (-b + 5 * c + 2 * d) / 6.0, (2 * c + 5 * d - e) / 6.0], axis=-1)


def js_weights_right(v, eps=1e-6):
    bt = betas(v)
    alpha = np.array([0.1, 0.6, 0.3]) / (eps + bt) ** 2
    return alpha / alpha.sum(axis=-1, keepdims=True)


def features(v, eps=1e-6):
    v = np.asarray(v, dtype=np.float64)
    bt = betas(v)
    S = bt.sum(axis=-1) + eps
    D = v[..., 0] - 4 * v[..., 1] + 6 * v[..., 2] - 4 * v[..., 3] + v[..., 4]
    return np.stack([bt[..., 0] / S, bt[..., 1] / S, bt[..., 2] / S, np.abs(bt[..., 0] - bt[..., 2]) / S,
                     D * D / (S + D * D)], axis=-1)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


# Q(t) of gelu_inference, lowest degree first (float32 values)
GELU_Q = np.array([0.497150153, -0.375513077, -0.0665387958, 0.157749414, -0.0645674914, 0.0113088572,
                   -0.00075154379], dtype=np.float32).astype(np.float64)
GELU_T = 3.75


def gelu_inference(x):
    """GELU as the inference evaluates it: max(x, 0) - t Q(t), t = min(|x|, 3.75)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.minimum(np.abs(x), GELU_T)
    Q = np.zeros_like(t)
    tk = np.ones_like(t)
    for q in GELU_Q:
        Q = Q + q * tk
        tk = tk * t
    return np.maximum(x, 0.0) - t * Q


def gelu_grad(x):
    u = GELU_C * (x + GELU_A * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


def forward(theta, X, OJS):
    """omega and the intermediates.  OJS: Jiang-Shu weights [n, 3] (one
    variable per sample; omega [n, 3]) or [n, V, 3] (shared form: the
    sample's logits correct each of its V variables' weights; omega
    [n, V, 3])."""
    p = unpack(theta)
    A1 = X @ p["W1"].T + p["b1"]
    H1 = gelu(A1)
    A2 = H1 @ p["W2"].T + p["b2"]
    H2 = gelu(A2)
    Zn = H2 @ p["W3"].T + p["b3"]
    OJS = np.asarray(OJS, dtype=np.float64)
    Z = (Zn if OJS.ndim == 2 else Zn[:, None, :]) + np.log(OJS)
    Z = Z - Z.max(axis=-1, keepdims=True)
    E = np.exp(Z)
    om = E / E.sum(axis=-1, keepdims=True)
    return om, (X, A1, H1, A2, H2)


def _per_var(C, T, OJS):
    """Candidates [n,V,3], targets [n,V] and baselines [n,V,3] (a single
    variable may come as [n,3], [n]; a baseline [n,3] serves every variable
    of its sample)."""
    C = np.asarray(C, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    OJS = np.asarray(OJS, dtype=np.float64)
    if C.ndim == 2:
        C, T = C[:, None, :], T[:, None]
    if OJS.ndim == 2:
        OJS = np.broadcast_to(OJS[:, None, :], C.shape)
    return C, T, OJS


def _loss_terms(om, C, T, OJS, lam):
    om = om if om.ndim == 3 else om[:, None, :]
    r = (om * C).sum(axis=2) - T
    L = float(np.mean((r * r).mean(axis=1)) + lam * np.mean(((om - OJS) ** 2).sum(axis=2).mean(axis=1)))
    return om, r, L


def loss(theta, X, C, T, OJS, lam):
    """C: normalised candidates [n,3] or [n,V,3]; T: normalised targets [n] or
    [n,V]; OJS: baseline (Jiang-Shu) weights [n,3] or, per variable,
    [n,V,3].  Error term: the mean over samples of the mean over variables of
    the squared error; regulariser: lam times the mean over samples and
    variables of |omega - omega_JS|^2."""
    om, _ = forward(theta, X, OJS)
    C, T, OJS = _per_var(C, T, OJS)
    return _loss_terms(om, C, T, OJS, lam)[2]


def loss_grad(theta, X, C, T, OJS, lam):
    """(loss, d loss / d theta) by reverse-mode differentiation."""
    p = unpack(theta)
    om, (X, A1, H1, A2, H2) = forward(theta, X, OJS)
    C, T, OJS = _per_var(C, T, OJS)
    n, nv = X.shape[0], C.shape[1]
    om, r, L = _loss_terms(om, C, T, OJS, lam)
    dom = (2.0 / (n * nv)) * (r[:, :, None] * C) + (2.0 * lam / (n * nv)) * (om - OJS)
    # softmax backward per variable; the variables share the logits
    dZ = (om * (dom - (dom * om).sum(axis=2, keepdims=True))).sum(axis=1)
    g = {}
    g["W3"] = dZ.T @ H2
    g["b3"] = dZ.sum(axis=0)
    dH2 = dZ @ p["W3"]
    dA2 = dH2 * gelu_grad(A2)
    g["W2"] = dA2.T @ H1
    g["b2"] = dA2.sum(axis=0)
    dH1 = dA2 @ p["W2"]
    dA1 = dH1 * gelu_grad(A1)
    g["W1"] = dA1.T @ X
    g["b1"] = dA1.sum(axis=0)
    return L, pack(g)


def edge_inputs(V, eps=1e-6):
    """Shared form: V [n, V, 5] holds every variable's stencil at one edge
    (right edge; pass the reversed stencils for a left edge).  Returns the
    pooled features [n,5] (maximum over the variables) and the variables'
    own Jiang-Shu weights [n,V,3], the baselines the shared logits correct."""
    V = np.asarray(V, dtype=np.float64)
    return features(V, eps).max(axis=1), js_weights_right(V, eps)


def init_params(seed=0, out_scale=0.0):
    """He-style hidden layers; output layer zero (omega = omega_JS) unless
    out_scale > 0, which draws it with that standard deviation."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, np.sqrt(2.0 / 5), (H, 5)),
        "b1": np.zeros(H),
        "W2": rng.normal(0, np.sqrt(2.0 / H), (H, H)),
        "b2": np.zeros(H),
        "W3": rng.normal(0, out_scale, (3, H)) if out_scale > 0 else np.zeros((3, H)),
        "b3": np.zeros(3),
    }
    return pack(p)


def forward_bf16(theta, X, OJS):
    """omega [n, 3] with the network evaluated as the solver's matrix cores
    do: bfloat16 features, weights of all three layers, first-layer bias and
    hidden activations (each rounded through float32, nearest, ties to
    even); second- and third-layer biases as given (float32 values); sums,
    softmax and everything else in float64."""
    p = unpack(np.asarray(theta, dtype=np.float32).astype(np.float64))
    r = bf16_round
    A1 = r(X) @ r(p["W1"]).T + r(p["b1"])
    H1 = r(gelu_inference(A1))
    A2 = H1 @ r(p["W2"]).T + p["b2"]
    H2 = r(gelu_inference(A2))
    with np.errstate(divide="ignore"):
        Z = H2 @ r(p["W3"]).T + p["b3"] + np.log(OJS)
    Z = Z - Z.max(1, keepdims=True)
    E = np.exp(Z)
    return E / E.sum(1, keepdims=True)


def bf16_round(x):
    """Round float64 values to bfloat16 (via float32, round to nearest even)."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
