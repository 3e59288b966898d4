"""Learned WENO weights: training data from the solver's own runs, and
training on the GPU through the library's forward/backward and Adam kernels.

Data (all generated here, seeded):
  * water|air shock tubes (``workloads.shock_tube_family``: interface
    U(0.3, 0.7), left pressure log-U(1e8, 1e9)) run with the FP64 solver on
    the coarse grid; the targets are the face values of the same problem run
    on a grid `refine` times finer with the coarse time steps split evenly
    (``mfx_mlp_face_targets``);
  * advected water slabs (``workloads.advected_slab``, u ~ U(100, 400) m/s),
    whose exact solution is the translated profile.
Every stored snapshot contributes, per cell and variable, the right-edge
stencil and the mirrored (left-edge) one (``mfx_mlp_sample_stencils``).
Flat stencils (max - min below 1e-6 of their magnitude: uniform regions and
rounding noise) carry no information and are dropped, and so are samples
whose normalised target lies more than twice the stencil's range away.

Network: logits that correct the Jiang-Shu weights,
omega = softmax(ln omega_JS + z); the output layer starts at zero, so
training starts from Jiang-Shu.

Training, two stages:
  1. minibatch Adam on the loss of ``mfx_mlp_loss_grad`` (squared
     stencil-normalised reconstruction error plus lam times the squared
     distance of the weights from Jiang-Shu's), cosine learning-rate decay,
     through the library's forward/backward kernels;
  2. fine-tuning of the output layer on what the reconstruction is for: the
     L1 error of whole solver runs (``SolutionObjective``) relative to the
     Jiang-Shu form's, with an evolution-strategies gradient estimate and
     the library's Adam kernel.  Stage 1 alone lowers the reconstruction
     loss yet leaves the solution error at or above Jiang-Shu's; stage 2 is
     what makes the learned form more accurate.

    python -m paper_2409_10729_amd.learned            # per-variable form
    python -m paper_2409_10729_amd.learned --edge     # shared per-edge form
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

from . import MFX_FP64, Solver, _native
from . import workloads as wl

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DEFAULT_PARAMS = os.path.join(DATA_DIR, "mlp_weno5.npy")  # per-variable form
EDGE_PARAMS = os.path.join(DATA_DIR, "mlp_weno5_edge.npy")  # shared per-edge form
N_PARAMS = _native.MLP_PARAMS
H = 32


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style hidden layers, zero biases and a zero output layer (the
    network starts as Jiang-Shu); layout W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, math.sqrt(2.0 / 5), H * 5), np.zeros(H), rng.normal(0, math.sqrt(2.0 / H), H * H),
             np.zeros(H), np.zeros(3 * H), np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


def load_params(path: str = DEFAULT_PARAMS) -> np.ndarray:
    p = np.load(path, allow_pickle=False).astype(np.float32)
    assert p.size == N_PARAMS
    return p


# ------------------------------------------------------------------ data

def _sample(spec, q_dev, face_prim_dev):
    """(stencils [14n, 5], targets [14n]) on the device for a 1D state."""
    import torch

    n = spec["n"][0]
    st = torch.empty((14 * n, 5), dtype=torch.float64, device="cuda")
    tg = torch.empty(14 * n, dtype=torch.float64, device="cuda")
    d = _native.make_desc(spec)
    _native.check_mlp(_native.lib().mfx_mlp_sample_stencils(ctypes.byref(d), _p(q_dev), _p(face_prim_dev), _p(st),
                                                            _p(tg), _stream()))
    return st, tg


def shock_tube_samples(seed: int, n: int = 500, refine: int = 8, steps: int = 150, every: int = 3):
    import torch

    Pc = wl.shock_tube_family(n=n, seed=seed)
    Pf = wl.shock_tube_family(n=n * refine, seed=seed)
    coarse = Solver(Pc["spec"], MFX_FP64)
    fine = Solver(Pf["spec"], MFX_FP64)
    coarse.set_primitive(torch.from_numpy(Pc["w"]).cuda())
    fine.set_primitive(torch.from_numpy(Pf["w"]).cuda())
    fd = _native.make_desc(Pf["spec"])
    face = torch.empty((7, n + 1), dtype=torch.float64, device="cuda")
    out = []
    for k in range(1, steps + 1):
        dt = coarse.rk3_step(sync=True)
        for _ in range(refine):
            fine.rk3_step(dt / refine)
        if k % every == 0:
            qf = fine.get_state()
            _native.check_mlp(_native.lib().mfx_mlp_face_targets(ctypes.byref(fd), _p(qf), refine, _p(face),
                                                                 _stream()))
            out.append(_sample(Pc["spec"], coarse.get_state(), face))
    return out


def slab_samples(seed: int, n: int = 256, steps: int = 120, every: int = 3):
    import torch

    P = wl.advected_slab(n=n, seed=seed)
    s = Solver(P["spec"], MFX_FP64)
    s.set_primitive(torch.from_numpy(P["w"]).cuda())
    t = 0.0
    out = []
    for k in range(1, steps + 1):
        t += s.rk3_step(sync=True)
        if k % every == 0:
            face = torch.from_numpy(np.ascontiguousarray(P["face_prims"](t))).cuda()
            out.append(_sample(P["spec"], s.get_state(), face))
    return out


def features(stencils, targets, eps: float = 1e-6):
    """Device tensors feat [m,5], cand [m,3], tnorm [m], omega_js [m,3]."""
    import torch

    m = stencils.shape[0]
    f32 = dict(dtype=torch.float32, device="cuda")
    feat = torch.empty((m, 5), **f32)
    cand = torch.empty((m, 3), **f32)
    tn = torch.empty(m, **f32)
    ojs = torch.empty((m, 3), **f32)
    _native.check_mlp(_native.lib().mfx_mlp_features(_p(stencils), _p(targets), m, eps, _p(feat), _p(cand), _p(tn),
                                                     _p(ojs), _stream()))
    return feat, cand, tn, ojs


def features_edge(stencils, targets, tmax: float = 2.0, eps: float = 1e-6):
    """Shared form: (feat [2n,5], cand [2n,7,3], tnorm [2n,7], base
    [2n,7,3]: each variable's Jiang-Shu weights) of one 1D sample set of n
    cells (``mfx_mlp_features_edge``)."""
    import torch

    ncell = stencils.shape[0] // 14
    m = 2 * ncell
    f32 = dict(dtype=torch.float32, device="cuda")
    feat = torch.empty((m, 5), **f32)
    cand = torch.empty((m, 7, 3), **f32)
    tn = torch.empty((m, 7), **f32)
    base = torch.empty((m, 7, 3), **f32)
    _native.check_mlp(_native.lib().mfx_mlp_features_edge(_p(stencils), _p(targets), ncell, eps, tmax, _p(feat),
                                                          _p(cand), _p(tn), _p(base), _stream()))
    return feat, cand, tn, base


def build_dataset(tube_seeds, slab_seeds, edge: bool = False, log=print):
    """Samples from seeded runs, flat stencils dropped; returns the feature
    tensors and the raw sample count before filtering.  edge=True builds the
    shared per-edge samples (all seven variables of an edge together;
    edges where every variable is flat or off target are dropped)."""
    import torch

    chunks = []
    for s in tube_seeds:
        chunks += shock_tube_samples(s)
    for s in slab_seeds:
        chunks += slab_samples(s)
    if edge:
        parts = [features_edge(st, tg) for st, tg in chunks]
        feat, cand, tn, base = (torch.cat([p[k] for p in parts]) for k in range(4))
        raw = feat.shape[0]
        keep = (cand.abs().sum(dim=(1, 2)) > 0) | (tn.abs().sum(dim=1) > 0)
        out = tuple(x[keep].contiguous() for x in (feat, cand, tn, base))
        log(f"[learned] edge samples: {raw} drawn, {out[0].shape[0]} kept")
        return out + (raw,)
    st = torch.cat([c[0] for c in chunks])
    tg = torch.cat([c[1] for c in chunks])
    raw = st.shape[0]
    span = st.max(dim=1).values - st.min(dim=1).values
    keep = span > 1e-6 * st.abs().max(dim=1).values
    st, tg = st[keep].contiguous(), tg[keep].contiguous()
    feat, cand, tn, ojs = features(st, tg)
    # a target far outside its stencil's range cannot be reached by any
    # convex combination of the candidates (the reference solution has moved
    # on where the sampled one is still flat): drop those as well
    ok = tn.abs() <= 2.0
    out = tuple(x[ok].contiguous() for x in (feat, cand, tn, ojs))
    log(f"[learned] samples: {raw} drawn, {int(keep.sum())} non-flat, {out[0].shape[0]} kept")
    return out + (raw,)


# ------------------------------------------------------------------ training

def loss_grad(params, feat, cand, tn, ojs, lam, ws=None):
    """Loss and gradient; cand [m,3] or [m,7,3] (shared form)."""
    import torch

    m = feat.shape[0]
    nvar = cand.shape[1] if cand.dim() == 3 else 1
    need = int(_native.lib().mfx_mlp_grad_workspace(m))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    grad = torch.empty(N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _native.check_mlp(_native.lib().mfx_mlp_loss_grad(_p(params), _p(feat), _p(cand), _p(tn), _p(ojs), m, nvar,
                                                      ctypes.c_float(lam), _p(ws), ws.numel(), _p(grad), _p(loss),
                                                      _stream()))
    return loss, grad, ws


def forward(params, feat, ojs, packed=False):
    """omega [m, 3] from features and Jiang-Shu weights: float32 network, or
    bfloat16 matrix cores (packed=True)."""
    import torch

    m = feat.shape[0]
    om = torch.empty((m, 3), dtype=torch.float32, device="cuda")
    L = _native.lib()
    if packed:
        pk = torch.empty(int(L.mfx_mlp_packed_bytes()), dtype=torch.uint8, device="cuda")
        _native.check_mlp(L.mfx_mlp_pack(_p(params), _p(pk), _stream()))
        _native.check_mlp(L.mfx_mlp_forward(None, _p(pk), _p(feat), _p(ojs), m, _p(om), _stream()))
    else:
        _native.check_mlp(L.mfx_mlp_forward(_p(params), None, _p(feat), _p(ojs), m, _p(om), _stream()))
    return om


def train(data, epochs=20, batch=65536, lr=2e-3, lam=0.02, seed=0, log=print):
    """Minibatch Adam with cosine decay; returns (params, history)."""
    import torch

    feat, cand, tn, ojs = data
    m = feat.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    perm = torch.randperm(m, generator=g, device="cuda")
    nval = max(1, m // 10)
    val, tr = perm[:nval], perm[nval:]
    V = tuple(x[val].contiguous() for x in (feat, cand, tn, ojs))
    params = torch.from_numpy(init_params(seed)).cuda()
    mom = torch.zeros_like(params)
    var = torch.zeros_like(params)
    steps_per_epoch = max(1, (tr.numel() + batch - 1) // batch)
    total = epochs * steps_per_epoch
    step = 0
    ws = None
    hist = []
    L = _native.lib()
    for ep in range(epochs):
        order = tr[torch.randperm(tr.numel(), generator=g, device="cuda")]
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            B = tuple(x[idx].contiguous() for x in (feat, cand, tn, ojs))
            _, grad, ws = loss_grad(params, *B, lam, ws)
            step += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
            _native.check_mlp(L.mfx_mlp_adam(_p(params), _p(mom), _p(var), _p(grad), step, ctypes.c_float(lr_t),
                                             _stream()))
        lv, _, ws = loss_grad(params, *V, lam, ws)
        hist.append(float(lv.item()))
        log(f"[learned] epoch {ep + 1}/{epochs}: validation loss {hist[-1]:.4e}")
    return params, hist


# ------------------------------------------------------------------ fine-tuning on the solution error

class SolutionObjective:
    """Error of whole solver runs with given network parameters, relative to
    the Jiang-Shu form's error on the same runs (1 = no gain).

    Problems (seeded, disjoint from the held-out ones that measure the gain):
      * shock tubes of ``shock_tube_family`` on `n_tube` cells for
        `tube_steps` steps; reference = an FP64 run `refine` times finer with
        the coarse time steps split evenly, averaged onto the coarse cells;
        error = sum over density, momentum and energy of
        mean|q - q_ref| / mean|q_ref|;
      * advected slabs on `n_slab` cells for `slab_steps` steps; reference =
        the exact cell averages of the translated alpha1 profile; error =
        mean|alpha1 - ref| / mean|ref|.
    Every run replays the time steps of the FP64 Jiang-Shu run of its
    problem, so all forms are compared at the same times.  Runs use the
    float32 form with learned weights (as deployed); a run that ends with a
    flagged or non-finite state scores `penalty`.
    """

    def __init__(self, tube_seeds=(0, 1, 2, 3), slab_seeds=(1000, 1001, 1002, 1003), n_tube=500, tube_steps=150,
                 refine=8, n_slab=256, slab_steps=200, penalty=10.0, weights=None):
        import torch

        from . import MFX_FP32_MIXED, MFX_WENO5_JS, MFX_WENO5_LEARNED

        weights = MFX_WENO5_LEARNED if weights is None else weights

        self.penalty = penalty
        self.runs = []
        for seed in tube_seeds:
            Pc = wl.shock_tube_family(n=n_tube, seed=seed)
            Pf = wl.shock_tube_family(n=n_tube * refine, seed=seed)
            coarse, fine = Solver(Pc["spec"], MFX_FP64), Solver(Pf["spec"], MFX_FP64)
            w0 = torch.from_numpy(Pc["w"]).cuda()
            coarse.set_primitive(w0)
            fine.set_primitive(torch.from_numpy(Pf["w"]).cuda())
            dts = []
            for _ in range(tube_steps):
                dt = coarse.rk3_step(sync=True)
                dts.append(dt)
                for _ in range(refine):
                    fine.rk3_step(dt / refine)
            qf = fine.get_state().reshape(7, n_tube, refine).mean(dim=2)
            ref = torch.stack([qf[0] + qf[1], qf[2], qf[5]])
            self.runs.append({"kind": "tube", "spec": Pc["spec"], "w0": w0, "dts": dts, "ref": ref})
        for seed in slab_seeds:
            P = wl.advected_slab(n=n_slab, seed=seed)
            s = Solver(P["spec"], MFX_FP64)
            w0 = torch.from_numpy(P["w"]).cuda()
            s.set_primitive(w0)
            dts = [s.rk3_step(sync=True) for _ in range(slab_steps)]
            ref = torch.from_numpy(P["alpha_cell_avg"](sum(dts))).cuda()
            self.runs.append({"kind": "slab", "spec": P["spec"], "w0": w0, "dts": dts, "ref": ref})
        # every problem runs on a stream of its own, so that the (latency-bound,
        # single-row) runs of one evaluation overlap on the device
        for r in self.runs:
            r["stream"] = torch.cuda.Stream()
            r["learned"] = Solver(r["spec"], MFX_FP32_MIXED, weights, stream=r["stream"])
            r["js"] = Solver(r["spec"], MFX_FP32_MIXED, MFX_WENO5_JS, stream=r["stream"])
        for r, e in zip(self.runs, self._run_all("js")):
            assert math.isfinite(e), "Jiang-Shu reference run failed"
            r["js_err"] = e

    @staticmethod
    def _error(r, q):
        q = q.reshape(7, -1)
        if r["kind"] == "tube":
            got = (q[0] + q[1], q[2], q[5])
            return sum((g - f).abs().mean() / f.abs().mean() for g, f in zip(got, r["ref"]))
        return (q[6] - r["ref"]).abs().mean() / r["ref"].abs().mean()

    def _run_all(self, which, params_dev=None):
        """Enqueue every problem's run on its stream, then collect the errors
        (NaN for a run whose state was flagged or is not finite)."""
        import torch

        from . import MfxError

        torch.cuda.synchronize()  # parameters uploaded on the current stream
        for r in self.runs:  # enqueue only: nothing here waits for the device
            s = r[which]
            if params_dev is not None:
                s.set_mlp(params_dev)
            s.set_primitive(r["w0"])
            for dt in r["dts"]:
                s.rk3_step(dt)
        out = []
        for r in self.runs:
            with torch.cuda.stream(r["stream"]):
                try:
                    e = float(self._error(r, r[which].get_state()).item())  # get_state waits for its stream
                except MfxError:  # state flagged non-physical
                    e = float("nan")
            out.append(e if math.isfinite(e) else float("nan"))
        return out

    def per_problem(self, params_dev):
        """Error ratios learned / Jiang-Shu per problem (penalty if a run fails)."""
        return [e / r["js_err"] if math.isfinite(e) else self.penalty
                for r, e in zip(self.runs, self._run_all("learned", params_dev))]

    def __call__(self, params_dev) -> float:
        return float(np.mean(self.per_problem(params_dev)))


OUT_LAYER = (H * 5 + H + H * H + H, N_PARAMS)  # W3 and b3 in the flat layout


def finetune(params, objective, iters=100, pairs=16, sigma=0.05, lr=0.05, seed=0, log=print):
    """Minimise objective(params) over the output layer (W3, b3) with an
    evolution-strategies gradient estimate (antithetic Gaussian
    perturbations, centred-rank fitness shaping; Salimans et al. 2017) fed
    to the library's Adam kernel.  Returns (best params, history)."""
    import torch

    rng = np.random.default_rng(seed)
    lo, hi = OUT_LAYER
    theta = params.detach().clone().float().contiguous()
    mom = torch.zeros_like(theta)
    var = torch.zeros_like(theta)
    L = _native.lib()
    f0 = objective(theta)
    best, best_f = theta.clone(), f0
    hist = [f0]
    log(f"[finetune] start: objective {f0:.4f}")
    base = theta.cpu().numpy()
    for it in range(1, iters + 1):
        eps = rng.standard_normal((pairs, hi - lo)).astype(np.float32)
        fit = np.empty(2 * pairs)
        for i in range(pairs):
            for j, sgn in enumerate((1.0, -1.0)):
                cand = base.copy()
                cand[lo:hi] += sgn * sigma * eps[i]
                fit[2 * i + j] = objective(torch.from_numpy(cand).cuda())
        ranks = np.empty(2 * pairs)
        ranks[np.argsort(fit)] = np.arange(2 * pairs)
        shaped = ranks / (2 * pairs - 1) - 0.5
        g = np.zeros_like(base)
        g[lo:hi] = ((shaped[0::2] - shaped[1::2])[:, None] * eps).sum(axis=0) / (2 * pairs * sigma)
        g_dev = torch.from_numpy(g).cuda()  # held until the step has read it
        _native.check_mlp(L.mfx_mlp_adam(_p(theta), _p(mom), _p(var), _p(g_dev), it, ctypes.c_float(lr), _stream()))
        base = theta.cpu().numpy()
        f = objective(theta)
        hist.append(f)
        if f < best_f:
            best, best_f = theta.clone(), f
        log(f"[finetune] iter {it}/{iters}: objective {f:.4f} (best {best_f:.4f}, population min {fit.min():.4f})")
    return best, hist


def js_validation_loss(data, lam):
    """Loss of the Jiang-Shu weights themselves on the same samples (the
    reference the network has to beat): error term only, regulariser 0."""
    feat, cand, tn, ojs = data
    if cand.dim() == 3:
        r = (ojs * cand).sum(dim=2) - tn
    else:
        r = (ojs * cand).sum(dim=1) - tn
    return float((r * r).mean().item())


def calibrate(path: str, scale: float, command: str) -> int:
    """Scale the output layer (W3, b3) of a saved network by `scale`: in the
    residual form the logits z = W3 h + b3 correct log(omega_JS), so this
    applies the learned correction at the given strength.  Recorded in the
    network's metadata (applied scales multiply)."""
    p = np.load(path, allow_pickle=False)
    lo, hi = OUT_LAYER
    p[lo:hi] *= np.float32(scale)
    np.save(path, p)
    mpath = os.path.splitext(path)[0] + ".json"
    meta = {}
    if os.path.exists(mpath):
        with open(mpath) as f:
            meta = json.load(f)
    meta.setdefault("calibration", []).append({"correction_scale": scale, "command": command})
    with open(mpath, "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta["calibration"]), flush=True)
    return 0


def _applied_scale(meta: dict) -> float:
    """Product of the correction scales already applied to a saved network."""
    f = 1.0
    for c in meta.get("calibration", []):
        f *= c["correction_scale"]
    return f


def density_l1(q, q64) -> float:
    """sum |rho - rho64| / sum |rho64| with rho = alpha1 rho1 + alpha2 rho2."""
    rho, rho64 = q[0] + q[1], q64[0] + q64[1]
    return float(np.abs(rho - rho64).sum() / np.abs(rho64).sum())


def select_strength(path: str, workload: str, n: int, seed: int, steps: int, strengths, bar: float,
                    command: str, edge: bool = False, apply: bool = True) -> int:
    """Choose the correction strength of a saved network on a problem other
    than the one it is benchmarked on: for each strength s (relative to the
    trained output layer), replay the FP64 run's time steps of `workload`
    (n^3 cells, `seed`) with the learned weights at strength s and measure
    the density L1 against the FP64 state; the largest s within `bar` is
    applied to the network and recorded, with every measurement, in its
    metadata (apply=False: measure only)."""
    import torch

    from . import MFX_FP32_MIXED, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE

    weights = MFX_WENO5_LEARNED_EDGE if edge else MFX_WENO5_LEARNED
    mpath = os.path.splitext(path)[0] + ".json"
    meta = {}
    if os.path.exists(mpath):
        with open(mpath) as f:
            meta = json.load(f)
    base = _applied_scale(meta)
    p_now = np.load(path, allow_pickle=False).astype(np.float32)
    lo, hi = OUT_LAYER
    P = getattr(wl, workload)(n=n, seed=seed)
    w_dev = torch.from_numpy(P["w"]).cuda()
    s64 = Solver(P["spec"], MFX_FP64)
    s64.set_primitive(w_dev)
    dts = [s64.rk3_step(sync=True) for _ in range(steps)]
    q64 = s64.get_state().cpu().numpy().reshape(7, -1)
    s64.destroy()
    l1 = {}
    for st in strengths:
        p = p_now.copy()
        p[lo:hi] *= np.float32(st / base)
        s = Solver(P["spec"], MFX_FP32_MIXED, weights)
        s.set_mlp(torch.from_numpy(p).cuda())
        s.set_primitive(w_dev)
        for dt in dts:
            s.rk3_step(dt)
        l1[st] = density_l1(s.get_state().cpu().numpy().reshape(7, -1), q64)
        s.destroy()
        print(f"[select] strength {st}: density L1 {l1[st]:.3e}", flush=True)
    ok = [st for st in strengths if l1[st] <= bar]
    if not apply:
        print(json.dumps({"workload": workload, "n": n, "seed": seed, "steps": steps,
                          "density_l1": {str(k): v for k, v in l1.items()}, "within_bar": ok}), flush=True)
        return 0
    chosen = max(ok) if ok else min(strengths)
    p = p_now.copy()
    p[lo:hi] *= np.float32(chosen / base)
    np.save(path, p)
    meta["calibration"] = [{"correction_scale": chosen,
                            "selected_on": {"workload": workload, "n": n, "seed": seed, "steps": steps, "bar": bar,
                                            "density_l1": {str(k): v for k, v in l1.items()}},
                            "command": command}]
    with open(mpath, "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta["calibration"]), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=None, help="default: data/mlp_weno5.npy, or data/mlp_weno5_edge.npy with --edge")
    ap.add_argument("--edge", action="store_true", help="train the shared per-edge form")
    ap.add_argument("--tubes", type=int, default=96, help="shock-tube runs (seeds 0..N-1)")
    ap.add_argument("--slabs", type=int, default=48, help="advected-slab runs (seeds 1000..)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lam", type=float, default=0.5)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--ft-iters", type=int, default=60, help="solution-error fine-tuning iterations (0: none)")
    ap.add_argument("--ft-pairs", type=int, default=16)
    ap.add_argument("--ft-sigma", type=float, default=0.05)
    ap.add_argument("--ft-lr", type=float, default=0.05)
    ap.add_argument("--ft-tubes", type=int, default=4, help="fine-tuning shock tubes (seeds 0..N-1)")
    ap.add_argument("--ft-slabs", type=int, default=4, help="fine-tuning slabs (seeds 1000..)")
    ap.add_argument("--calibrate", type=float, default=None,
                    help="no training: scale the output layer of the existing --out network (the network's "
                         "correction to the Jiang-Shu log-weights is linear in it) by this factor and record it")
    ap.add_argument("--select-strength", action="store_true",
                    help="no training: choose the correction strength of the existing --out network on a held-out "
                         "problem (--select-workload/-n/-seed/-steps) as the largest of --strengths whose density "
                         "L1 against the FP64 path stays within --bar, apply it and record the measurements")
    ap.add_argument("--select-workload", default="shock_droplet")
    ap.add_argument("--select-n", type=int, default=256)
    ap.add_argument("--select-seed", type=int, default=1)
    ap.add_argument("--select-steps", type=int, default=200)
    ap.add_argument("--strengths", default="1.0,0.9,0.8,0.7,0.6,0.5")
    ap.add_argument("--bar", type=float, default=1e-4)
    ap.add_argument("--measure-only", action="store_true", help="with --select-strength: report, change nothing")
    args = ap.parse_args(argv)
    if args.out is None:
        args.out = EDGE_PARAMS if args.edge else DEFAULT_PARAMS
    cmd = "python -m paper_2409_10729_amd.learned " + " ".join(sys.argv[1:] if argv is None else argv)
    if args.select_strength:
        return select_strength(args.out, args.select_workload, args.select_n, args.select_seed, args.select_steps,
                               [float(v) for v in args.strengths.split(",")], args.bar, cmd, edge=args.edge,
                               apply=not args.measure_only)
    if args.calibrate is not None:
        return calibrate(args.out, args.calibrate,
                         "python -m paper_2409_10729_amd.learned " + " ".join(sys.argv[1:] if argv is None else argv))
    import torch

    from . import MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE

    assert torch.cuda.is_available(), "training runs on the GPU"
    t0 = time.time()
    *data, raw = build_dataset(range(args.tubes), range(1000, 1000 + args.slabs), edge=args.edge)
    t1 = time.time()
    params, hist = train(tuple(data), epochs=args.epochs, lam=args.lam, lr=args.lr)
    t2 = time.time()
    js = js_validation_loss(tuple(data), args.lam)
    ft_hist = []
    if args.ft_iters > 0:
        obj = SolutionObjective(tube_seeds=tuple(range(args.ft_tubes)),
                                slab_seeds=tuple(range(1000, 1000 + args.ft_slabs)),
                                weights=MFX_WENO5_LEARNED_EDGE if args.edge else MFX_WENO5_LEARNED)
        params, ft_hist = finetune(params, obj, iters=args.ft_iters, pairs=args.ft_pairs, sigma=args.ft_sigma,
                                   lr=args.ft_lr)
    t3 = time.time()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params.cpu().numpy())
    meta = {"samples_drawn": raw, "samples_kept": int(data[0].shape[0]), "epochs": args.epochs, "lam": args.lam,
            "lr": args.lr, "val_loss": hist, "js_error_term_all_samples": js,
            "data_seconds": round(t1 - t0, 1), "train_seconds": round(t2 - t1, 1),
            "tubes": args.tubes, "slabs": args.slabs, "form": "edge" if args.edge else "variable",
            "finetune": {"iters": args.ft_iters, "pairs": args.ft_pairs, "sigma": args.ft_sigma, "lr": args.ft_lr,
                         "tubes": args.ft_tubes, "slabs": args.ft_slabs, "objective": ft_hist,
                         "seconds": round(t3 - t2, 1)},
            "command": "python -m paper_2409_10729_amd.learned " + " ".join(sys.argv[1:] if argv is None else argv)}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    sys.exit(main())
