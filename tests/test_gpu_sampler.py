"""Training-data helpers of the learned weights against a plain numpy
extraction from the same state.

mfx_mlp_sample_stencils: for every cell i and variable v of a 1D state, the
primitives of cells i-2..i+2 (ghosts by the boundary rule: periodic wraps,
transmissive clamps to the end cell) with target face_prim[v][i+1], and the
mirrored stencil i+2..i-2 with target face_prim[v][i].  mfx_mlp_face_targets:
coarse face i of a grid `refine` times coarser lies on fine face refine*i,
whose value is the mean of the primitives of the two fine cells beside it
(the end cell at a domain end).  The numpy side converts with the oracle's
cons_to_prim and indexes the arrays directly; targets are copies and must
match bit for bit, stencils to the conversion's rounding.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import _native
from paper_2409_10729_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _ghost(i, n, bc):
    """Cell index of position i (any integer) under the x boundary rule."""
    if bc == 0:
        return i % n
    return min(max(i, 0), n - 1)


def _state(n, seed, bc):
    P = wl.shock_tube_family(n=n, seed=seed)
    spec = dict(P["spec"], bc=((bc, bc), (0, 0), (0, 0)))
    g = oracle.make_grid(spec)
    return spec, g, oracle.prim_to_cons(g, P["w"])


@pytest.mark.parametrize("bc,n,seed", [(0, 37, 1), (1, 64, 2), (1, 5, 3)])
def test_sample_stencils_match_numpy_extraction(bc, n, seed):
    spec, g, q = _state(n, seed, bc)
    rng = np.random.default_rng(seed)
    face = rng.normal(size=(7, n + 1))
    st = torch.empty((14 * n, 5), dtype=torch.float64, device="cuda")
    tg = torch.empty(14 * n, dtype=torch.float64, device="cuda")
    d = _native.make_desc(spec)
    print(f"sample stencils: bc {bc} n {n} seed {seed}", flush=True)
    # (device copies held by names: a temporary would be freed, and its memory
    # reused, before the launch)
    q_dev, face_dev = torch.from_numpy(q).cuda(), torch.from_numpy(face).cuda()
    _native.check_mlp(_native.lib().mfx_mlp_sample_stencils(ctypes.byref(d), _p(q_dev), _p(face_dev), _p(st), _p(tg),
                                                            _stream()))
    torch.cuda.synchronize()
    st, tg = st.cpu().numpy(), tg.cpu().numpy()
    w = oracle.cons_to_prim(g, q).reshape(7, n)
    ref_st = np.empty((14 * n, 5))
    ref_tg = np.empty(14 * n)
    for v in range(7):
        for i in range(n):
            cells = [_ghost(i - 2 + k, n, bc) for k in range(5)]
            right, left = v * n + i, (7 + v) * n + i
            ref_st[right] = w[v, cells]
            ref_st[left] = w[v, cells[::-1]]
            ref_tg[right] = face[v, i + 1]
            ref_tg[left] = face[v, i]
    assert np.array_equal(tg, ref_tg)
    scale = np.maximum(np.abs(w).max(axis=1), 1e-300).repeat(n)  # (v = w = 0 in a tube)
    scale = np.concatenate([scale, scale])[:, None]
    err = np.abs(st - ref_st) / scale
    print(f"  max stencil error {err.max():.2e} (relative to each variable's magnitude)", flush=True)
    assert err.max() <= 1e-14


@pytest.mark.parametrize("bc,nc,refine,seed", [(1, 40, 4, 5), (0, 24, 3, 6), (1, 1, 8, 7)])
def test_face_targets_match_numpy_extraction(bc, nc, refine, seed):
    nf = nc * refine
    spec, g, q = _state(nf, seed, bc)
    out = torch.empty((7, nc + 1), dtype=torch.float64, device="cuda")
    d = _native.make_desc(spec)
    print(f"face targets: bc {bc} coarse n {nc} refine {refine} seed {seed}", flush=True)
    q_dev = torch.from_numpy(q).cuda()
    _native.check_mlp(_native.lib().mfx_mlp_face_targets(ctypes.byref(d), _p(q_dev), refine, _p(out), _stream()))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    w = oracle.cons_to_prim(g, q).reshape(7, nf)
    ref = np.empty((7, nc + 1))
    for i in range(nc + 1):
        f = refine * i
        ref[:, i] = 0.5 * (w[:, _ghost(f - 1, nf, bc)] + w[:, _ghost(f, nf, bc)])
    err = np.abs(out - ref) / np.maximum(np.abs(w).max(axis=1), 1e-300)[:, None]
    print(f"  max face-value error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-14


def test_helpers_reject_walls_and_inflow():
    spec, g, q = _state(16, 1, 1)
    qd = torch.from_numpy(q).cuda()
    st = torch.empty((14 * 16, 5), dtype=torch.float64, device="cuda")
    tg = torch.empty(14 * 16, dtype=torch.float64, device="cuda")
    face = torch.zeros((7, 17), dtype=torch.float64, device="cuda")
    for bc in (2, 3):
        d = _native.make_desc(dict(spec, bc=((bc, 1), (0, 0), (0, 0))))
        assert _native.lib().mfx_mlp_sample_stencils(ctypes.byref(d), _p(qd), _p(face), _p(st), _p(tg),
                                                     _stream()) == _native.MFX_EINVAL
        assert _native.lib().mfx_mlp_face_targets(ctypes.byref(d), _p(qd), 2, _p(face), _stream()) == _native.MFX_EINVAL
