"""Host-side checks of the C ABI (no GPU needed): the library builds/loads,
exports every symbol include/mfx.h declares, sizes workspaces, and rejects
bad descriptors before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2409_10729_amd import _native
from paper_2409_10729_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mfx.h")).read()
    return sorted(set(re.findall(r"\b(mfx_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_native.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _native.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _desc(**over):
    spec = wl.spec((32, 16, 8), ((1, 1), (0, 0), (0, 0)))
    d = _native.make_desc(spec)
    for k, v in over.items():
        setattr(d, k, v)
    return d


def test_workspace_bytes_scales_with_grid():
    L = _native.lib()
    d = _desc()
    b = L.mfx_workspace_bytes(ctypes.byref(d))
    N = 32 * 16 * 8
    assert b >= 4 * 7 * 8 * N  # q, two stage buffers, RHS
    d2 = _native.make_desc(wl.spec((64, 16, 8), ((1, 1), (0, 0), (0, 0))))
    assert L.mfx_workspace_bytes(ctypes.byref(d2)) > b


def test_workspace_bytes_three_fluids():
    """Nine variables: the state buffers and the RHS hold nine fields, and
    the x rows' boundary faces ten values per face (flux components and the
    face velocity), two faces per row."""
    L = _native.lib()
    n = (32, 16, 8)
    N = n[0] * n[1] * n[2]
    d3 = _native.make_desc(wl.spec_fluids(n, ((1, 1), (0, 0), (0, 0)), 3))
    b3 = L.mfx_workspace_bytes(ctypes.byref(d3))
    assert b3 >= 4 * 9 * 8 * N + 10 * 2 * 8 * n[1] * n[2]
    assert b3 > L.mfx_workspace_bytes(ctypes.byref(_desc()))


@pytest.mark.parametrize("field,value", [
    ("cfl", 0.0), ("cfl", 1.5), ("weno_eps", 0.0), ("precision", 7), ("weights", 9), ("weno_order", 4),
    ("weno_order", 1),
])
def test_bad_scalars_rejected(field, value):
    L = _native.lib()
    d = _desc(**{field: value})
    assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0
    ctx = ctypes.c_void_p()
    rc = L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(ctx))
    assert rc == _native.MFX_EINVAL
    assert ctx.value is None
    assert L.mfx_last_error(None)


def test_bad_arrays_rejected():
    L = _native.lib()
    for mutate in (lambda d: d.n.__setitem__(1, 0), lambda d: d.dx.__setitem__(0, -1.0),
                   lambda d: d.bc[0].__setitem__(0, 5), lambda d: d.gamma.__setitem__(1, 1.0),
                   lambda d: d.pi_inf.__setitem__(0, -1.0)):
        d = _desc()
        mutate(d)
        assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0
        ctx = ctypes.c_void_p()
        assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(ctx)) == _native.MFX_EINVAL


def test_unpaired_periodic_rejected():
    L = _native.lib()
    d = _desc()
    d.bc[1][0] = 0
    d.bc[1][1] = 1
    ctx = ctypes.c_void_p()
    assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None,
                           ctypes.byref(ctx)) == _native.MFX_EINVAL
    assert b"paired" in L.mfx_last_error(None)


def test_reflective_sides_accepted_and_checked():
    """Reflective (slip-wall) sides pass validation alone or beside a
    transmissive side; a reflective direction with 2 cells is rejected."""
    L = _native.lib()
    for k in range(3):
        for pair in ((2, 2), (2, 1), (1, 2)):
            d = _desc()
            d.bc[k][0], d.bc[k][1] = pair
            assert L.mfx_workspace_bytes(ctypes.byref(d)) > 0, (k, pair)
    d = _desc()
    d.bc[0][0] = d.bc[0][1] = _native.MFX_BC_REFLECTIVE
    d.n[0] = 2
    assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0
    ctx = ctypes.c_void_p()
    assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None,
                           ctypes.byref(ctx)) == _native.MFX_EINVAL
    assert b"reflective" in L.mfx_last_error(None)
    d = _desc()
    d.bc[2][1] = 3
    assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0


def test_inflow_sides_accepted_and_checked():
    """An inflow side needs a valid conserved ghost state: finite, partial
    densities >= 0 with a positive sum, alpha_1 in [0, 1]."""
    L = _native.lib()
    good = [1.0, 1.2, 10.0, 0.0, 0.0, 3.0e5, 0.5]
    for k in range(3):
        for pair in ((3, 1), (1, 3), (3, 3), (3, 2)):
            d = _desc()
            d.bc[k][0], d.bc[k][1] = pair
            for s in range(2):
                for v in range(7):
                    d.inflow[k][s][v] = good[v]
            assert L.mfx_workspace_bytes(ctypes.byref(d)) > 0, (k, pair)
    for v, bad in ((0, -1.0), (6, 1.5), (5, float("nan")), (1, float("inf"))):
        d = _desc()
        d.bc[0][0] = _native.MFX_BC_INFLOW
        for u in range(7):
            d.inflow[0][0][u] = good[u]
        d.inflow[0][0][v] = bad
        assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0, (v, bad)
        ctx = ctypes.c_void_p()
        assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(ctx)) == _native.MFX_EINVAL
        assert b"inflow" in L.mfx_last_error(None)
    # the state of a side that is not inflow is ignored
    d = _desc()
    d.inflow[1][0][0] = float("nan")
    assert L.mfx_workspace_bytes(ctypes.byref(d)) > 0
    # reflective and inflow sides need an active direction
    for kind in (_native.MFX_BC_REFLECTIVE, _native.MFX_BC_INFLOW):
        d = _desc()
        d.n[2] = 1
        d.bc[2][0] = d.bc[2][1] = kind
        for s in range(2):
            for v in range(7):
                d.inflow[2][s][v] = good[v]
        assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0


def test_small_or_misaligned_workspace_rejected():
    L = _native.lib()
    d = _desc()
    need = L.mfx_workspace_bytes(ctypes.byref(d))
    ctx = ctypes.c_void_p()
    assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(4096), need - 1, None,
                           ctypes.byref(ctx)) == _native.MFX_ENOMEM
    assert L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(4096 + 8), need, None,
                           ctypes.byref(ctx)) == _native.MFX_EINVAL
    assert L.mfx_init_grid(ctypes.byref(d), None, need, None, ctypes.byref(ctx)) == _native.MFX_EINVAL


def test_null_context_calls_rejected():
    L = _native.lib()
    assert L.mfx_set_state(None, None) == _native.MFX_EINVAL
    assert L.mfx_rhs(None, None) == _native.MFX_EINVAL
    assert L.mfx_rk3_step(None, 0.0, None) == _native.MFX_EINVAL
    assert L.mfx_stats(None, None, None, None, None) == _native.MFX_EINVAL


def test_weno_order_options():
    """Orders 5 and 3 are accepted (0 reads as 5); the learned weights need 5."""
    L = _native.lib()
    for order in (0, 3, 5):
        assert L.mfx_workspace_bytes(ctypes.byref(_desc(weno_order=order))) > 0
    d = _desc(weno_order=3, weights=_native.MFX_WENO5_LEARNED, precision=_native.MFX_FP32_MIXED)
    assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0
    # WENO-Z weights: fifth order only, either precision form
    for prec in (_native.MFX_FP64, _native.MFX_FP32_MIXED):
        assert L.mfx_workspace_bytes(ctypes.byref(_desc(weights=_native.MFX_WENO5_Z, precision=prec))) > 0
    assert L.mfx_workspace_bytes(ctypes.byref(_desc(weights=_native.MFX_WENO5_Z, weno_order=3))) == 0


def test_size_limits():
    """Extents up to 65535 per direction and up to 2^31 cells are accepted
    (workspace sized with 64-bit arithmetic); beyond either, rejected."""
    L = _native.lib()
    ok = _native.make_desc(wl.spec((65535, 1, 1), ((1, 1), (0, 0), (0, 0))))
    assert L.mfx_workspace_bytes(ctypes.byref(ok)) > 4 * 7 * 8 * 65535
    big = _native.make_desc(wl.spec((2048, 1024, 1024), ((1, 1), (0, 0), (0, 0))))  # exactly 2^31 cells
    b = L.mfx_workspace_bytes(ctypes.byref(big))
    assert b >= 4 * 7 * 8 * (1 << 31)
    for n in ((65536, 1, 1), (2048, 1024, 1025)):
        d = _native.make_desc(wl.spec(n, ((1, 1), (0, 0), (0, 0))))
        assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0


def _static_need(n, elem, nv=7):
    """Scratch bytes of mfx_rhs_static as its declaration states them."""
    def a(x):
        return (x + 255) // 256 * 256
    return 768 + a(elem * 2 * (nv + 1) * n[1] * n[2]) + a(elem * nv * n[0] * n[1] * n[2])


@pytest.mark.parametrize("n,precision,nf", [((134, 134, 134), _native.MFX_FP64, 2),
                                            ((168, 168, 168), _native.MFX_FP32_MIXED, 2),
                                            ((2000, 2000, 1), _native.MFX_FP64, 2),
                                            ((124, 124, 124), _native.MFX_FP64, 3)])
def test_static_rhs_rejects_grids_beyond_its_scratch(n, precision, nf):
    """Grids whose scratch exceeds the static array are refused before any
    device call (MFX_ENOMEM); the limit follows the header's formula."""
    L = _native.lib()
    elem = 8 if precision == _native.MFX_FP64 else 4
    nv = 2 * nf + 3
    assert _static_need(n, elem, nv) > _native.STATIC_SCRATCH_BYTES
    d = _native.make_desc(wl.spec_fluids(n, ((1, 1), (0, 0), (0, 0)), nf), precision)
    nb = nv * 8 * n[0] * n[1] * n[2]
    rc = L.mfx_rhs_static(ctypes.byref(d), ctypes.c_void_p(1 << 40), ctypes.c_void_p((1 << 40) + nb), None)
    assert rc == _native.MFX_ENOMEM
    assert b"scratch" in L.mfx_last_error(None)


def test_static_rhs_limits_admit_the_stated_sizes():
    assert _static_need((128, 128, 128), 8) <= _native.STATIC_SCRATCH_BYTES
    assert _static_need((160, 160, 160), 4) <= _native.STATIC_SCRATCH_BYTES
    assert _static_need((120, 120, 120), 8, 9) <= _native.STATIC_SCRATCH_BYTES


@pytest.mark.parametrize("case", ["learned", "null", "overlap", "bad_desc"])
def test_static_rhs_rejects_bad_arguments(case):
    L = _native.lib()
    spec = wl.spec((16, 8, 4), ((1, 1), (0, 0), (0, 0)))
    weights = _native.MFX_WENO5_LEARNED if case == "learned" else _native.MFX_WENO5_JS
    precision = _native.MFX_FP32_MIXED if case == "learned" else _native.MFX_FP64
    d = _native.make_desc(spec, precision, weights)
    if case == "bad_desc":
        d.cfl = 0.0
    q, r = 1 << 40, (1 << 40) + 7 * 8 * 16 * 8 * 4
    if case == "null":
        r = 0
    if case == "overlap":
        r = q + 8
    rc = L.mfx_rhs_static(ctypes.byref(d), ctypes.c_void_p(q), ctypes.c_void_p(r), None)
    assert rc == _native.MFX_EINVAL
