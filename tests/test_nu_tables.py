"""Host-side checks of unequal cell widths (Sec. III-A local mesh refinement;
no GPU needed): the WENO5 coefficients the library derives from the widths
(mfx_weno5_nu_coefficients, the values its per-position tables hold) give the
oracle's reconstruction, reduce to the published uniform coefficients on equal
widths, and descriptors with face coordinates are validated before any device
call."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2409_10729_amd import _native, weno5_nu_coefficients
from paper_2409_10729_amd import workloads as wl


def _recon(K, v, eps=1e-6):
    """(left, right) from the 33 library coefficients: candidates A + B xi +
    C xi^2, indicators B^2 + 13/3 C^2, Jiang-Shu weights with the tabled
    ideal weights (plain numpy, for comparison with the oracle)."""
    a, b, c = K[0:9].reshape(3, 3), K[9:18].reshape(3, 3), K[18:27].reshape(3, 3)
    dr, dl = K[27:30], K[30:33]
    A = np.array([a[k] @ v[k:k + 3] for k in range(3)])
    B = np.array([b[k] @ v[k:k + 3] for k in range(3)])
    C = np.array([c[k] @ v[k:k + 3] for k in range(3)])
    beta = B * B + 13.0 / 3.0 * C * C
    pr, pl = A + 0.5 * B + 0.25 * C, A - 0.5 * B + 0.25 * C
    ar, al = dr / (eps + beta) ** 2, dl / (eps + beta) ** 2
    return (al @ pl) / al.sum(), (ar @ pr) / ar.sum(), beta


def test_equal_widths_give_the_uniform_coefficients():
    # Jiang-Shu's uniform scheme: candidate right-edge values (2a-7b+11c)/6,
    # (-b+5c+2d)/6, (2c+5d-e)/6, ideal weights 1/10, 6/10, 3/10 (right edge)
    # and 3/10, 6/10, 1/10 (left edge)
    for h in (1.0, 0.37, 2.5e-3):
        K = weno5_nu_coefficients([h] * 5)
        a, b, c = K[0:9].reshape(3, 3), K[9:18].reshape(3, 3), K[18:27].reshape(3, 3)
        right = a + 0.5 * b + 0.25 * c
        left = a - 0.5 * b + 0.25 * c
        np.testing.assert_allclose(right, np.array([[2, -7, 11], [-1, 5, 2], [2, 5, -1]]) / 6.0, atol=1e-13)
        np.testing.assert_allclose(left, np.array([[-1, 5, 2], [2, 5, -1], [11, -7, 2]]) / 6.0, atol=1e-13)
        np.testing.assert_allclose(K[27:30], [0.1, 0.6, 0.3], atol=1e-13)
        np.testing.assert_allclose(K[30:33], [0.3, 0.6, 0.1], atol=1e-13)
        # indicators: 13/12 (a-2b+c)^2 + 1/4 (a-4b+3c)^2 for candidate 0
        v = np.array([0.3, -1.2, 2.0, 0.7, 0.1])
        _, _, beta = _recon(K, v)
        assert beta[0] == pytest.approx(13 / 12 * (v[0] - 2 * v[1] + v[2]) ** 2 + 0.25 * (v[0] - 4 * v[1] + 3 * v[2]) ** 2,
                                        rel=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_library_coefficients_reproduce_the_oracle(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        h = np.exp(rng.uniform(np.log(0.4), np.log(2.5), 5)) * 10.0 ** rng.uniform(-4, 0)
        v = rng.normal(size=5) * 10.0 ** rng.uniform(-2, 3)
        K = weno5_nu_coefficients(h)
        left, right, beta = _recon(K, v)
        ol, orr = oracle.weno5_nu(h, v)
        scale = np.abs(v).max()
        assert abs(left - ol) <= 1e-12 * scale and abs(right - orr) <= 1e-12 * scale
        np.testing.assert_allclose(beta, oracle.weno5_nu_betas(h, v), rtol=1e-11, atol=1e-14 * scale ** 2)
        dr, dl = oracle.ideal_weights_nu(h)
        np.testing.assert_allclose(K[27:30], dr, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(K[30:33], dl, rtol=1e-11, atol=1e-13)


def test_tanh_stretched_positions_reproduce_the_oracle():
    xf = wl.tanh_faces(48, depth=0.7, sharpness=10.0)
    h = np.diff(xf)
    rng = np.random.default_rng(3)
    for c in range(2, 46):
        v = rng.normal(size=5)
        left, right, _ = _recon(weno5_nu_coefficients(h[c - 2:c + 3]), v)
        ol, orr = oracle.weno5_nu(h[c - 2:c + 3], v)
        assert abs(left - ol) <= 1e-13 and abs(right - orr) <= 1e-13


def test_quadratics_exact_on_unequal_cells():
    # any weights: every candidate reproduces a quadratic's edge values
    rng = np.random.default_rng(7)
    h = rng.uniform(0.5, 2.0, 5)
    x = np.concatenate([[0.0], np.cumsum(h)])
    p = lambda t: 0.3 - 1.1 * t + 0.7 * t * t
    P = lambda t: 0.3 * t - 0.55 * t * t + 0.7 / 3.0 * t ** 3
    v = (P(x[1:]) - P(x[:-1])) / h
    left, right, _ = _recon(weno5_nu_coefficients(h), v)
    assert left == pytest.approx(p(x[2]), abs=1e-12)
    assert right == pytest.approx(p(x[3]), abs=1e-12)


def _desc(spec, **over):
    d = _native.make_desc(spec)
    for k, v in over.items():
        setattr(d, k, v)
    return d


def _rejected(d):
    L = _native.lib()
    assert L.mfx_workspace_bytes(ctypes.byref(d)) == 0
    ctx = ctypes.c_void_p()
    rc = L.mfx_init_grid(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(ctx))
    assert rc == _native.MFX_EINVAL and ctx.value is None
    return L.mfx_last_error(None).decode()


def test_faces_grow_the_workspace_by_their_tables():
    L = _native.lib()
    base = wl.spec((32, 16, 8), ((1, 1), (0, 0), (0, 0)))
    b0 = L.mfx_workspace_bytes(ctypes.byref(_desc(base)))
    sp = dict(base, faces=(wl.tanh_faces(32), None, wl.tanh_faces(8)))
    b1 = L.mfx_workspace_bytes(ctypes.byref(_desc(sp)))
    assert b1 >= b0 + 8 * 36 * (34 + 10)


def test_bad_faces_rejected():
    base = wl.spec((32, 16, 1), ((1, 1), (0, 0), (0, 0)))
    xf = wl.tanh_faces(32)
    bad = xf.copy()
    bad[5] = bad[4]
    assert "increasing" in _rejected(_desc(dict(base, faces=(bad, None, None))))
    bad = xf.copy()
    bad[-1] = np.nan
    assert "increasing" in _rejected(_desc(dict(base, faces=(bad, None, None))))
    # an inactive direction
    assert "active" in _rejected(_desc(dict(base, faces=(None, None, np.array([0.0, 1.0])))))
    # schemes other than WENO5 with Jiang-Shu weights
    for over in ({"weno_order": 3}, {"weights": _native.MFX_WENO5_Z}, {"weights": _native.MFX_WENO5_LEARNED}):
        msg = _rejected(_desc(dict(base, faces=(xf, None, None)), **over))
        assert "Jiang-Shu" in msg or "learned" in msg


def test_binding_checks_face_count():
    base = wl.spec((32, 16, 1), ((1, 1), (0, 0), (0, 0)))
    with pytest.raises(ValueError):
        _native.make_desc(dict(base, faces=(wl.tanh_faces(31), None, None)))


def test_static_entry_rejects_unequal_cells():
    L = _native.lib()
    sp = wl.spec((32, 16, 1), ((1, 1), (0, 0), (0, 0)))
    d = _desc(dict(sp, faces=(wl.tanh_faces(32), None, None)))
    rc = L.mfx_rhs_static(ctypes.byref(d), None, None, None)
    assert rc == _native.MFX_EINVAL
    assert "uniform" in L.mfx_last_error(None).decode()


def test_coefficients_reject_bad_widths():
    with pytest.raises(_native.MfxError):
        weno5_nu_coefficients([1.0, 1.0, 0.0, 1.0, 1.0])
    with pytest.raises(_native.MfxError):
        weno5_nu_coefficients([1.0, np.inf, 1.0, 1.0, 1.0])
