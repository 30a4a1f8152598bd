"""Pins of the learned-filter oracle (oracle/learned.py) against brute force,
library routines, adjoint identities, finite differences and closed forms.
CPU only."""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import learned as ol
import workloads as wl


def brute_conv(x, w, b):
    """Definition written out with scalar loops (tiny inputs only)."""
    rows, cin, n = x.shape
    cout, _, k = w.shape
    out = np.zeros((rows, cout, n))
    for r in range(rows):
        for o in range(cout):
            for xx in range(n):
                s = b[o]
                for i in range(cin):
                    for t in range(k):
                        j = xx + t - k // 2
                        if 0 <= j < n:
                            s += w[o, i, t] * x[r, i, j]
                out[r, o, xx] = s
    return out


def test_conv_matches_scalar_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 11))
    w = rng.standard_normal((2, 3, 9))
    b = rng.standard_normal(2)
    assert np.allclose(ol.conv(x, w, b), brute_conv(x, w, b), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 4, 9, 30])
def test_single_channel_conv_is_library_correlation(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    w = rng.standard_normal(9)
    # scipy's zero-padded 'same' correlation of a length-n row with 9 taps
    ref = scipy.signal.correlate(np.pad(x, 4), w, mode="valid")
    got = ol.conv(x[None, None, :], w[None, None, :])[0, 0]
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("t0", [0, 3, 4, 8])
def test_one_hot_tap_is_shift(t0):
    x = np.arange(1.0, 13.0)[None, None, :]
    w = np.zeros((1, 1, 9))
    w[0, 0, t0] = 1.0
    s = t0 - 4
    ref = np.zeros(12)
    for xx in range(12):
        if 0 <= xx + s < 12:
            ref[xx] = x[0, 0, xx + s]
    assert np.array_equal(ol.conv(x, w)[0, 0], ref)


@pytest.mark.parametrize("cin,cout,n", [(1, 32, 40), (32, 32, 17), (32, 1, 9), (3, 5, 2)])
def test_backward_data_is_adjoint(cin, cout, n):
    rng = np.random.default_rng(cin * 100 + cout + n)
    x = rng.standard_normal((3, cin, n))
    y = rng.standard_normal((3, cout, n))
    w = rng.standard_normal((cout, cin, 9))
    lhs = float(np.sum(ol.conv(x, w) * y))
    rhs = float(np.sum(x * ol.conv_backward_data(y, w)))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * np.abs(w).sum()


def test_backward_weight_by_unit_weights():
    """L(w, b) = <conv(x, w, b), g> is linear: dL/dw[o,i,t] = L(e_oit, 0)."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 3, 13))
    g = rng.standard_normal((2, 2, 13))
    gw, gb = ol.conv_backward_weight(x, g)
    for o in range(2):
        for i in range(3):
            for t in range(9):
                e = np.zeros((2, 3, 9))
                e[o, i, t] = 1.0
                assert math.isclose(gw[o, i, t], float(np.sum(brute_conv(x, e, np.zeros(2)) * g)),
                                    rel_tol=1e-12, abs_tol=1e-12)
    for o in range(2):
        eb = np.zeros(2)
        eb[o] = 1.0
        assert math.isclose(gb[o], float(np.sum(brute_conv(x, np.zeros((2, 3, 9)), eb) * g)),
                            rel_tol=1e-12)


@pytest.mark.parametrize("residual", [True, False])
def test_net_gradient_by_central_differences(residual):
    rng = np.random.default_rng(11)
    q = rng.standard_normal((4, 37))
    ramp = rng.standard_normal((4, 37)) if residual else None
    gy = rng.standard_normal((4, 37))
    p = ol.init_params(3, residual=False)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    alpha = 0.7
    y, cache = ol.net_forward(q, p, alpha, ramp)
    g = ol.net_backward(gy, p, alpha, cache)
    d = {k: rng.standard_normal(p[k].shape) for k in p}
    h = 1e-5

    def L(s):
        pp = {k: p[k] + s * d[k] for k in p}
        return float(np.sum(ol.net_forward(q, pp, alpha, ramp)[0] * gy))
    fd = (L(h) - L(-h)) / (2 * h)
    an = sum(float(np.sum(g[k] * d[k])) for k in p)
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_residual_form_starts_at_ramp():
    p = ol.init_params(5, residual=True)
    rng = np.random.default_rng(5)
    q = rng.standard_normal((3, 20))
    ramp = rng.standard_normal((3, 20))
    y, _ = ol.net_forward(q, p, 1.3, ramp)
    assert np.array_equal(y, ramp)


def test_cosine_weight_is_ray_cosine():
    """sdd / |ray| equals the cosine between the ray to the pixel and the
    principal ray, computed from the world positions of source and pixel
    (detector centre, axes and pitches of the circular orbit)."""
    scan = dict(wl.CONFIGS["c1"]["scan"], theta0=0.3, u_off=1.5, v_off=-2.0)
    nh, nw = 7, 9
    raw = np.ones((1, nh, nw))
    got = ol.cosine_weight(raw, scan)[0]
    th = scan["theta0"]
    e_r = np.array([math.cos(th), math.sin(th), 0.0])
    e_u = np.array([-math.sin(th), math.cos(th), 0.0])
    e_v = np.array([0.0, 0.0, 1.0])
    src = scan["sod"] * e_r
    det = -(scan["sdd"] - scan["sod"]) * e_r
    cu = (nw - 1) / 2 + scan["u_off"]
    cv = (nh - 1) / 2 + scan["v_off"]
    for r in range(nh):
        for c in range(nw):
            pix = det + (c - cu) * scan["du"] * e_u + (r - cv) * scan["dv"] * e_v
            ray = pix - src
            cosang = float(np.dot(ray, -e_r)) / np.linalg.norm(ray)
            assert math.isclose(got[r, c], cosang, rel_tol=1e-13)


def test_cosine_weight_then_ramp_is_fdk_filter():
    """The C oracle's filter = Ram-Lak correlation of the numpy cosine-weighted
    rows, times tau arc / (2 np)."""
    scan = dict(wl.CONFIGS["c1"]["scan"], u_off=0.5, v_off=-1.0)
    rng = np.random.default_rng(9)
    raw = rng.standard_normal((2, 5, 33))
    q = ol.cosine_weight(raw, scan)
    tau = scan["du"] * scan["sod"] / scan["sdd"]
    n = np.arange(-32, 33)
    h = np.zeros(n.size)
    h[n == 0] = 1 / (4 * tau * tau)
    odd = n % 2 != 0
    h[odd] = -1 / (math.pi ** 2 * n[odd] ** 2 * tau * tau)
    ref = np.zeros_like(q)
    for s in range(2):
        for r in range(5):
            ref[s, r] = np.convolve(q[s, r], h, mode="full")[32:32 + 33]
    ref *= tau * scan["arc"] / (2 * 17)
    got = oracle.fdk_filter(raw, scan, np_total=17)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_sqerr_closed_form():
    b = np.random.default_rng(2).standard_normal(50)
    loss, grad = ol.sqerr(b + 0.25, b)
    assert math.isclose(loss, 50 * 0.0625, rel_tol=1e-12)
    assert np.allclose(grad, 2 * 0.25 / 50, rtol=1e-12)


def test_adam_first_step_and_constant_gradient():
    g = np.array([3.0, -0.5, 1e-3])
    p0 = np.array([1.0, 2.0, -1.0])
    lr, eps = 0.01, 1e-8
    p, m, v = ol.adam(p0, g, np.zeros(3), np.zeros(3), 1, lr, eps=eps)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=1e-13)
    # constant gradient: bias-corrected moments are exactly g and g^2 at every step
    for t in range(2, 30):
        p, m, v = ol.adam(p, g, m, v, t, lr, eps=eps)
    assert np.allclose(p, p0 - 29 * lr * g / (np.abs(g) + eps), rtol=1e-10)


def test_adam_minimises_quadratic():
    p, m, v = np.array([5.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        p, m, v = ol.adam(p, 2 * (p - 1.5), m, v, t, 0.05)
    assert abs(p[0] - 1.5) < 1e-3
