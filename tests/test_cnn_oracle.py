"""Pins of the CNN oracle (oracle/cnn_ref.py) against library routines,
finite differences and closed forms."""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import cnn_ref as C


@pytest.mark.parametrize("stride", [1, 2])
@pytest.mark.parametrize("shape", [(5, 7), (8, 8), (9, 4)])
def test_conv_matches_scipy_correlate(stride, shape):
    rng = np.random.default_rng(1)
    H, W = shape
    x = rng.normal(size=(2, H, W, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = C.conv3x3(x, w, b, stride)
    for n in range(2):
        for co in range(4):
            ref = sum(signal.correlate2d(x[n, :, :, ci], w[co, :, :, ci], mode="same") for ci in range(3))
            ref = ref[::stride, ::stride] + b[co]
            np.testing.assert_allclose(y[n, :, :, co], ref, rtol=1e-12, atol=1e-12)
    assert y.shape[1:3] == (math.ceil(H / stride), math.ceil(W / stride))


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 5, 6, 2))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=3)
    gy = rng.normal(size=C.conv3x3(x, w, b, stride).shape)
    gx, gw, gb = C.conv3x3_backward(x, w, gy, stride)
    f = lambda xx, ww, bb: float((gy * C.conv3x3(xx, ww, bb, stride)).sum())
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 4, 5, 1), (0, 2, 3, 0)]:
        e = np.zeros_like(x); e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - gx[idx]) < 1e-6
    for idx in [(0, 0, 0, 0), (2, 2, 1, 1), (1, 1, 1, 0)]:
        e = np.zeros_like(w); e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - gw[idx]) < 1e-6
    e = np.zeros_like(b); e[1] = h
    assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * h) - gb[1]) < 1e-6


def test_bce_closed_form_and_gradient():
    loss, g = C.bce(np.zeros((2, 3)), np.full((2, 3), 0.25))
    assert abs(loss - math.log(2.0)) < 1e-15
    np.testing.assert_allclose(g, (0.5 - 0.25) / 6)
    z = np.array([[-3.0, 0.4], [2.5, 7.0]])
    t = np.array([[0.0, 0.3], [1.0, 0.6]])
    _, g = C.bce(z, t)
    h = 1e-6
    for i in range(2):
        for j in range(2):
            e = np.zeros_like(z); e[i, j] = h
            num = (C.bce(z + e, t)[0] - C.bce(z - e, t)[0]) / (2 * h)
            assert abs(num - g[i, j]) < 1e-8


def test_network_gradient_finite_differences():
    """Whole-network backward (no bf16 rounding) against central differences."""
    rng = np.random.default_rng(3)
    theta = rng.normal(scale=0.3, size=C.n_params())
    x = rng.normal(size=(2, 32, 32, 8))
    t = rng.uniform(size=(2, 2, 2))
    loss, g = C.backward(theta, x, t, round_bf16=False)
    h = 1e-5
    for k in rng.choice(C.n_params(), size=25, replace=False):
        e = np.zeros_like(theta); e[k] = h
        lp = C.bce(C.forward(theta + e, x, False)[0], t)[0]
        lm = C.bce(C.forward(theta - e, x, False)[0], t)[0]
        num = (lp - lm) / (2 * h)
        assert abs(num - g[k]) <= 1e-6 + 1e-4 * abs(num), (k, num, g[k])


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    grad = rng.normal(size=50)
    new, m, v = C.adam(theta, grad, np.zeros(50), np.zeros(50), 1, 0.01)
    # |step| = lr * |g| / (|g| + eps): within eps / |g| of lr
    np.testing.assert_allclose(theta - new, 0.01 * np.sign(grad), rtol=1e-4)


def test_bf16_rounding():
    """bf16 keeps 7 mantissa bits: spacing 2^-7 at 1; halfway cases go to even."""
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5, 3.140625])
    np.testing.assert_array_equal(C.bf16(vals), [1.0, 1.0, 1.0, 1.0 + 2 ** -7, -2.5, 3.140625])


def test_pack_and_tiles():
    D = np.full((20, 24), 3.0)
    D[5:15, 8:20] = 11.0
    c = s = math.cos(math.pi / 4)
    x = C.pack(D, c, s, np.float32(1.4142135), 30)
    assert np.all(x[..., 4] == C.bf16(np.cos(np.pi / 4))) and np.all(x[..., 7] == 0)
    mag = x[..., 2] ** 2 + x[..., 3] ** 2
    assert np.all(np.abs(mag - 1) < 0.02)
    M = np.zeros((2, 40, 35))
    M[1, :16, :16] = 1
    M[1, 16:32, 0:8] = 1
    f = C.tile_fraction(M)
    assert f.shape == (2, 3, 3) and f[0].sum() == 0
    assert f[1, 0, 0] == 1.0 and f[1, 1, 0] == 0.5 and f[1, 2, 2] == 0.0


def test_pack_angle_channels_are_cos_sin_of_atan2():
    """Channels 2, 3 are cos and sin of A = atan2(E_y, E_x) of Eq. (1)."""
    rng = np.random.default_rng(5)
    D = rng.normal(size=(20, 30)) * 3
    x = C.pack(D, math.cos(math.pi / 6), 0.5, np.float32(1.0), 10)
    ex = np.zeros_like(D)
    ey = np.zeros_like(D)
    ex[:, :-1] = D[:, 1:] - D[:, :-1]
    ey[:-1, :] = D[1:, :] - D[:-1, :]
    A = np.arctan2(ey, ex)
    assert np.abs(x[..., 2] - C.bf16(np.cos(A))).max() < 1e-15
    assert np.abs(x[..., 3] - C.bf16(np.sin(A))).max() < 1e-15
    # last row: E_y = 0, so sin A is exactly 0 and cos A = sign(E_x)
    assert np.all(x[-1, :, 3] == 0.0)
    assert np.all(np.abs(x[-1, :-1, 2]) == 1.0)
    # E = 0 (last pixel): A = atan2(0, 0) = 0
    assert x[-1, -1, 2] == 1.0 and x[-1, -1, 3] == 0.0
    np.testing.assert_array_equal(x[..., 1], C.bf16(np.hypot(ex, ey) / 8.0))


@pytest.mark.parametrize("band", [(0.05, 0.95), (0.02, 0.98), (0.3, 0.7), (0.5, 0.5), (0.0, 1.0), (0.2, 1.0)])
def test_tile_routing_rule(band):
    """The routing states against their definition by probabilities: a tile
    is filled with 0 when sigmoid(z) < lo, with 1 when sigmoid(z) > hi, else
    it takes the exact path.  The bounds are the logits of lo and hi rounded
    to fp32, so the rule is checked (a) against sigmoid itself wherever z is
    more than 1e-5 from a bound, (b) exactly on the fp32 neighbours of each
    rounded bound, (c) on infinities, signed zeros and NaN (exact path)."""
    lo, hi = band
    z = np.concatenate([np.linspace(-12, 12, 2001, dtype=np.float32),
                        np.array([-np.inf, np.inf, 0.0, -0.0], np.float32)])
    bounds = {p: np.float32(math.log(p / (1 - p))) for p in (lo, hi) if 0 < p < 1}
    for b in bounds.values():
        z = np.concatenate([z, [np.nextafter(b, np.float32(-np.inf)), b, np.nextafter(b, np.float32(np.inf))]])
    st = C.tile_states(z, lo, hi)
    for zz, s in zip(z.tolist(), st.tolist()):
        if math.isfinite(zz) and all(abs(zz - math.log(p / (1 - p))) > 1e-5 for p in bounds):
            sg = 1.0 / (1.0 + math.exp(-zz))
            assert s == (0 if sg < lo else (1 if sg > hi else 2)), (zz, s)
        zl = bounds.get(lo, -math.inf if lo <= 0 else math.inf)
        zh = bounds.get(hi, math.inf if hi >= 1 else -math.inf)
        assert s == (0 if zz < zl else (1 if zz > zh else 2)), (zz, s)
    assert C.tile_states(np.array([np.nan], np.float32), lo, hi)[0] == 2
    assert C.tile_states(np.array([-np.inf, np.inf], np.float32), 0.0, 1.0).tolist() == [2, 2]
