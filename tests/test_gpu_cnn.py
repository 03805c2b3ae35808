"""GPU parity of the learned tile proposal and of the routed exact fallback.

Network kernels (pack, forward, backward, Adam, tile targets) are compared
with the fp64 oracle in oracle/cnn_ref.py on the same bf16 inputs and
weights.  Both sides round weights, activations and activation gradients to
bf16 with ties to even, so the only differences are the fp32 accumulation
order of the MFMA sums and the rare bf16 rounding decision that this order
flips; the tolerances below follow from that (derivation in each test).

The routed fallback is held to the exact path's bar: on tiles the logits
leave uncertain the mask is bit-identical to the oracle's exact mask, and
filled tiles hold exactly their fill value.
"""
import math

import numpy as np
import pytest

from oracle import cnn_ref
from paper_2408_14050_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    return t


@pytest.fixture(scope="module")
def gctx(torch):
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    yield ctx
    ctx.occl_release()


def bf16_to_f64(x_int16):
    u = np.ascontiguousarray(x_int16).view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def f64_to_bf16_bits(x):
    """bf16 bit patterns (int16 storage) of the oracle's bf16 rounding."""
    r = cnn_ref.bf16(x).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def rand_input(rng, N, H, W):
    x = rng.normal(size=(N, H, W, 8))
    x[..., 7] = 0.0
    return f64_to_bf16_bits(x)


def rand_theta(rng, scale=1.0):
    """He-like random weights and small random biases (every layer active)."""
    th = []
    for ci, co, _, _ in cnn_ref.LAYERS:
        th.append(rng.uniform(-1, 1, size=co * 9 * ci) * math.sqrt(6.0 / (9 * ci)) * scale)
        th.append(rng.normal(scale=0.05, size=co))
    return np.concatenate(th).astype(np.float32)


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------------------
# pack
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [5, 6])
def test_pack_matches_oracle(gctx, torch, ref, seed):
    sc = scenes.make_scene("c0", seed)
    D = to_dev(torch, sc.D.astype(np.float32))
    angles = np.array([0.0, 45.0, 180.0, 292.5])
    ratios = np.array([1.0, 1.4142135, 2.0, 0.75], np.float32)
    Ls = np.array([32, 45, 60, 24], np.int32)
    X = gctx.occl_cnn_pack(D, angles, ratios, Ls).cpu().numpy()
    got = bf16_to_f64(X)
    for v in range(4):
        c, sn = ref.direction(angles[v])
        exp = cnn_ref.pack(sc.D, float(c), float(sn), ratios[v], Ls[v])
        # both sides round to bf16; a different fp32 / fp64 intermediate may
        # move a value across a bf16 rounding boundary: at most 1 bf16 ulp
        # (relative 2^-7), and rarely
        ulp = np.maximum(np.abs(exp), 1e-30) * 2.0 ** -7
        assert np.all(np.abs(got[v] - exp) <= ulp + 1e-30), f"view {v}"
        assert np.mean(got[v] != exp) < 1e-3, f"view {v}"


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------
def conv_layer_ref(x, theta, li):
    """Layer li of the oracle network on the bf16 input x (fp64 result)."""
    w, b = cnn_ref.unflatten(theta.astype(np.float64))[li]
    _, _, stride, relu = cnn_ref.LAYERS[li]
    y = cnn_ref.conv3x3(x, cnn_ref.bf16(w), b, stride)
    return np.maximum(y, 0.0) if relu else y


@pytest.mark.parametrize("shape", [(2, 70, 90), (1, 256, 256), (3, 33, 17), (1, 16, 16), (1, 1, 1)])
def test_forward_layers_match_oracle(gctx, torch, shape):
    """Every layer against the oracle layer applied to the GPU's own input
    of that layer: the sums are the same bf16 products (fp32 accumulation
    on the GPU, fp64 in the oracle), so a bf16 output can only differ where
    the exact sum lies within the fp32 accumulation error (~ sqrt(K) 2^-24
    relative, K <= 288) of a bf16 rounding midpoint: at most 1 bf16 ulp,
    on a small fraction of the elements.  The fp32 logits agree to 1e-5
    relative of the sum of the magnitudes of their terms."""
    N, H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    theta = rand_theta(rng)
    gctx.occl_cnn_set_state(theta)
    Xb = rand_input(rng, N, H, W)
    Z = gctx.occl_cnn_forward(to_dev(torch, Xb)).cpu().numpy().astype(np.float64)
    x = bf16_to_f64(Xb)
    for li in range(5):
        got = bf16_to_f64(gctx.occl_cnn_activation(li, N, H, W).cpu().numpy())
        exp = cnn_ref.bf16(conv_layer_ref(x, theta, li))
        assert got.shape == exp.shape
        diff = got != exp
        # 1 bf16 ulp, or the accumulation error itself where the sum sits at
        # the ReLU's kink (tiny positive on one side, clamped on the other)
        w, b = cnn_ref.unflatten(theta.astype(np.float64))[li]
        mag = cnn_ref.conv3x3(np.abs(x), np.abs(cnn_ref.bf16(w)), np.abs(b), cnn_ref.LAYERS[li][2])
        tol = 2.0 ** -7 * np.maximum(np.abs(exp), np.abs(got)) + 1e-5 * mag
        assert np.all(np.abs(got - exp) <= tol), (li, np.abs(got - exp).max())
        assert diff.mean() <= 2e-3, (li, diff.mean())
        x = got
    zr = conv_layer_ref(x, theta, 5)[..., 0]
    w5, b5 = cnn_ref.unflatten(theta.astype(np.float64))[5]
    mag = cnn_ref.conv3x3(np.abs(x), np.abs(cnn_ref.bf16(w5)), np.abs(b5), 1)[..., 0]
    assert np.all(np.abs(Z - zr) <= 1e-5 * mag + 1e-7)


@pytest.mark.parametrize("shape", [(2, 70, 90), (1, 256, 256)])
def test_forward_end_to_end_close_to_oracle(gctx, torch, shape):
    """Whole network on both sides independently.  bf16 rounding flips from
    the different accumulation order (see above) propagate, so the logits
    agree only to about 1 % of their RMS; any indexing mistake (a wrong tap,
    channel or stride) is off by O(1)."""
    N, H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    theta = rand_theta(rng)
    gctx.occl_cnn_set_state(theta)
    Xb = rand_input(rng, N, H, W)
    Z = gctx.occl_cnn_forward(to_dev(torch, Xb)).cpu().numpy().astype(np.float64)
    Zr, _ = cnn_ref.forward(theta.astype(np.float64), bf16_to_f64(Xb))
    scale = np.sqrt(np.mean(Zr ** 2)) + 1e-3
    err = np.abs(Z - Zr)
    assert err.max() <= 3e-2 * scale, (err.max(), scale)
    assert err.mean() <= 3e-3 * scale, (err.mean(), scale)


# ---------------------------------------------------------------------------
# backward, Adam, targets
# ---------------------------------------------------------------------------
def layer_slices():
    out, k = [], 0
    for ci, co, _, _ in cnn_ref.LAYERS:
        n = co * 9 * ci + co
        out.append(slice(k, k + n))
        k += n
    return out


# (9, 256, 256): more than 64 weight-gradient partials in layers 0 and 1 and in
# the last layer (576, 144 and 72), so both levels of the ordered partial sums
# run, with a partly filled last group in layer 1 and the last layer
@pytest.mark.parametrize("shape", [(2, 64, 80), (1, 100, 36), (9, 256, 256)])
def test_backward_matches_oracle(gctx, torch, shape):
    N, H, W = shape
    rng = np.random.default_rng(7 + H)
    theta = rand_theta(rng)
    gctx.occl_cnn_set_state(theta)
    Xb = rand_input(rng, N, H, W)
    T = rng.uniform(size=(N, -(-H // 16), -(-W // 16))).astype(np.float32)
    loss, g = gctx.occl_cnn_backward(to_dev(torch, Xb), to_dev(torch, T))
    loss_r, g_r = cnn_ref.backward(theta.astype(np.float64), bf16_to_f64(Xb), T.astype(np.float64))
    assert abs(loss - loss_r) <= 1e-5 * abs(loss_r) + 1e-7
    # per layer: the gradients are sums over all pixels of bf16 products in
    # fp32; rare bf16 flips of activation gradients (relative 2^-8 each) add
    # up to well under 1 % of the layer's gradient norm
    for li, sl in enumerate(layer_slices()):
        a, b = g[sl].astype(np.float64), g_r[sl]
        nrm = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 1e-2 * nrm + 1e-9, (li, np.linalg.norm(a - b), nrm)
        assert float(a @ b) >= 0.9999 * np.linalg.norm(a) * nrm - 1e-12, li


@pytest.mark.parametrize("shape", [(2, 48, 64), (9, 256, 256)])
def test_backward_is_deterministic(gctx, torch, shape):
    N, H, W = shape
    rng = np.random.default_rng(11)
    theta = rand_theta(rng)
    gctx.occl_cnn_set_state(theta)
    X = to_dev(torch, rand_input(rng, N, H, W))
    T = to_dev(torch, rng.uniform(size=(N, -(-H // 16), -(-W // 16))).astype(np.float32))
    l1, g1 = gctx.occl_cnn_backward(X, T)
    l2, g2 = gctx.occl_cnn_backward(X, T)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)


def test_adam_step_matches_oracle(gctx, torch):
    rng = np.random.default_rng(12)
    theta = rand_theta(rng)
    n = theta.size
    m0 = rng.normal(scale=1e-3, size=n).astype(np.float32)
    v0 = rng.uniform(0, 1e-5, size=n).astype(np.float32)
    gctx.occl_cnn_set_state(theta, m0, v0, step=4)
    X = to_dev(torch, rand_input(rng, 2, 48, 48))
    T = to_dev(torch, rng.uniform(size=(2, 3, 3)).astype(np.float32))
    _, g = gctx.occl_cnn_backward(X, T)
    gctx.occl_cnn_train_step(X, T, lr=1e-3)
    th1, m1, v1, step = gctx.occl_cnn_get_state()
    assert step == 5
    exp_th, exp_m, exp_v = cnn_ref.adam(theta.astype(np.float64), g.astype(np.float64),
                                        m0.astype(np.float64), v0.astype(np.float64), 5, 1e-3)
    # fp32 moments: each term rounded once (plus 0.9f, 0.999f as fp32
    # constants), so the error is ~1e-6 of the terms' magnitudes
    gd = g.astype(np.float64)
    tol_m = 1e-6 * (0.9 * np.abs(m0) + 0.1 * np.abs(gd)) + 1e-30
    tol_v = 1e-6 * (0.999 * v0 + 0.001 * gd * gd) + 1e-30
    assert np.all(np.abs(m1 - exp_m) <= tol_m)
    assert np.all(np.abs(v1 - exp_v) <= tol_v)
    # fp32 update of size <= lr: error a few fp32 ulps of theta plus ~1e-6 lr
    np.testing.assert_allclose(th1, exp_th, rtol=1e-6, atol=1e-8)


def test_state_roundtrip_and_resume(gctx, torch):
    """Checkpoint / resume: a run split by get_state / set_state is
    bit-identical to the uninterrupted run."""
    from paper_2408_14050_amd import occl
    rng = np.random.default_rng(13)
    X = to_dev(torch, rand_input(rng, 2, 64, 64))
    T = to_dev(torch, rng.uniform(size=(2, 4, 4)).astype(np.float32))
    gctx.occl_cnn_init(99)
    for _ in range(3):
        gctx.occl_cnn_train_step(X, T, 1e-3)
    ck = gctx.occl_cnn_get_state()
    for _ in range(3):
        gctx.occl_cnn_train_step(X, T, 1e-3)
    full = gctx.occl_cnn_get_state()
    other = occl.Context(0)
    try:
        other.occl_cnn_set_state(ck[0], ck[1], ck[2], ck[3])
        for _ in range(3):
            other.occl_cnn_train_step(X, T, 1e-3)
        resumed = other.occl_cnn_get_state()
    finally:
        other.occl_release()
    for a, b in zip(full[:3], resumed[:3]):
        np.testing.assert_array_equal(a, b)
    assert full[3] == resumed[3] == 6


def test_init_is_seeded(gctx):
    gctx.occl_cnn_init(5)
    a = gctx.occl_cnn_get_state()[0]
    gctx.occl_cnn_init(5)
    b = gctx.occl_cnn_get_state()[0]
    gctx.occl_cnn_init(6)
    c = gctx.occl_cnn_get_state()[0]
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.size == cnn_ref.n_params() == 39617


def test_training_reduces_loss(gctx, torch):
    """A few hundred Adam steps on tile targets of exact masks lower the loss."""
    from paper_2408_14050_amd import occl
    rng = np.random.default_rng(21)
    Xs, Ts = [], []
    for seed in range(4):
        sc = scenes.make_scene("c0", 300 + seed)
        D = to_dev(torch, sc.D.astype(np.float32))
        angles = np.array([0.0, 90.0, 180.0, 270.0])
        ratios = np.ones(4, np.float32)
        Ls = np.full(4, 32, np.int32)
        M = gctx.occl_detect(D, angles, ratios, occl.params(scan_len=32, flags=occl.FLAG_SYNC))
        Xs.append(gctx.occl_cnn_pack(D, angles, ratios, Ls))
        Ts.append(gctx.occl_cnn_tile_targets(M))
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    gctx.occl_cnn_init(1)
    first = gctx.occl_cnn_train_step(X, T, 2e-3)
    for _ in range(150):
        last = gctx.occl_cnn_train_step(X, T, 2e-3)
    assert last < 0.6 * first, (first, last)


def test_tile_targets_match_oracle(gctx, torch):
    rng = np.random.default_rng(14)
    M = (rng.uniform(size=(3, 37, 50)) < 0.3).astype(np.uint8)
    M[1] = 0
    M[2, :16, :16] = 1
    T = gctx.occl_cnn_tile_targets(to_dev(torch, M)).cpu().numpy()
    exp = cnn_ref.tile_fraction(M).astype(np.float32)  # count / area, rounded once
    np.testing.assert_array_equal(T, exp)


def test_cnn_calls_validate(gctx, torch):
    from paper_2408_14050_amd import occl
    other = occl.Context(0)
    try:
        X = torch.zeros((1, 16, 16, 8), dtype=torch.int16, device="cuda")
        with pytest.raises(occl.OcclError) as e:
            other.occl_cnn_forward(X)
        assert e.value.status == -5  # no model
        other.occl_cnn_init(0)
        with pytest.raises(occl.OcclError):
            other.occl_cnn_set_state(np.full(cnn_ref.n_params(), np.nan, np.float32))
        with pytest.raises(ValueError):
            other.occl_cnn_set_state(np.zeros(10, np.float32))
        T = torch.zeros((1, 1, 1), dtype=torch.float32, device="cuda")
        with pytest.raises(occl.OcclError):
            other.occl_cnn_train_step(X, T, lr=0.0)
    finally:
        other.occl_release()


# ---------------------------------------------------------------------------
# routed exact fallback
# ---------------------------------------------------------------------------
def tile_states(z, lo, hi):
    """The oracle's routing rule (probability band -> fill 0 / fill 1 / exact)."""
    return cnn_ref.tile_states(z, lo, hi)


def expand(st, H, W):
    return np.repeat(np.repeat(st, 16, axis=-2), 16, axis=-1)[..., :H, :W]


def check_routed(M, M_exact, st, what):
    V, H, W = M_exact.shape
    full = expand(st, H, W)
    ex = full == 2
    bad = int((M[ex] != M_exact[ex]).sum())
    assert bad == 0, f"{what}: {bad} mismatches on exact tiles"
    assert np.all(M[full == 0] == 0), what
    assert np.all(M[full == 1] == 1), what


@pytest.mark.parametrize("cfg,seed", [("c0", 3), ("c0", 4), ("c1", 1003)])
@pytest.mark.parametrize("band", [(0.05, 0.95), (0.3, 0.7), (0.0, 1.0), (0.5, 0.5)])
def test_routed_matches_oracle_on_exact_tiles(gctx, torch, ref, cfg, seed, band):
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene(cfg, seed)
    V, (H, W) = sc.n_views, sc.D.shape
    rng = np.random.default_rng(seed)
    z = rng.normal(scale=3.0, size=(V, -(-H // 16), -(-W // 16))).astype(np.float32)
    z[0, 0, 0] = np.nan
    M_ref, _, _ = ref.detect_scene(sc)
    D = to_dev(torch, sc.D.astype(np.float32))
    st_dev = torch.empty(z.shape, dtype=torch.uint8, device="cuda")
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC,
                      cnn_lo=band[0], cnn_hi=band[1])
    M = gctx.occl_detect_routed(D, sc.angles, sc.ratios, prm, to_dev(torch, z),
                                tile_state=st_dev).cpu().numpy()
    st = tile_states(z, *band)
    np.testing.assert_array_equal(st_dev.cpu().numpy(), st)
    check_routed(M, M_ref, st, f"{cfg} seed {seed} band {band}")
    if band == (0.0, 1.0):
        np.testing.assert_array_equal(M, M_ref)


def test_routed_ragged_and_diagonal(gctx, torch, ref):
    """Frame sizes off the tile grid, diagonal and odd-angle views, long L."""
    from paper_2408_14050_amd import occl
    rng = np.random.default_rng(77)
    for H, W in [(61, 83), (130, 47), (17, 300)]:
        sc = scenes.make_scene("c0", int(rng.integers(1000)))
        D = np.ascontiguousarray(sc.D[:H, :W]) if sc.D.shape[0] >= H and sc.D.shape[1] >= W else None
        if D is None:
            D = rng.uniform(0, 20, size=(H, W)).astype(np.float32)
            D[H // 3:2 * H // 3, W // 3:2 * W // 3] += 15
        angles = np.array([0.0, 45.0, 135.0, 200.0, 333.0])
        ratios = np.array([1.0, 1.4142135, 1.4142135, 0.8, 2.5], np.float32)
        L = np.array([33, 48, 90, 20, 120], np.int32)
        z = rng.normal(scale=2.0, size=(5, -(-H // 16), -(-W // 16))).astype(np.float32)
        M_ref, _, _ = ref.detect(D, angles, ratios, L)
        prm = occl.params(scan_len_per_view=L, flags=occl.FLAG_SYNC, cnn_lo=0.2, cnn_hi=0.8)
        M = gctx.occl_detect_routed(to_dev(torch, D.astype(np.float32)), angles, ratios, prm,
                                    to_dev(torch, z)).cpu().numpy()
        check_routed(M, M_ref, tile_states(z, 0.2, 0.8), f"{H}x{W}")


def test_use_cnn_equals_forward_then_routed(gctx, torch, ref):
    """occl_detect with the learned proposal = pack -> forward -> routed."""
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c1", 1004)
    D = to_dev(torch, sc.D.astype(np.float32))
    gctx.occl_cnn_init(3)
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len,
                      flags=occl.FLAG_SYNC | occl.FLAG_USE_CNN, cnn_lo=0.3, cnn_hi=0.7)
    M_cnn = gctx.occl_detect(D, sc.angles, sc.ratios, prm).cpu().numpy()
    X = gctx.occl_cnn_pack(D, sc.angles, sc.ratios, sc.scan_len)
    Z = gctx.occl_cnn_forward(X)
    prm2 = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC,
                       cnn_lo=0.3, cnn_hi=0.7)
    M_r = gctx.occl_detect_routed(D, sc.angles, sc.ratios, prm2, Z).cpu().numpy()
    np.testing.assert_array_equal(M_cnn, M_r)
    M_ref, _, _ = ref.detect_scene(sc)
    check_routed(M_cnn, M_ref, tile_states(Z.cpu().numpy(), 0.3, 0.7), "use_cnn")


def test_routed_validates(gctx, torch):
    from paper_2408_14050_amd import occl
    D = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    z = torch.zeros((1, 2, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(occl.OcclError):
        gctx.occl_detect_routed(D, [0.0], [1.0], occl.params(scan_len=8, cnn_lo=0.9, cnn_hi=0.1), z)
    with pytest.raises(occl.OcclError):
        from paper_2408_14050_amd.occl import lib, _ptr
        import ctypes as C
        a = np.zeros(1); r = np.ones(1, np.float32)
        p = occl.params(scan_len=8)
        M = torch.empty((1, 32, 32), dtype=torch.uint8, device="cuda")
        st = lib().occl_detect_routed(gctx.h, _ptr(D), 32, 32, 1, a.ctypes.data_as(C.POINTER(C.c_double)),
                                      r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(p), None,
                                      _ptr(M), None)
        gctx._check(st, "routed without logits")


def test_committed_weights_quality(gctx, torch, record_property):
    """The shipped proposal (trained by train_tile_cnn on 20k crops, its
    logits temperature-calibrated on frames 4200..4215) on held-out
    1920x1080 frames at the configured band [0.05, 0.95]: IoU of the
    routed masks against the exact masks (Eq. 7 counts) must reach 0.99.
    The speed of CNN + fallback against the exact path is measured and
    recorded; the target (faster than exact) is not met on this GPU: the
    exact path already skips the tiles the network is confident about."""
    import time
    from paper_2408_14050_amd import occl
    from paper_2408_14050_amd.train_tile_cnn import load_state
    meta = load_state(gctx)
    assert meta["frames"] * meta["crops_per_frame"] >= 20000
    assert "calibration" in meta and meta["calibration"]["band"] == [0.05, 0.95]
    angles, ratios = scenes.views_3x3()
    tp = fp = fn = 0
    for seed in (4100, 4101, 4115):
        sc = scenes.make_c1_like(seed, W=1920, H=1080)
        D = to_dev(torch, sc.D)
        M = gctx.occl_detect(D, angles, ratios, occl.params(scan_len_per_view=sc.scan_len))
        prm = occl.params(scan_len_per_view=sc.scan_len, flags=occl.FLAG_USE_CNN | occl.FLAG_SYNC)
        assert (prm.cnn_lo, prm.cnn_hi) == pytest.approx((0.05, 0.95))
        Mc = gctx.occl_detect(D, angles, ratios, prm)
        c = gctx.occl_confusion(Mc, M)
        tp, fp, fn = tp + c["tp"], fp + c["fp"], fn + c["fn"]
    iou = tp / max(1, tp + fp + fn)
    record_property("iou_band_0.05_0.95", iou)
    assert iou >= 0.99, (tp, fp, fn)

    def timed(p, reps=30):
        for _ in range(3):
            gctx.occl_detect(D, angles, ratios, p, M=M)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gctx.occl_detect(D, angles, ratios, p, M=M)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_exact = timed(occl.params(scan_len_per_view=sc.scan_len))
    t_cnn = timed(occl.params(scan_len_per_view=sc.scan_len, flags=occl.FLAG_USE_CNN))
    ratio = t_exact / t_cnn
    record_property("speed_vs_exact", ratio)
    print(f"CNN + fallback: IoU {iou:.5f} at [0.05, 0.95]; {t_cnn * 1e3:.4f} ms against "
          f"{t_exact * 1e3:.4f} ms exact, speed ratio {ratio:.3f} (target > 1: not met)", flush=True)
    assert ratio > 0


@pytest.mark.parametrize("shape", [(192, 256), (61, 83), (1080, 1920), (17, 300), (1, 1)])
def test_propose_equals_pack_then_forward(gctx, torch, shape):
    """occl_cnn_propose (packing fused into the first layer, all views per
    tile) gives the same logits, bit for bit, as packing every view and
    running the network on the packed input."""
    H, W = shape
    rng = np.random.default_rng(H + W)
    gctx.occl_cnn_set_state(rand_theta(rng))
    D = rng.uniform(0, 30, size=(H, W)).astype(np.float32)
    D[H // 4:H // 2, W // 3:W // 2] += 12.0
    Dt = to_dev(torch, D)
    angles = np.array([0.0, 45.0, 90.0, 135.0, 200.0, 333.0])
    ratios = np.array([1.0, 1.4142135, 1.0, 1.4142135, 0.8, 2.5], np.float32)
    Ls = np.array([33, 48, 51, 70, 20, 120], np.int32)
    from paper_2408_14050_amd import occl
    Z1 = gctx.occl_cnn_propose(Dt, angles, ratios, Ls).cpu().numpy()
    a1 = gctx.occl_cnn_activation(1, 6, H, W).cpu().numpy()
    with pytest.raises(occl.OcclError):  # layer 0 stays in LDS on this path
        gctx.occl_cnn_activation(0, 6, H, W)
    X = gctx.occl_cnn_pack(Dt, angles, ratios, Ls)
    Z2 = gctx.occl_cnn_forward(X).cpu().numpy()
    b1 = gctx.occl_cnn_activation(1, 6, H, W).cpu().numpy()
    np.testing.assert_array_equal(a1, b1)
    np.testing.assert_array_equal(Z1, Z2)
