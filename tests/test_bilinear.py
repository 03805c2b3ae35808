"""The bilinear-V variant (OCCL_FLAG_BILINEAR): oracle pins on the CPU and
GPU parity, bit for bit."""
import numpy as np
import pytest

from paper_2408_14050_amd import scenes


def test_bilinear_reproduces_affine_maps(ref):
    """Bilinear interpolation is exact for affine functions: on
    D = a + b x + c y (values exact in fp32) the sample at any real position
    is a + b px + c py up to fp32 rounding."""
    H, W = 40, 60
    y, x = np.mgrid[0:H, 0:W]
    a, b, c = 10.0, 0.25, -0.5
    D = (a + b * x + c * y).astype(np.float32)
    rng = np.random.default_rng(0)
    for _ in range(200):
        px, py = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        px, py = np.float32(px), np.float32(py)
        v = ref.sample(D, px, py, bilinear=True)
        assert abs(float(v) - (a + b * float(px) + c * float(py))) < 2e-5


def test_bilinear_at_pixels_and_convexity(ref):
    rng = np.random.default_rng(1)
    D = rng.uniform(-5, 20, size=(12, 17)).astype(np.float32)
    for yy in range(12):
        for xx in range(17):
            assert ref.sample(D, xx, yy, bilinear=True) == D[yy, xx]
    for _ in range(200):
        px, py = np.float32(rng.uniform(0, 16)), np.float32(rng.uniform(0, 11))
        x0, y0 = int(np.floor(px)), int(np.floor(py))
        taps = D[y0:min(y0 + 2, 12), x0:min(x0 + 2, 17)]
        v = ref.sample(D, px, py, bilinear=True)
        assert taps.min() - 1e-5 <= v <= taps.max() + 1e-5


def test_bilinear_equals_nearest_on_axis_views(ref):
    sc = scenes.make_c1_like(3, W=160, H=120, n_objects=8)
    ang, rat = [0, 90, 180, 270], [1.0, 1.0, 1.0, 1.0]
    L = [40] * 4
    M0, _, n0 = ref.detect(sc.D, ang, rat, L)
    M1, _, n1 = ref.detect(sc.D, ang, rat, L, bilinear=True)
    np.testing.assert_array_equal(M0, M1)
    np.testing.assert_array_equal(n0, n1)


def test_bilinear_monotone_in_thresholds(ref):
    sc = scenes.make_c1_like(4, W=128, H=96, n_objects=6)
    prev = None
    for beta in (2.0, 1.0, 0.5):
        M, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len, disp_thr=beta, bilinear=True)
        if prev is not None:
            assert np.all(M >= prev)
        prev = M


def test_bilinear_differs_on_diagonals(ref):
    """On diagonal views the sample positions are not pixel centres, so the
    variant changes some decisions (it is a different method, not a no-op)."""
    sc = scenes.make_c1_like(5, W=160, H=120, n_objects=8)
    M0, _, _ = ref.detect(sc.D, [45, 135], [1.4142135] * 2, [60, 60])
    M1, _, _ = ref.detect(sc.D, [45, 135], [1.4142135] * 2, [60, 60], bilinear=True)
    assert (M0 != M1).sum() > 0


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,seed", [("c0", 11), ("c1", 1001), ("c1", 1005)])
def test_gpu_bilinear_parity(ref, cfg, seed):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        sc = scenes.make_scene(cfg, seed)
        D = torch.from_numpy(sc.D).cuda()
        prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len,
                          flags=occl.FLAG_SYNC | occl.FLAG_BILINEAR)
        M = ctx.occl_detect(D, sc.angles, sc.ratios, prm).cpu().numpy()
        Mr, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len, bilinear=True, **sc.params)
        assert int((M != Mr).sum()) == 0
    finally:
        ctx.occl_release()


@pytest.mark.gpu
def test_gpu_bilinear_odd_angles_long_scanlines_and_batched(ref):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        sc = scenes.make_scene("c2", 2001)
        D = np.ascontiguousarray(sc.D[300:620, 900:1400])
        Ls = np.minimum(sc.scan_len, 300)
        prm = occl.params(**sc.params, scan_len_per_view=Ls, flags=occl.FLAG_SYNC | occl.FLAG_BILINEAR)
        M = ctx.occl_detect(torch.from_numpy(D).cuda(), sc.angles, sc.ratios, prm).cpu().numpy()
        Mr, _, _ = ref.detect(D, sc.angles, sc.ratios, Ls, bilinear=True, **sc.params)
        assert int((M != Mr).sum()) == 0
        # batched path with the variant: every frame as the single-frame call
        frames = [scenes.make_c1_like(40 + k, W=w, H=h) for k, (w, h) in enumerate([(320, 240), (200, 150)])]
        Ds = [torch.from_numpy(f.D).cuda() for f in frames]
        Ms = [torch.empty((8, f.H, f.W), dtype=torch.uint8, device="cuda") for f in frames]
        prm = occl.params(**frames[0].params, flags=occl.FLAG_BILINEAR)
        ctx.occl_detect_batched([(d, m, f.scan_len) for d, m, f in zip(Ds, Ms, frames)],
                                frames[0].angles, frames[0].ratios, prm)
        torch.cuda.synchronize()
        for m, f in zip(Ms, frames):
            Mr, _, _ = ref.detect(f.D, f.angles, f.ratios, f.scan_len, bilinear=True, **f.params)
            assert int((m.cpu().numpy() != Mr).sum()) == 0
    finally:
        ctx.occl_release()
