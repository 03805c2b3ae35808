"""GPU parity of the candidate-thinning variant (OCCL_FLAG_THIN: followers on
a candidate's scanline are skipped, run heads scan a window extended over the
run; the thinner candidate list of the paper's summary, Sec. 6) against the
oracle's variant, element by element.  Bar: bit-exact masks."""
import numpy as np
import pytest

from paper_2408_14050_amd import scenes
from tests.test_gpu_exact import assert_parity, gctx, torch  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu

UNSUPPORTED = -4  # OCCL_ERR_UNSUPPORTED


def _thin_gpu(gctx, torch, D, angles, ratios, L, flags=0, **kw):
    """The thinned masks and Eq. (2) candidate counts of the C-ABI call."""
    from paper_2408_14050_amd import occl
    Dt = torch.from_numpy(np.ascontiguousarray(D, dtype=np.float32)).cuda()
    prm = occl.params(scan_len_per_view=np.broadcast_to(np.atleast_1d(L), np.atleast_1d(angles).shape),
                      flags=occl.FLAG_SYNC | occl.FLAG_THIN | flags, **kw)
    M = gctx.occl_detect(Dt, angles, ratios, prm).cpu().numpy()
    return M, gctx.occl_last_candidate_counts(len(np.atleast_1d(angles)))


@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_thin_c1_parity(gctx, torch, ref, seed):
    """Full 1280x960 frames, 8 views, the configured scan lengths."""
    sc = scenes.make_scene("c1", seed)
    M_ref, _, nc_ref = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len, thin=True)
    M, nc = _thin_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len)
    assert_parity(M, M_ref, what=f"thin c1 seed {seed}")
    np.testing.assert_array_equal(nc, nc_ref)  # Eq. (2)'s candidates are unchanged
    M_exact, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len)
    assert (M_exact != M_ref).any()  # the variant is not the method on these scenes


@pytest.mark.parametrize("shape", [(97, 131), (240, 333), (64, 1000)])
@pytest.mark.parametrize("variant", ["plain", "n3", "bilinear"])
def test_thin_ragged_parity(gctx, torch, ref, shape, variant):
    """Ragged frames, off-octant directions, N = 3 and bilinear V composed
    with thinning."""
    from paper_2408_14050_amd import occl
    H, W = shape
    D = scenes.make_c1_like(H * 7 + W, W=W, H=H, n_objects=10, dmax=24.0).D
    angles = [0, 45, 90, 135, 180, 225, 270, 315, 10, 77, 26.56505117707799, 200]
    ratios = np.float32([1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 1.3, 0.8, 2.236068, 1.1])
    L = [27, 35, 27, 35, 27, 35, 27, 35, 31, 21, 55, 29]
    nb = 3 if variant == "n3" else 1
    bil = variant == "bilinear"
    M_ref, _, nc_ref = ref.detect(D, angles, ratios, L, neighbours=nb, bilinear=bil, thin=True)
    M, nc = _thin_gpu(gctx, torch, D, angles, ratios, L, flags=occl.FLAG_BILINEAR if bil else 0,
                      neighbours=nb)
    assert_parity(M, M_ref, what=f"thin {shape} {variant}")
    np.testing.assert_array_equal(nc, nc_ref)


@pytest.mark.parametrize("L", [1, 3, 43, 63, 64, 129, 683])
def test_thin_longest_runs(gctx, torch, ref, L):
    """Ramps whose every pixel is a candidate: one head per row scans
    3 floor(L/2) + 1 samples (1024 at the largest L) and every other
    candidate is a follower.  L = 43 fills one 64-sample slot exactly; at
    L = 63 the merged window (94) outgrows the first attempt's slot and runs
    again with two; L = 1 decides followers outside its one-sample window."""
    H, W = 6, 700
    x = np.arange(W, dtype=np.float32)
    up = np.broadcast_to(np.float32(1.5) * x, (H, W)).copy()
    down = np.ascontiguousarray(up[:, ::-1])
    for D, angles in ((up, [0, 45]), (down, [180, 135])):
        M_ref, _, _ = ref.detect(D, angles, np.float32([0.4, 0.3]), [L, L], thin=True)
        M, _ = _thin_gpu(gctx, torch, D, angles, np.float32([0.4, 0.3]), [L, L])
        assert_parity(M, M_ref, what=f"ramp L={L} {angles}")
    Dt = np.ascontiguousarray(up.T)  # a vertical ramp, 700 x 6
    M_ref, _, _ = ref.detect(Dt, [90], [0.4], [L], thin=True)
    M, _ = _thin_gpu(gctx, torch, Dt, [90], [0.4], [L])
    assert_parity(M, M_ref, what=f"vertical ramp L={L}")


def test_thin_rejections(gctx, torch):
    """Thinning serves single frames of the exact path: routed tiles, batches
    and L beyond 683 are refused before anything is enqueued."""
    from paper_2408_14050_amd import occl
    D = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    thin = occl.FLAG_SYNC | occl.FLAG_THIN
    with pytest.raises(occl.OcclError) as e:
        gctx.occl_detect(D, [0], [1.0], occl.params(scan_len=5, flags=thin | occl.FLAG_USE_CNN))
    assert e.value.status == UNSUPPORTED
    with pytest.raises(occl.OcclError) as e:
        gctx.occl_detect(D, [0], [1.0], occl.params(scan_len=684, flags=thin))
    assert e.value.status == UNSUPPORTED
    M = torch.empty((1, 32, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(occl.OcclError) as e:
        gctx.occl_detect_batched([(D, M, None)], [0], [1.0], occl.params(scan_len=5, flags=thin))
    assert e.value.status == UNSUPPORTED
    out = gctx.occl_detect(D, [0], [1.0], occl.params(scan_len=683, flags=thin))
    assert int(out.sum().item()) == 0


def test_thin_autotuned_shape(gctx, torch, ref):
    """The single-frame autotuner accepts the flag (its trial launches run the
    thinned path) and the tuned shape gives the same bit-exact masks."""
    from paper_2408_14050_amd import occl
    sc = scenes.make_c1_like(5, W=640, H=480, n_objects=12, dmax=24.0)
    angles, ratios, L = [0, 45, 200, 300], np.float32([1.0, 1.4142135, 1.2, 0.9]), [31, 41, 35, 27]
    D = torch.from_numpy(sc.D).cuda()
    M = torch.empty((4,) + sc.D.shape, dtype=torch.uint8, device="cuda")
    prm = occl.params(scan_len_per_view=L, flags=occl.FLAG_SYNC | occl.FLAG_THIN)
    shape = gctx.occl_autotune(D, angles, ratios, prm, M, reps=3)
    assert shape["edge_rows"] > 0 and shape["scan_blocks_per_cu"] > 0
    M_ref, _, _ = ref.detect(sc.D, angles, ratios, L, thin=True)
    assert_parity(M.cpu().numpy(), M_ref, what="masks left by the autotuner")
    M2, _ = _thin_gpu(gctx, torch, sc.D, angles, ratios, L)
    assert_parity(M2, M_ref, what="tuned shape")


def test_thin_large_frame_split_over_dies(gctx, torch, ref):
    """A frame of >= 16 MB takes the scanline pass's per-die split; the
    thinning decision rides along unchanged."""
    sc = scenes.make_c1_like(7, W=2048, H=2100, n_objects=30, dmax=40.0)
    angles, ratios, L = [0, 135], np.float32([1.0, 1.4142135]), [45, 61]
    M_ref, _, nc_ref = ref.detect(sc.D, angles, ratios, L, thin=True)
    M, nc = _thin_gpu(gctx, torch, sc.D, angles, ratios, L)
    assert_parity(M, M_ref, what="thin 2100x2048")
    np.testing.assert_array_equal(nc, nc_ref)


def test_thin_eq3_scan_length(gctx, torch, ref):
    """Eq. (3)'s L read from D on the device (scan_len = -1): longer windows,
    larger register classes, thinned."""
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c1", 1001)
    Ls = ref.scan_len(sc.D, sc.ratios, -1)
    assert Ls.max() <= 683
    M_ref, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, Ls, thin=True)
    D = torch.from_numpy(sc.D).cuda()
    M = gctx.occl_detect(D, sc.angles, sc.ratios,
                         occl.params(**sc.params, scan_len=-1, flags=occl.FLAG_SYNC | occl.FLAG_THIN))
    assert_parity(M.cpu().numpy(), M_ref, what=f"thin Eq. (3) L {Ls.tolist()}")
