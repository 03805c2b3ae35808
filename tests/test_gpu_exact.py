"""GPU parity of the exact path: the HIP library (through its C ABI) against
the CPU oracle, element by element, on seeded synthetic scenes.

Bar: bit-exact masks.  The oracle's `tight` map (pixels whose value rests on
a decision within 1e-4 px of its threshold, at most 0.01 % of the pixels,
checked here on every map passed in) would exempt mismatches; every test
here additionally reports the mismatch count, which has been zero
throughout.
"""
import numpy as np
import pytest

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


def run_gpu(gctx, torch, D, angles, ratios, L, counts=False, **kw):
    from paper_2408_14050_amd import occl
    Dt = torch.from_numpy(np.ascontiguousarray(D, dtype=np.float32)).cuda()
    prm = occl.params(scan_len_per_view=np.broadcast_to(np.atleast_1d(L), np.atleast_1d(angles).shape),
                      flags=occl.FLAG_SYNC, **kw)
    M = gctx.occl_detect(Dt, angles, ratios, prm).cpu().numpy()
    nc = gctx.occl_last_candidate_counts(len(np.atleast_1d(angles))) if counts else None
    return M, nc


def assert_parity(M_gpu, M_ref, tight=None, what=""):
    diff = M_gpu != M_ref
    n_bad = int(diff.sum())
    if tight is not None:
        assert int(tight.sum()) <= 1e-4 * M_ref.size, f"{what}: tight map above 0.01 %"
    if n_bad and tight is not None:
        assert not (diff & (tight == 0)).any(), f"{what}: {n_bad} mismatches outside the tight map"
        assert n_bad <= 1e-4 * M_ref.size, f"{what}: {n_bad} mismatches > 0.01 %"
    else:
        assert n_bad == 0, f"{what}: {n_bad} mismatching mask bytes"


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(100))
def test_c0_parity(gctx, torch, ref, seed):
    sc = scenes.make_scene("c0", seed)
    M_ref, T, nc_ref = ref.detect_scene(sc, want_tight=True)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, T, f"c0 seed {seed}")


@pytest.mark.parametrize("seed", range(1000, 1016))
def test_c1_parity(gctx, torch, ref, seed):
    sc = scenes.make_scene("c1", seed)
    M_ref, T, nc_ref = ref.detect_scene(sc, want_tight=True)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, T, f"c1 seed {seed}")
    assert M_ref.sum() > 0


@pytest.mark.parametrize("seed", [2000, 2001])
def test_c2_crops_parity(gctx, torch, ref, seed):
    """Crops of the 4x4-array workload (15 views, L up to 366) checked in full."""
    sc = scenes.make_scene("c2", seed)
    rng = np.random.default_rng(seed)
    for _ in range(2):
        y0 = int(rng.integers(0, sc.H - 400))
        x0 = int(rng.integers(0, sc.W - 520))
        D = np.ascontiguousarray(sc.D[y0:y0 + 400, x0:x0 + 520])
        M_ref, T, nc_ref = ref.detect(D, sc.angles, sc.ratios, sc.scan_len, want_tight=True, **sc.params)
        M, nc = run_gpu(gctx, torch, D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
        np.testing.assert_array_equal(nc, nc_ref)
        assert_parity(M, M_ref, T, f"c2 crop {seed} ({y0},{x0})")


def test_c2_full_frame(gctx, torch, ref):
    """Full 3840x2160 x 15 views (L up to 366) against the whole-frame oracle."""
    sc = scenes.make_scene("c2", 2000)
    print(f"c2 seed 2000 {sc.W}x{sc.H} x{sc.n_views} views", flush=True)
    M_ref, T, nc_ref = ref.detect_scene(sc, want_tight=True)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, T, "c2 full frame")
    assert M_ref.sum() > 0


def test_c4_frame_parity(gctx, torch, ref):
    sc = scenes.make_scene("c4", 4100)
    M_ref, T, nc_ref = ref.detect_scene(sc, want_tight=True)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, T, "c4 1920x1080")


def test_batched_equals_per_frame_and_oracle(gctx, torch, ref):
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3000, n_frames=6, sizes=((640, 480), (320, 200), (1280, 960)))
    sc0 = frames[0]
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.full((f.n_views, f.H, f.W), 9, dtype=torch.uint8, device="cuda") for f in frames]
    prm = occl.params(**sc0.params, flags=occl.FLAG_SYNC)
    gctx.occl_detect_batched([(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)],
                             sc0.angles, sc0.ratios, prm)
    for f, D, M in zip(frames, Ds, Ms):
        M_ref, _, _ = ref.detect_scene(f)
        assert_parity(M.cpu().numpy(), M_ref, None, f"batched {f.W}x{f.H}")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
EDGE_SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (16, 64), (17, 65), (31, 257), (65, 130),
               (100, 255), (192, 258), (33, 1023)]


@pytest.mark.parametrize("shape", EDGE_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_ragged_shapes(gctx, torch, ref, shape):
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    D = rng.choice(np.float32([0, 1.5, 3, 6.25, 11]), size=(H, W)).astype(np.float32)
    D += rng.normal(0, 0.2, size=(H, W)).astype(np.float32)
    angles = [0, 45, 90, 135, 180, 225, 270, 315, 17.5, 200.25]
    ratios = np.float32([1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 2.5, 0.7])
    L = [9, 13, 9, 13, 9, 13, 9, 13, 31, 7]
    M_ref, _, nc_ref = ref.detect(D, angles, ratios, L)
    M, nc = run_gpu(gctx, torch, D, angles, ratios, L, counts=True)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, None, f"shape {shape}")


def test_misaligned_pointer(gctx, torch, ref):
    """D starting 1 float past an aligned address takes the scalar path."""
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c0", 3)
    H, W = sc.D.shape
    flat = torch.zeros(H * W + 1, dtype=torch.float32, device="cuda")
    flat[1:] = torch.from_numpy(sc.D.ravel()).cuda()
    D = flat[1:].view(H, W)
    assert D.data_ptr() % 16 != 0
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
    M = gctx.occl_detect(D, sc.angles, sc.ratios, prm).cpu().numpy()
    M_ref, _, _ = ref.detect_scene(sc)
    assert_parity(M, M_ref, None, "misaligned")


@pytest.mark.parametrize("L", [1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 511, 512, 1023])
def test_scan_length_classes(gctx, torch, ref, L):
    sc = scenes.make_c1_like(77, W=200, H=150, n_objects=6)
    M_ref, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, L)
    M, _ = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, L)
    assert_parity(M, M_ref, None, f"L={L}")


def test_long_scanline_forms_many_runs(gctx, torch, ref):
    """The long-scanline classes' three-quarter forms (K = 3 for 129..192
    samples, K = 6 for 257..384) and the full forms at their boundaries, on
    a block pattern that cuts every scanline into many monotone runs
    (a disparity step of 20 every 5 to 7 pixels: about n / 6 runs), so the
    padded bitonic route of the ordering runs as well as the co-rank merge."""
    H, W = 420, 440
    y, x = np.mgrid[0:H, 0:W]
    D = (20.0 * (((x // 5) + (y // 7)) % 2) + 0.01 * x + 0.02 * y).astype(np.float32)
    angles = np.array([0.0, 90.0, 45.0, 180.0, 27.5, 0.0, 270.0, 135.0, 0.0])
    ratios = np.ones(len(angles), np.float32)
    L = np.array([128, 150, 191, 192, 256, 300, 383, 384, 511])  # n = L + 1 (even L) or L
    M_ref, T, nc_ref = ref.detect(D, angles, ratios, L, want_tight=True)
    M, nc = run_gpu(gctx, torch, D, angles, ratios, L, counts=True)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, T, "block pattern, long scanlines")
    assert M_ref.sum() > 0


@pytest.mark.parametrize("N", [1, 2, 3, 4, 7, 64])
def test_neighbour_counts(gctx, torch, ref, N):
    sc = scenes.make_c1_like(78, W=256, H=160, n_objects=8)
    M_ref, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len, neighbours=N, dist_thr=2.0)
    M, _ = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, neighbours=N, dist_thr=2.0)
    assert_parity(M, M_ref, None, f"N={N}")


def test_many_views_arbitrary_geometry(gctx, torch, ref):
    rng = np.random.default_rng(11)
    sc = scenes.make_c1_like(79, W=320, H=240, n_objects=10)
    V = 64
    angles = rng.uniform(-400, 400, V)
    ratios = rng.uniform(0.3, 3.0, V).astype(np.float32)
    L = rng.integers(1, 140, V)
    M_ref, _, nc_ref = ref.detect(sc.D, angles, ratios, L, edge_thr=0.8, disp_thr=0.3, dist_thr=1.5)
    M, nc = run_gpu(gctx, torch, sc.D, angles, ratios, L, counts=True, edge_thr=0.8, disp_thr=0.3,
                    dist_thr=1.5)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, None, "64 views")


def test_constant_and_negative_maps(gctx, torch, ref):
    D = np.full((50, 70), -3.5, np.float32)
    M, nc = run_gpu(gctx, torch, D, [0, 45, 180], np.float32([1, 1.4, 2]), 20, counts=True)
    assert M.sum() == 0 and (nc == 0).all()
    D[10:30, 20:40] = 4.0
    M_ref, _, _ = ref.detect(D, [0, 45, 180], np.float32([1, 1.4, 2]), 20)
    M, _ = run_gpu(gctx, torch, D, [0, 45, 180], np.float32([1, 1.4, 2]), 20)
    assert_parity(M, M_ref, None, "negative")
    assert M.sum() > 0


def test_deterministic(gctx, torch):
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c1", 1005)
    D = torch.from_numpy(sc.D).cuda()
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
    first = gctx.occl_detect(D, sc.angles, sc.ratios, prm).clone()
    for _ in range(9):
        assert torch.equal(gctx.occl_detect(D, sc.angles, sc.ratios, prm), first)


def test_empty_inputs(gctx, torch):
    from paper_2408_14050_amd import occl
    prm = occl.params(scan_len=10, flags=occl.FLAG_SYNC)
    D = torch.zeros((0, 5), dtype=torch.float32, device="cuda")
    M = gctx.occl_detect(D, [0.0], [1.0], prm)
    assert M.shape == (1, 0, 5)
    D = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    M = gctx.occl_detect(D, np.zeros(0), np.zeros(0, np.float32), prm)
    assert M.shape == (0, 4, 5)
    gctx.occl_detect_batched([], [0.0], [1.0], prm)


# ---------------------------------------------------------------------------
# auto scan length, edges, confusion counts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, -1])
def test_auto_scan_length(gctx, torch, ref, mode):
    from paper_2408_14050_amd import occl
    sc = scenes.make_c1_like(80, W=256, H=192, n_objects=8)
    L_ref = ref.scan_len(sc.D, sc.ratios, mode=0 if mode == 0 else 1)
    if mode == 0:
        np.testing.assert_array_equal(L_ref, sc.scan_len)
    M_ref, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, L_ref)
    prm = occl.params(scan_len=mode, flags=occl.FLAG_SYNC)
    M = gctx.occl_detect(torch.from_numpy(sc.D).cuda(), sc.angles, sc.ratios, prm).cpu().numpy()
    assert_parity(M, M_ref, None, f"auto L mode {mode}")


def test_edges_exact_magnitude(gctx, torch, ref):
    sc = scenes.make_scene("c1", 1001)
    D = torch.from_numpy(sc.D).cuda()
    E = torch.empty_like(D)
    A = torch.empty_like(D)
    gctx.occl_edges(D, E, A)
    gctx.occl_sync()
    _, _, E_ref, A_ref = ref.edges(sc.D)
    np.testing.assert_array_equal(E.cpu().numpy(), E_ref)      # correctly rounded sqrt both sides
    np.testing.assert_allclose(A.cpu().numpy(), A_ref, rtol=0, atol=2e-6)


def test_confusion_counts(gctx, torch, ref):
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2, 1_000_003).astype(np.uint8)
    b = rng.integers(0, 2, 1_000_003).astype(np.uint8)
    got = gctx.occl_confusion(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    assert got == ref.confusion(a, b)


# ---------------------------------------------------------------------------
# C-ABI contract: errors are reported before anything is enqueued
# ---------------------------------------------------------------------------
def test_invalid_arguments_have_no_side_effects(gctx, torch):
    import ctypes as C
    from paper_2408_14050_amd import occl
    D = torch.rand((32, 40), device="cuda") * 10
    M = torch.full((2, 32, 40), 7, dtype=torch.uint8, device="cuda")
    good = dict(scan_len=10, flags=occl.FLAG_SYNC)
    cases = [
        (dict(good), [0.0, 1.0], [1.0, 0.0]),                  # ratio 0
        (dict(good), [0.0, float("nan")], [1.0, 1.0]),         # NaN angle
        (dict(good, neighbours=0), [0.0, 90.0], [1.0, 1.0]),
        (dict(good, edge_thr=float("inf")), [0.0, 90.0], [1.0, 1.0]),
        (dict(good, scan_len=2000), [0.0, 90.0], [1.0, 1.0]),  # unsupported L
        (dict(good, scan_len=-2), [0.0, 90.0], [1.0, 1.0]),
    ]
    for kw, a, r in cases:
        with pytest.raises(occl.OcclError):
            gctx.occl_detect(D, a, np.float32(r), occl.params(**kw), M=M)
    prm = occl.params(**good)
    prm.struct_size = 4
    with pytest.raises(occl.OcclError):
        gctx.occl_detect(D, [0.0, 90.0], np.float32([1, 1]), prm, M=M)
    st = occl.lib().occl_detect(gctx.h, None, 32, 40, 2,
                                np.zeros(2).ctypes.data_as(C.POINTER(C.c_double)),
                                np.ones(2, np.float32).ctypes.data_as(C.POINTER(C.c_float)),
                                C.byref(occl.params(**good)), C.c_void_p(M.data_ptr()))
    assert st == -1
    # frames wider or taller than 65535 (packed candidate coordinates) are
    # refused before anything is enqueued; the sizes are checked first, so
    # small buffers suffice
    for H, W in ((2, 65536), (65536, 2)):
        st = occl.lib().occl_detect(gctx.h, C.c_void_p(D.data_ptr()), H, W, 2,
                                    np.zeros(2).ctypes.data_as(C.POINTER(C.c_double)),
                                    np.ones(2, np.float32).ctypes.data_as(C.POINTER(C.c_float)),
                                    C.byref(occl.params(**good)), C.c_void_p(M.data_ptr()))
        assert st == -4, (H, W, st)
    torch.cuda.synchronize()
    assert (M == 7).all()
    with pytest.raises(occl.OcclError):
        gctx.occl_last_candidate_counts(5)


def test_validate_input_rejects_nan(gctx, torch):
    from paper_2408_14050_amd import occl
    D = torch.ones((16, 16), device="cuda")
    D[3, 4] = float("nan")
    M = torch.full((1, 16, 16), 7, dtype=torch.uint8, device="cuda")
    with pytest.raises(occl.OcclError):
        gctx.occl_detect(D, [0.0], [1.0], occl.params(scan_len=5, flags=occl.FLAG_VALIDATE_INPUT), M=M)
    torch.cuda.synchronize()
    assert (M == 7).all()


def test_second_context_on_its_own_stream(torch, ref):
    from paper_2408_14050_amd import occl
    s = torch.cuda.Stream()
    ctx2 = occl.Context(0, stream=s)
    sc = scenes.make_scene("c0", 42)
    with torch.cuda.stream(s):
        run = occl.detect_scene(ctx2, sc)
    ctx2.occl_sync()
    M_ref, _, _ = ref.detect_scene(sc)
    assert_parity(run.M.cpu().numpy(), M_ref, None, "second context")
    ctx2.occl_release()


@pytest.mark.parametrize("seed", range(12))
def test_integer_maps_with_ties(gctx, torch, ref, seed):
    """Integer disparities and axis / diagonal / arbitrary baselines produce
    many exactly equal W across runs: the (W, g) tie rule is exercised."""
    rng = np.random.default_rng(500 + seed)
    H, W = int(rng.integers(20, 90)), int(rng.integers(20, 120))
    D = np.full((H, W), float(rng.integers(0, 3)), np.float32)
    for _ in range(int(rng.integers(2, 9))):
        h, w = int(rng.integers(2, H)), int(rng.integers(2, W))
        y0, x0 = int(rng.integers(-2, H - 1)), int(rng.integers(-2, W - 1))
        D[max(0, y0):max(0, y0 + h), max(0, x0):max(0, x0 + w)] = float(rng.integers(0, 24))
    if seed % 3 == 0:
        D += rng.integers(0, 2, size=(H, W)).astype(np.float32)   # integer noise: many runs
    angles = [0, 90, 180, 270, 45, 135, 225, 315, 30, 60]
    ratios = np.float32([1, 1, 2, 1, 1.4142135, 1, 2, 1.4142135, 1, 0.5])
    L = [30, 31, 60, 17, 45, 33, 70, 45, 25, 9]
    for N, zeta in ((1, 1.0), (1, 2.0), (3, 2.0)):
        M_ref, _, nc_ref = ref.detect(D, angles, ratios, L, neighbours=N, dist_thr=zeta)
        M, nc = run_gpu(gctx, torch, D, angles, ratios, L, counts=True, neighbours=N, dist_thr=zeta)
        np.testing.assert_array_equal(nc, nc_ref)
        assert_parity(M, M_ref, None, f"integer seed {seed} N={N} zeta={zeta}")


def test_prepared_call_and_frames_in_flight(torch, ref):
    """The prepared per-frame call, and frames in flight on three contexts
    with their own streams (the throughput launch configuration), give the
    oracle's masks for every frame, also with frames of different maps
    interleaved across the streams."""
    from paper_2408_14050_amd import occl
    scs = [scenes.make_scene("c0", 60 + i) for i in range(6)]
    sc0 = scs[0]
    streams = [torch.cuda.Stream() for _ in range(3)]
    ctxs = [occl.Context(0, stream=s) for s in streams]
    prm = occl.params(scan_len_per_view=sc0.scan_len, **sc0.params)
    dets = [c.occl_detect_prepared(sc0.angles, sc0.ratios, prm) for c in ctxs]
    Ds = [torch.from_numpy(np.ascontiguousarray(s.D)).cuda() for s in scs]
    torch.cuda.synchronize()
    Ms = [torch.empty((len(sc0.angles),) + s.D.shape, dtype=torch.uint8, device="cuda") for s in scs]
    for rep in range(3):
        for i in range(len(scs)):
            dets[i % 3](Ds[i], Ms[i])
    for c in ctxs:
        c.occl_sync()
    for s, M in zip(scs, Ms):
        M_ref, _, _ = ref.detect(s.D, sc0.angles, sc0.ratios, sc0.scan_len, **sc0.params)
        assert_parity(M.cpu().numpy(), M_ref, None, "frames in flight")
    for c in ctxs:
        c.occl_release()


def test_time_scanlines_leaves_masks_unchanged(gctx, torch, ref):
    """The measurement entry point re-runs the last frame's scanline pass: the
    masks stay those of the oracle, and without an exact-path frame the call
    is refused."""
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    with pytest.raises(occl.OcclError):
        ctx.occl_time_scanlines(3)
    sc = scenes.make_scene("c0", 7)
    D = torch.from_numpy(np.ascontiguousarray(sc.D)).cuda()
    prm = occl.params(scan_len_per_view=sc.scan_len, **sc.params)
    M = ctx.occl_detect(D, sc.angles, sc.ratios, prm)
    ms = ctx.occl_time_scanlines(20)
    assert 0.0 < ms < 100.0
    M_ref, _, _ = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len, **sc.params)
    assert_parity(M.cpu().numpy(), M_ref, None, "after re-timed scanline passes")
    ctx.occl_release()


@pytest.mark.parametrize("shape", [(24, 65535), (65535, 24)], ids=["24x65535", "65535x24"])
def test_maximum_frame_extent(gctx, torch, ref, shape):
    """The largest accepted width and height (candidate coordinates packed
    into 16 bits each reach 65534): bit-exact with the oracle."""
    H, W = shape
    sc = scenes.extent_scene(H, W, 70000 + H)
    M_ref, _, nc_ref = ref.detect(sc.D, sc.angles, sc.ratios, sc.scan_len)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True)
    np.testing.assert_array_equal(nc, nc_ref)
    assert nc.sum() > 0
    assert_parity(M, M_ref, None, f"{H}x{W}")


@pytest.mark.parametrize("seed", [4242, 4243])
def test_large_frame_split_over_dies(gctx, torch, ref, seed):
    """A 2048 x 2048 frame (D of 16 MiB, where the scanline pass splits each
    view's items over the dies), c1 statistics, 8 views: the whole mask equals
    the oracle's."""
    sc = scenes.make_c1_like(seed, W=2048, H=2048)
    assert sc.D.nbytes >= 16 << 20
    M_ref, _, nc_ref = ref.detect_scene(sc)
    M, nc = run_gpu(gctx, torch, sc.D, sc.angles, sc.ratios, sc.scan_len, counts=True, **sc.params)
    np.testing.assert_array_equal(nc, nc_ref)
    assert_parity(M, M_ref, None, f"2048x2048 seed {seed}")
