"""Batched path (one captured graph per batch signature) and the launch-shape
autotuner, on the GPU through the C ABI, against the CPU oracle."""
import os

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


def _ref(ref, sc):
    return ref.detect_scene(sc)[0]


def _run_batch(gctx, torch, frames, fill=9):
    from paper_2408_14050_amd import occl
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.full((f.n_views, f.H, f.W), fill, dtype=torch.uint8, device="cuda") for f in frames]
    prm = occl.params(**frames[0].params, flags=occl.FLAG_SYNC)
    gctx.occl_detect_batched([(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)],
                             frames[0].angles, frames[0].ratios, prm)
    return Ds, Ms


def test_mixed_sizes_and_ragged_frames(gctx, torch, ref):
    sizes = ((640, 480), (37, 19), (1280, 960), (258, 131), (1920, 1080), (5, 3))
    frames = [scenes.make_c1_like(7000 + i, W=w, H=h) for i, (w, h) in enumerate(sizes)]
    _, Ms = _run_batch(gctx, torch, frames)
    for f, M in zip(frames, Ms):
        assert np.array_equal(M.cpu().numpy(), _ref(ref, f)), f"{f.W}x{f.H}"


def test_mixed_scan_classes(gctx, torch, ref):
    """Frames whose scan lengths fall in different register classes (K up to 8)."""
    frames = []
    for i, L in enumerate((40, 150, 300, 70)):
        f = scenes.make_c1_like(7100 + i, W=320, H=240, n_objects=8)
        f.scan_len = np.full(f.n_views, L, np.int32)
        frames.append(f)
    _, Ms = _run_batch(gctx, torch, frames)
    for f, M in zip(frames, Ms):
        assert np.array_equal(M.cpu().numpy(), _ref(ref, f)), f"L={f.scan_len[0]}"


def test_graph_replays_with_eager_work_between(gctx, torch, ref):
    """The same batch signature replays one graph; every replay (with new
    frame contents, and single-frame eager calls in between) is exact."""
    from paper_2408_14050_amd import occl
    sizes = ((320, 240), (640, 480), (320, 240))
    frames = [scenes.make_c1_like(7200 + i, W=w, H=h) for i, (w, h) in enumerate(sizes)]
    for f in frames:
        f.scan_len = np.full(f.n_views, 50, np.int32)   # fixed shapes: one graph
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.empty((f.n_views, f.H, f.W), dtype=torch.uint8, device="cuda") for f in frames]
    prm = occl.params(**frames[0].params, flags=occl.FLAG_SYNC)
    eager = scenes.make_scene("c0", 5)
    for rep in range(4):
        # new contents in the same buffers
        for i, f in enumerate(frames):
            g = scenes.make_c1_like(7300 + 10 * rep + i, W=f.W, H=f.H)
            f.D = g.D
            Ds[i].copy_(torch.from_numpy(g.D))
        gctx.occl_detect_batched([(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)],
                                 frames[0].angles, frames[0].ratios, prm)
        for f, M in zip(frames, Ms):
            assert np.array_equal(M.cpu().numpy(), _ref(ref, f)), f"replay {rep} {f.W}x{f.H}"
        run = occl.detect_scene(gctx, eager)
        assert np.array_equal(run.M.cpu().numpy(), _ref(ref, eager))


def test_more_frames_than_one_launch(gctx, torch, ref):
    rng = np.random.default_rng(3)
    frames = []
    for i in range(1030):
        f = scenes.make_c1_like(int(rng.integers(1 << 30)), W=int(rng.integers(4, 24)),
                                H=int(rng.integers(4, 24)), n_objects=2)
        f.scan_len = np.full(f.n_views, 9, np.int32)
        frames.append(f)
    _, Ms = _run_batch(gctx, torch, frames)
    for k in (0, 1, 500, 1023, 1024, 1029):
        assert np.array_equal(Ms[k].cpu().numpy(), _ref(ref, frames[k])), k


@pytest.mark.parametrize("edge_rows,bpc", [(1, 2), (2, 16), (4, 8), (8, 4), (16, 1)])
def test_every_launch_shape_gives_the_same_mask(gctx, torch, ref, tmp_path, edge_rows, bpc):
    """A tune file forcing each shape for the frame's bucket: same masks."""
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c1", 1007)
    D = torch.from_numpy(sc.D).cuda()
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
    M = torch.empty((8, sc.H, sc.W), dtype=torch.uint8, device="cuda")
    ctx = occl.Context(0)
    ctx.occl_autotune(D, sc.angles, sc.ratios, prm, M, reps=1)   # learn the bucket key
    path = tmp_path / "t.txt"
    ctx.occl_tune_save(str(path))
    lines = [l for l in path.read_text().splitlines() if not l.startswith("#")]
    key = lines[0].split()[0]
    path.write_text(f"{key} {edge_rows} {bpc}\n")
    ctx.occl_tune_load(str(path))
    M2 = ctx.occl_detect(D, sc.angles, sc.ratios, prm)
    assert np.array_equal(M2.cpu().numpy(), _ref(ref, sc))
    ctx.occl_release()


def test_autotune_and_tune_file(gctx, torch, ref, tmp_path):
    from paper_2408_14050_amd import occl
    sc = scenes.make_scene("c1", 1008)
    D = torch.from_numpy(sc.D).cuda()
    M = torch.empty((8, sc.H, sc.W), dtype=torch.uint8, device="cuda")
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
    best = gctx.occl_autotune(D, sc.angles, sc.ratios, prm, M, reps=3)
    assert best["edge_rows"] in (1, 2, 4, 8, 16) and 1 <= best["scan_blocks_per_cu"] <= 64
    assert best["ms"] > 0
    assert np.array_equal(M.cpu().numpy(), _ref(ref, sc))          # trials leave the right mask
    p = tmp_path / "tune.txt"
    gctx.occl_tune_save(str(p))
    gctx.occl_tune_load(str(p))
    bad = tmp_path / "bad.txt"
    bad.write_text("12 3 8\n")                                       # 3 is not a power of two
    with pytest.raises(occl.OcclError):
        gctx.occl_tune_load(str(bad))
    frames = scenes.make_batch(seed=3100, n_frames=5, sizes=((640, 480), (320, 240)))
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.empty((f.n_views, f.H, f.W), dtype=torch.uint8, device="cuda") for f in frames]
    bb = gctx.occl_autotune_batched([(D_, M_, f.scan_len) for D_, M_, f in zip(Ds, Ms, frames)],
                                    frames[0].angles, frames[0].ratios, occl.params(**frames[0].params),
                                    reps=2)
    assert bb["ms"] > 0
    for f, M_ in zip(frames, Ms):
        assert np.array_equal(M_.cpu().numpy(), _ref(ref, f))


def test_extreme_extents_in_one_batch(gctx, torch, ref):
    """Frames 65535 wide and 65535 tall batched with a small one (same views):
    every mask equals the oracle's."""
    frames = [scenes.extent_scene(24, 65535, 70024), scenes.extent_scene(65535, 24, 70035),
              scenes.extent_scene(40, 300, 70040)]
    _, Ms = _run_batch(gctx, torch, frames)
    for f, M in zip(frames, Ms):
        np.testing.assert_array_equal(M.cpu().numpy(), _ref(ref, f), err_msg=f.name)



@pytest.mark.parametrize("sizes", [
    ((640, 480),),                                    # one frame: one branch
    ((320, 240), (640, 480)),                         # two frames: one per branch
    ((1920, 1080), (64, 48), (32, 24), (16, 12)),     # the first frame holds most pixels
    ((16, 12), (32, 24), (64, 48), (1920, 1080)),     # the last frame holds most pixels
])
def test_branch_split_edge_cases(gctx, torch, ref, sizes):
    """The batch is split into graph branches of about equal pixel counts;
    every branch keeps at least one frame whatever the size mix."""
    frames = [scenes.make_c1_like(7400 + i, W=w, H=h) for i, (w, h) in enumerate(sizes)]
    _, Ms = _run_batch(gctx, torch, frames)
    for f, M in zip(frames, Ms):
        assert np.array_equal(M.cpu().numpy(), _ref(ref, f)), f"{f.W}x{f.H}"


def _oracle_masks(ref, frames, threads=16):
    """The oracle on every frame, on a host thread pool (ctypes releases the
    GIL; the oracle itself stays single-threaded per call)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda f: ref.detect_scene(f, want_tight=True), frames))


def test_c3_benched_shape(gctx, torch, ref):
    """The batched workload exactly as the benchmark times it: 64 frames from
    make_batch(seed 3000) (sizes 640x480 .. 2048x1536), 8 views each, launch
    shape from the batched autotuner, the graph's branches side by side;
    every frame and view against the oracle (bit-exact; tight map <= 0.01 %)."""
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3000, n_frames=64)
    print(f"c3: {len(frames)} frames, {sum(f.pixel_views for f in frames)} pixel-views", flush=True)
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.full((f.n_views, f.H, f.W), 9, dtype=torch.uint8, device="cuda") for f in frames]
    batch = [(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)]
    prm = occl.params(**frames[0].params)
    shape = gctx.occl_autotune_batched(batch, frames[0].angles, frames[0].ratios, prm, reps=2)
    for M in Ms:
        M.fill_(9)
    gctx.occl_detect_batched(batch, frames[0].angles, frames[0].ratios, prm)
    torch.cuda.synchronize()
    refs = _oracle_masks(ref, frames)
    bad = 0
    for i, (f, M, (M_ref, T, _)) in enumerate(zip(frames, Ms, refs)):
        assert int(T.sum()) <= 1e-4 * T.size, f"frame {i}: tight map above 0.01 %"
        diff = M.cpu().numpy() != M_ref
        assert not (diff & (T == 0)).any(), f"frame {i} {f.W}x{f.H}: {int(diff.sum())} mismatches ({shape})"
        bad += int(diff.sum())
    assert bad <= 1e-4 * sum(f.pixel_views for f in frames)
    assert {(f.W, f.H) for f in frames} == {(640, 480), (1280, 960), (1920, 1080), (2048, 1536)}
