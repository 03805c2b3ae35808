"""The fused form of a batch (mask fill + one persistent pass over tiles,
Eqs. (1)-(6) per tile with the candidates kept in LDS) against the oracle,
bit for bit, and against the two-pass form.  The form is chosen through
the autotuner's bucket of the batch: edge_rows 0 is the fused pass."""
import os
import tempfile

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


def _force(ctx, batch, angles, ratios, prm, edge_rows):
    """Sets the batch's tuning bucket to `edge_rows` (0: fused)."""
    ctx.occl_autotune_batched(batch, angles, ratios, prm, reps=1)
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    ctx.occl_tune_save(path)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    with open(path, "w") as f:
        for k, er, bpc in rows:
            f.write(f"{k} {edge_rows if int(k) & 1 else er} {bpc}\n")
    ctx.occl_tune_load(path)


def _run(ctx, torch, frames, edge_rows, prm=None):
    from paper_2408_14050_amd import occl
    Ds = [torch.from_numpy(np.ascontiguousarray(f.D)).cuda() for f in frames]
    Ms = [torch.full((f.n_views, f.H, f.W), 7, dtype=torch.uint8, device="cuda") for f in frames]
    batch = [(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)]
    prm = prm or occl.params(**frames[0].params)
    _force(ctx, batch, frames[0].angles, frames[0].ratios, prm, edge_rows)
    for M in Ms:
        M.fill_(7)
    ctx.occl_detect_batched(batch, frames[0].angles, frames[0].ratios, prm)
    torch.cuda.synchronize()
    return [M.cpu().numpy() for M in Ms], batch, prm


def _oracle(ref, frames):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(16) as ex:
        return list(ex.map(lambda f: ref.detect_scene(f)[0], frames))


def test_fused_c3_benched_batch(torch, ref):
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3000, n_frames=64)
    print(f"fused c3: {len(frames)} frames", flush=True)
    ctx = occl.Context(0)
    try:
        Mf, batch, prm = _run(ctx, torch, frames, 0)
        st = ctx.occl_time_batched(2)
        assert st["form"] == "fused" and st["fused"] > 0 and st["clear"] > 0
    finally:
        ctx.occl_release()
    for i, (M, R) in enumerate(zip(Mf, _oracle(ref, frames))):
        assert np.array_equal(M, R), f"frame {i}: {int((M != R).sum())} bytes differ"


@pytest.mark.parametrize("seed", [1, 2])
def test_fused_ragged_frames_and_short_scanlines(torch, ref, seed):
    """Frame sizes off every tile and vector boundary, one with a single
    row and one with a single column; L from 1 to 127 (n up to 127)."""
    from paper_2408_14050_amd import occl
    rng = np.random.default_rng(seed)
    sizes = [(333, 77), (257, 17), (1, 300), (300, 1), (640, 481), (31, 5), (1030, 33)]
    frames = [scenes.make_c1_like(int(rng.integers(0, 1 << 30)), W=w, H=h, n_objects=6) for w, h in sizes]
    Ls = [1, 2, 33, 64, 65, 126, 127, 90]
    for f in frames:
        f.scan_len = np.asarray(rng.choice(Ls, size=8), np.int32)
    print(f"fused ragged seed {seed}", flush=True)
    ctx = occl.Context(0)
    try:
        Mf, _, _ = _run(ctx, torch, frames, 0)
        Mt, _, _ = _run(ctx, torch, frames, 4)
    finally:
        ctx.occl_release()
    for i, (M, T, R) in enumerate(zip(Mf, Mt, _oracle(ref, frames))):
        assert np.array_equal(M, R), f"frame {i} {frames[i].W}x{frames[i].H}: {int((M != R).sum())} differ"
        assert np.array_equal(T, R)


@pytest.mark.parametrize("H,W", [(64, 600), (67, 601)])
def test_fused_dense_candidates_overflow_rounds(torch, ref, H, W):
    """A ramp whose every pixel is strong: a tile's strong pixels exceed
    what one queue holds for all views, so they go in rounds, and the
    rounds after the first take the differences from D again (at the
    frame's right and bottom borders too, and with the scalar loads of a
    width that is not a multiple of 4)."""
    from paper_2408_14050_amd import occl
    print(f"fused dense {W}x{H}", flush=True)
    yy, xx = np.mgrid[0:H, 0:W]
    D = (1.5 * xx + 1.25 * yy + 0.01 * ((xx * 7 + yy * 13) % 11)).astype(np.float32) % 40.0
    angles, ratios = scenes.views_3x3()
    sc = scenes.Scene("ramp", 0, np.ascontiguousarray(D), angles, ratios, np.array([50, 70] * 4, np.int32))
    ctx = occl.Context(0)
    try:
        Mf, _, _ = _run(ctx, torch, [sc, sc], 0)
    finally:
        ctx.occl_release()
    R = ref.detect_scene(sc)[0]
    for M in Mf:
        assert np.array_equal(M, R)


def test_fused_graph_replays_with_eager_work_between(torch, ref):
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3005, n_frames=6, sizes=((640, 480), (1280, 960)))
    ctx = occl.Context(0)
    try:
        Mf, batch, prm = _run(ctx, torch, frames, 0)
        R = _oracle(ref, frames)
        for rep in range(4):
            for _, M, _ in batch:
                M.fill_(5)
            x = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            ctx.occl_detect_batched(batch, frames[0].angles, frames[0].ratios, prm)
            torch.cuda.synchronize()
            assert float(x) == float(x)
            for (_, M, _), r in zip(batch, R):
                assert np.array_equal(M.cpu().numpy(), r), f"replay {rep}"
    finally:
        ctx.occl_release()


def test_fused_not_taken_when_the_batch_does_not_allow_it(torch, ref):
    """N = 3 (more than one neighbour per side) and scanlines of more than
    128 samples keep the two-pass form even with edge_rows 0 requested."""
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3007, n_frames=3, sizes=((640, 480),))
    p3 = occl.params(**dict(frames[0].params, neighbours=3))
    ctx = occl.Context(0)
    try:
        Mf, _, _ = _run(ctx, torch, frames, 0, prm=p3)
    finally:
        ctx.occl_release()
    for f, M in zip(frames, Mf):
        R, _, _ = ref.detect(f.D, f.angles, f.ratios, f.scan_len, **dict(f.params, neighbours=3))
        assert np.array_equal(M, R)


def test_two_pass_form_on_the_c3_batch(torch, ref):
    """The two-pass form (edge pass, per-frame prefix, scanline pass) stays
    bit-exact on the benched batch when the bucket selects it."""
    from paper_2408_14050_amd import occl
    frames = scenes.make_batch(seed=3000, n_frames=64)
    ctx = occl.Context(0)
    try:
        Mt, _, _ = _run(ctx, torch, frames, 16)
        assert ctx.occl_time_batched(1)["form"] == "two-pass"
    finally:
        ctx.occl_release()
    for i, (M, R) in enumerate(zip(Mt, _oracle(ref, frames))):
        assert np.array_equal(M, R), f"frame {i}"


def test_default_form_follows_the_tile_count(torch, ref):
    """Without a tuned bucket a batch takes the fused pass from 8 tiles per
    resident block (4,096 tiles on 256 CUs): one 1280x960 frame (300 tiles)
    keeps the two passes, 16 frames of the mixed batch (5,642 tiles) go
    fused; both bit-exact."""
    from paper_2408_14050_amd import occl
    cases = [([scenes.make_scene("c1", 1002)], "two-pass"), (scenes.make_batch(seed=3000, n_frames=16), "fused")]
    for frames, form in cases:
        print(f"default form: {len(frames)} frames, expect {form}", flush=True)
        ctx = occl.Context(0)
        try:
            Ds = [torch.from_numpy(np.ascontiguousarray(f.D)).cuda() for f in frames]
            Ms = [torch.full((f.n_views, f.H, f.W), 7, dtype=torch.uint8, device="cuda") for f in frames]
            batch = [(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)]
            ctx.occl_detect_batched(batch, frames[0].angles, frames[0].ratios, occl.params(**frames[0].params))
            torch.cuda.synchronize()
            assert ctx.occl_time_batched(1)["form"] == form
            Mg = [M.cpu().numpy() for M in Ms]
        finally:
            ctx.occl_release()
        for i, (M, R) in enumerate(zip(Mg, _oracle(ref, frames))):
            assert np.array_equal(M, R), f"{form} frame {i}"


def test_alternating_batches_keep_their_own_frame_table(torch, ref):
    """A repeated batch skips its frame-table upload; alternating two batches
    of different frames (and buffers) on one context, and then the first
    again with new contents in the same buffers, each result is still the
    oracle's."""
    from paper_2408_14050_amd import occl
    fa = scenes.make_batch(seed=3001, n_frames=16)
    fb = [scenes.make_scene("c1", 1003)] * 2
    fa2 = [scenes.Scene(f.name, f.seed, np.ascontiguousarray(f.D[:, ::-1]), f.angles, f.ratios, f.scan_len,
                        dict(f.params)) for f in fa]  # same shapes, mirrored contents
    print("alternating batches", flush=True)
    ctx = occl.Context(0)
    try:
        def put(frames):
            Ds = [torch.from_numpy(np.ascontiguousarray(f.D)).cuda() for f in frames]
            Ms = [torch.full((f.n_views, f.H, f.W), 7, dtype=torch.uint8, device="cuda") for f in frames]
            return Ds, Ms
        Da, Ma = put(fa)
        Db, Mb = put(fb)
        prm = occl.params(**fa[0].params)
        outs = []
        for frames, Ds, Ms in ((fa, Da, Ma), (fb, Db, Mb), (fa, Da, Ma)):
            batch = [(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)]
            ctx.occl_detect_batched(batch, frames[0].angles, frames[0].ratios, prm)
            torch.cuda.synchronize()
            outs.append((frames, [M.cpu().numpy() for M in Ms]))
        # same buffers and shapes, new contents: the table is the same, the masks are not
        for D, f in zip(Da, fa2):
            D.copy_(torch.from_numpy(f.D))
        batch = [(D, M, f.scan_len) for D, M, f in zip(Da, Ma, fa2)]
        ctx.occl_detect_batched(batch, fa2[0].angles, fa2[0].ratios, prm)
        torch.cuda.synchronize()
        outs.append((fa2, [M.cpu().numpy() for M in Ma]))
    finally:
        ctx.occl_release()
    for frames, Ms in outs:
        for i, (M, R) in enumerate(zip(Ms, _oracle(ref, frames))):
            assert np.array_equal(M, R), f"frame {i}"


@pytest.mark.parametrize("n_views", [1, 64])
def test_fused_one_and_the_most_views(torch, ref, n_views):
    """The fused pass with one view and with its maximum of 64 (a round then
    holds 64 strong pixels; the view index takes the entry's top bits):
    random angles, ratios in [1, 2.83], L from 1 to 127 per view and frame."""
    from paper_2408_14050_amd import occl
    rng = np.random.default_rng(900 + n_views)
    sizes = [(256, 160), (300, 97), (517, 40)]
    frames = [scenes.make_c1_like(int(rng.integers(0, 1 << 30)), W=w, H=h, n_objects=6) for w, h in sizes]
    angles = rng.uniform(0.0, 360.0, n_views)
    ratios = rng.uniform(1.0, 2.83, n_views).astype(np.float32)
    for f in frames:
        f.angles, f.ratios = angles, ratios
        f.scan_len = rng.integers(1, 128, n_views).astype(np.int32)
    print(f"fused {n_views} views", flush=True)
    ctx = occl.Context(0)
    try:
        Mf, _, _ = _run(ctx, torch, frames, 0)
        assert ctx.occl_time_batched(1)["form"] == "fused"
    finally:
        ctx.occl_release()
    for i, (M, f) in enumerate(zip(Mf, frames)):
        R = ref.detect(f.D, f.angles, f.ratios, f.scan_len, **f.params)[0]
        assert np.array_equal(M, R), f"frame {i} {f.W}x{f.H}: {int((M != R).sum())} bytes differ"
