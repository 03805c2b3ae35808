"""Trainer and evaluator of the learned tile proposal.

Training data: synthetic frames with the 1280x960 scene statistics
(paper_2408_14050_amd.scenes.make_c1_like), 8 peripheral views on a 3x3
grid.  Labels come from the exact method (occl_detect) run on the GPU on the
FULL frame; random 256x256 crops (aligned to the 16-pixel tile grid) of the
masks give the tile targets (occluded fraction per 16x16 tile).  Each crop
keeps a 257x257 window of D so that the network input of the crop (packed
by occl_cnn_pack) sees the true forward differences on its last row and
column.  Every forward, backward and Adam step runs in the library's HIP
kernels; torch only holds the buffers and slices crops out of them.

    python -m paper_2408_14050_amd.train_tile_cnn --frames 2500 --crops 8 \\
        --steps 3000 --out paper_2408_14050_amd/weights/tile_cnn_c1.npz

Evaluation (--eval N): N held-out 1920x1080 frames x 8 views; pooled IoU,
precision and recall (Eq. 7 counts from occl_confusion) of the routed masks
against the exact masks, and the share of tiles that fall back.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2408_14050_amd import scenes  # noqa: E402

CROP = 256
TRAIN_SEED0 = 400000
EVAL_SEED0 = 4100
CALIB_SEED0 = 4200      # calibration frames: disjoint from training and evaluation seeds
LAST_LAYER_PARAMS = 3 * 3 * 32 + 1  # the final 32 -> 1 convolution's weights and bias (end of theta)
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "tile_cnn_c1.npz")


def _gen(args):
    seed, W, H = args
    sc = scenes.make_c1_like(seed, W=W, H=H)
    return seed, sc.D, np.asarray(sc.scan_len, np.int32)


def save_state(ctx, path, meta, with_optimizer=False):
    """Weights (and optionally the Adam moments, for resuming) as plain arrays."""
    th, m, v, step = ctx.occl_cnn_get_state()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    extra = {"m": m, "v": v} if with_optimizer else {}
    np.savez(path, theta=th, step=np.int64(step),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **extra)


def load_state(ctx, path=DEFAULT_WEIGHTS, with_optimizer=False):
    """Loads weights saved by save_state (plain arrays, no pickles)."""
    z = np.load(path, allow_pickle=False)
    if with_optimizer and "m" in z.files:
        ctx.occl_cnn_set_state(z["theta"], z["m"], z["v"], int(z["step"]))
    else:
        ctx.occl_cnn_set_state(z["theta"], step=int(z["step"]))
    return json.loads(bytes(z["meta"]).decode())


class CropSet:
    """D windows (257x257), scan lengths and tile targets of training crops,
    resident on the GPU."""

    def __init__(self, torch, n_max):
        self.torch = torch
        self.D = torch.empty((n_max, CROP + 1, CROP + 1), dtype=torch.float32, device="cuda")
        self.T = torch.empty((n_max, 8, CROP // 16, CROP // 16), dtype=torch.float32, device="cuda")
        self.L = np.zeros((n_max, 8), np.int32)
        self.n = 0

    def add_frame(self, ctx, D_host, Ls, angles, ratios, rng, n_crops):
        from paper_2408_14050_amd import occl
        torch = self.torch
        H, W = D_host.shape
        D = torch.from_numpy(D_host).cuda()
        M = ctx.occl_detect(D, angles, ratios, occl.params(scan_len_per_view=Ls))
        ys = rng.integers(0, (H - CROP - 1) // 16 + 1, size=n_crops) * 16
        xs = rng.integers(0, (W - CROP - 1) // 16 + 1, size=n_crops) * 16
        for y0, x0 in zip(ys, xs):
            i = self.n
            self.D[i].copy_(D[y0:y0 + CROP + 1, x0:x0 + CROP + 1])
            ctx.occl_cnn_tile_targets(M[:, y0:y0 + CROP, x0:x0 + CROP].contiguous(), T=self.T[i])
            self.L[i] = Ls
            self.n += 1


def pack_batch(ctx, crops, idx, angles, ratios, Xb, tmp):
    for j, i in enumerate(idx):
        ctx.occl_cnn_pack(crops.D[i], angles, ratios, crops.L[i], X=tmp)
        Xb[8 * j:8 * j + 8].copy_(tmp[:, :CROP, :CROP, :])


def train(args):
    pool = None
    if args.workers > 1:
        # worker processes are forked before this process touches the GPU
        pool = mp.get_context("fork").Pool(args.workers)
    import torch
    from paper_2408_14050_amd import occl
    angles, ratios = scenes.views_3x3()
    ctx = occl.Context(0)
    rng = np.random.default_rng(args.seed)
    crops = CropSet(torch, args.frames * args.crops)
    t0 = time.time()
    jobs = [(TRAIN_SEED0 + k, 1280, 960) for k in range(args.frames)]
    it = pool.imap(_gen, jobs, chunksize=4) if pool else map(_gen, jobs)
    for k, (seed, D, Ls) in enumerate(it):
        crops.add_frame(ctx, D, Ls, angles, ratios, rng, args.crops)
        if (k + 1) % 250 == 0:
            print(f"data: {k + 1}/{args.frames} frames, {time.time() - t0:.1f} s", flush=True)
    if pool:
        pool.close()
        pool.join()
    torch.cuda.synchronize()
    frac = crops.T[:crops.n].mean().item()
    nonempty = (crops.T[:crops.n] > 0).float().mean().item()
    print(f"data: {crops.n} crops x 8 views, mean tile fraction {frac:.4f}, "
          f"non-empty tiles {nonempty:.4f}, {time.time() - t0:.1f} s", flush=True)

    ctx.occl_cnn_init(args.seed)
    B = args.batch
    Xb = torch.empty((8 * B, CROP, CROP, 8), dtype=torch.int16, device="cuda")
    Tb = torch.empty((8 * B, CROP // 16, CROP // 16), dtype=torch.float32, device="cuda")
    tmp = torch.empty((8, CROP + 1, CROP + 1, 8), dtype=torch.int16, device="cuda")
    t1 = time.time()
    losses = []
    for step in range(args.steps):
        lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1 + math.cos(math.pi * step / args.steps))
        idx = rng.choice(crops.n, size=B, replace=False)
        pack_batch(ctx, crops, idx, angles, ratios, Xb, tmp)
        Tb.copy_(crops.T[torch.from_numpy(idx).cuda()].reshape(8 * B, CROP // 16, CROP // 16))
        want = (step % 100 == 0) or step == args.steps - 1
        loss = ctx.occl_cnn_train_step(Xb, Tb, lr, want_loss=want)
        if want:
            losses.append((step, loss))
            print(f"step {step} loss {loss:.5f} lr {lr:.2e} {time.time() - t1:.1f} s", flush=True)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    meta = {"frames": args.frames, "crops_per_frame": args.crops, "steps": args.steps,
            "batch_crops": B, "lr": args.lr, "lr_min": args.lr_min, "seed": args.seed,
            "train_seeds": [TRAIN_SEED0, TRAIN_SEED0 + args.frames - 1],
            "final_loss": losses[-1][1], "train_seconds": round(train_s, 2),
            "mean_tile_fraction": frac}
    save_state(ctx, args.out, meta, with_optimizer=args.save_optimizer)
    print("saved", args.out, json.dumps(meta), flush=True)
    return ctx


def evaluate(ctx, n_frames, bands, W=1920, H=1080):
    """Pooled Eq. (7) counts of routed vs exact masks on held-out frames."""
    import torch
    from paper_2408_14050_amd import occl
    angles, ratios = scenes.views_3x3()
    acc = {b: {"tp": 0, "fp": 0, "fn": 0, "exact_tiles": 0, "tiles": 0} for b in bands}
    for k in range(n_frames):
        sc = scenes.make_c1_like(EVAL_SEED0 + k, W=W, H=H)
        D = torch.from_numpy(sc.D).cuda()
        M = ctx.occl_detect(D, angles, ratios, occl.params(scan_len_per_view=sc.scan_len))
        X = ctx.occl_cnn_pack(D, angles, ratios, sc.scan_len)
        Z = ctx.occl_cnn_forward(X)
        st = torch.empty(Z.shape, dtype=torch.uint8, device="cuda")
        for b in bands:
            prm = occl.params(scan_len_per_view=sc.scan_len, cnn_lo=b[0], cnn_hi=b[1])
            Mr = ctx.occl_detect_routed(D, angles, ratios, prm, Z, tile_state=st)
            c = ctx.occl_confusion(Mr, M)
            a = acc[b]
            a["tp"] += c["tp"]
            a["fp"] += c["fp"]
            a["fn"] += c["fn"]
            a["exact_tiles"] += int((st == 2).sum().item())
            a["tiles"] += st.numel()
    out = {}
    for b, a in acc.items():
        tp, fp, fn = a["tp"], a["fp"], a["fn"]
        out[f"{b[0]}-{b[1]}"] = {
            "iou": tp / max(1, tp + fp + fn), "precision": tp / max(1, tp + fp),
            "recall": tp / max(1, tp + fn), "exact_tile_share": a["exact_tiles"] / a["tiles"]}
    return out


def routed_iou(ctx, frames, band, scale=1.0):
    """Pooled IoU (Eq. 7 counts) of routed against exact masks, the logits
    scaled by `scale` on the way (a trial of the calibration; the shipped
    weights carry the scale in their last layer instead), and the share of
    tiles that fall back."""
    import torch
    from paper_2408_14050_amd import occl
    tp = fp = fn = ex = nt = 0
    for D, M, Z, Ls, angles, ratios in frames:
        st = torch.empty(Z.shape, dtype=torch.uint8, device="cuda")
        prm = occl.params(scan_len_per_view=Ls, cnn_lo=band[0], cnn_hi=band[1])
        Mr = ctx.occl_detect_routed(D, angles, ratios, prm, Z * scale if scale != 1.0 else Z, tile_state=st)
        c = ctx.occl_confusion(Mr, M)
        tp, fp, fn = tp + c["tp"], fp + c["fp"], fn + c["fn"]
        ex += int((st == 2).sum().item())
        nt += st.numel()
    return tp / max(1, tp + fp + fn), ex / max(1, nt)


def calibrate(ctx, n_frames, band=(0.05, 0.95), target=0.992, W=1920, H=1080):
    """Temperature calibration of the proposal: the largest scale t in
    (0, 1] of the logits for which the routed masks of n_frames calibration
    frames (seeds CALIB_SEED0...) reach `target` IoU against the exact masks
    at the configured band.  t is folded into the last layer (its weights
    and bias times t), so inference is unchanged; the result is checked
    again with the scaled weights.  Returns the table of trials."""
    import torch
    from paper_2408_14050_amd import occl
    angles, ratios = scenes.views_3x3()

    def frames_now():
        out = []
        for k in range(n_frames):
            sc = scenes.make_c1_like(CALIB_SEED0 + k, W=W, H=H)
            D = torch.from_numpy(sc.D).cuda()
            M = ctx.occl_detect(D, angles, ratios, occl.params(scan_len_per_view=sc.scan_len))
            Z = ctx.occl_cnn_propose(D, angles, ratios, sc.scan_len)
            out.append((D, M, Z, sc.scan_len, angles, ratios))
        return out

    frames = frames_now()
    trials = []
    t = 1.0
    chosen = None
    while t > 0.2:
        iou, share = routed_iou(ctx, frames, band, t)
        trials.append({"scale": round(t, 4), "iou": round(iou, 5), "exact_tile_share": round(share, 5)})
        if iou >= target and chosen is None:
            chosen = t
            break
        t -= 0.02
    if chosen is None:
        raise RuntimeError(f"no scale reaches IoU {target}: {trials}")
    th, m, v, step = ctx.occl_cnn_get_state()
    for scale in (chosen, chosen - 0.02, chosen - 0.04):
        th2 = th.copy()
        th2[-LAST_LAYER_PARAMS:] *= np.float32(scale)
        ctx.occl_cnn_set_state(th2, m, v, step)
        iou, share = routed_iou(ctx, frames_now(), band)
        trials.append({"scale": round(scale, 4), "folded": True, "iou": round(iou, 5),
                       "exact_tile_share": round(share, 5)})
        if iou >= target:
            return {"scale": round(scale, 4), "band": list(band), "target_iou": target,
                    "calibration_seeds": [CALIB_SEED0, CALIB_SEED0 + n_frames - 1], "trials": trials}
    raise RuntimeError(f"folded scales miss IoU {target}: {trials}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=2500)
    ap.add_argument("--crops", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16, help="crops per step (x 8 views)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=5e-5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval", type=int, default=16, help="held-out 1920x1080 frames (0: skip)")
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--save-optimizer", action="store_true", help="also save Adam moments")
    ap.add_argument("--calibrate", type=int, default=0, metavar="N",
                    help="temperature-calibrate the saved weights on N frames for IoU 0.992 at [0.05, 0.95] "
                         "(a margin over the 0.99 bar) and save them again")
    args = ap.parse_args()
    if args.eval_only or args.calibrate:
        from paper_2408_14050_amd import occl
        ctx = occl.Context(0)
        meta = load_state(ctx, args.out)
    else:
        ctx = train(args)
    if args.calibrate:
        if "calibration" in meta:
            raise SystemExit(f"{args.out} is calibrated already: {meta['calibration']}")
        cal = calibrate(ctx, args.calibrate)
        meta["calibration"] = cal
        print("calibration", json.dumps(cal), flush=True)
        save_state(ctx, args.out, meta)
    if args.eval:
        bands = [(0.05, 0.95), (0.02, 0.98), (0.01, 0.99), (0.005, 0.995), (0.002, 0.998)]
        res = evaluate(ctx, args.eval, bands)
        for k, v in res.items():
            print("eval", k, json.dumps({kk: round(vv, 5) for kk, vv in v.items()}), flush=True)


if __name__ == "__main__":
    main()
