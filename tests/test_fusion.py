"""Median fusion of per-view disparity maps (the step before the detector):
the oracle against numpy's nanmedian and order-statistic properties on the
CPU; the GPU kernel against the oracle, bit for bit."""
import warnings

import numpy as np
import pytest

from paper_2408_14050_amd import scenes


def _nanmedian(m):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        return np.nanmedian(m, axis=0)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 7, 8, 9, 16])
def test_oracle_median_is_nanmedian(ref, K):
    rng = np.random.default_rng(K)
    m = rng.normal(size=(K, 31, 45)).astype(np.float32)
    m[rng.uniform(size=m.shape) < 0.25] = np.nan
    m[:, 0, :3] = np.nan                      # all-NaN pixels
    out = ref.median_fuse(m)
    np.testing.assert_array_equal(out, _nanmedian(m))
    assert np.isnan(out[0, :3]).all()


def test_median_rejects_minority_outliers(ref):
    """With fewer than half of the values outliers, the median stays inside
    the range of the inliers (a property of the order statistic)."""
    rng = np.random.default_rng(3)
    K = 9
    D = np.full((20, 20), 10.0, np.float32)
    m = np.repeat(D[None], K, axis=0) + rng.uniform(-0.2, 0.2, size=(K, 20, 20)).astype(np.float32)
    m[:4] = rng.uniform(100, 200, size=(4, 20, 20))   # 4 of 9 outliers everywhere
    out = ref.median_fuse(m)
    assert np.all(out >= 9.8) and np.all(out <= 10.2)


def test_fusion_recovers_scene(ref):
    sc = scenes.make_c1_like(5, W=160, H=120, n_objects=8)
    maps = scenes.fusion_maps(9, sc.D, K=8)
    out = ref.median_fuse(maps)
    err = np.abs(out - sc.D)
    assert np.nanmedian(err) < 0.25 and np.mean(err < 1.0) > 0.99


@pytest.mark.gpu
@pytest.mark.parametrize("K", list(range(1, 17)))
def test_gpu_median_parity(ref, K):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        rng = np.random.default_rng(100 + K)
        for H, W in [(37, 53), (1, 1), (3, 4), (960, 1280)]:
            m = (rng.normal(size=(K, H, W)) * 10).astype(np.float32)
            m[rng.uniform(size=m.shape) < 0.2] = np.nan
            if H > 1:
                m[:, 1, :5] = np.nan
            D = ctx.occl_median_fuse(torch.from_numpy(m).cuda()).cpu().numpy()
            np.testing.assert_array_equal(D, ref.median_fuse(m), err_msg=f"K={K} {H}x{W}")
    finally:
        ctx.occl_release()


@pytest.mark.gpu
def test_gpu_median_rejects_too_many_maps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        with pytest.raises(occl.OcclError):
            ctx.occl_median_fuse(torch.zeros((17, 4, 4), dtype=torch.float32, device="cuda"))
    finally:
        ctx.occl_release()
