"""The limitation cases of Sec. 5 on the GPU: the library's masks and its
D-only z-buffer equal the oracle's bit for bit, and miss against the
ground truth of every painted surface exactly the pixels the CPU tests
predict (tests/test_limitations.py)."""
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


@pytest.mark.parametrize("kind", scenes.LIMITATION_CASES)
def test_limitation_case_on_gpu(torch, ref, kind):
    from oracle import layered_gt
    from paper_2408_14050_amd import occl
    from test_limitations import PREDICTED
    sc, layers = scenes.limitation_scene(kind)
    ctx = occl.Context(0)
    try:
        D = torch.from_numpy(sc.D).cuda()
        prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
        M = ctx.occl_detect(D, sc.angles, sc.ratios, prm).cpu().numpy()
        Z = ctx.occl_zbuffer(D, sc.angles, sc.ratios, sc.params["disp_thr"]).cpu().numpy()
    finally:
        ctx.occl_release()
    M_ref, _, _ = ref.detect_scene(sc)
    np.testing.assert_array_equal(M, M_ref)
    np.testing.assert_array_equal(Z, ref.zbuffer(sc.D, sc.angles, sc.ratios, sc.params["disp_thr"]))
    Z_T = layered_gt.zbuffer_layers(sc.D, layers, sc.angles, sc.ratios, sc.params["disp_thr"])
    x0, x1, y0, y1 = PREDICTED[kind]
    missed = Z_T.astype(bool) & ~M.astype(bool)
    assert int(missed.sum()) == (x1 - x0) * (y1 - y0)
    assert missed[0, y0:y1, x0:x1].all()
