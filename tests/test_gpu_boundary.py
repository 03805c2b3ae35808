"""C-ABI contract on the GPU: the workspace cap, a context's own stream,
Eq. (7)'s ratios from the library and the binding's tensor checks."""
import ctypes as C

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


def test_workspace_cap_refuses_before_enqueueing(torch, ref):
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        sc = scenes.make_scene("c1", 1004)
        D = torch.from_numpy(sc.D).cuda()
        prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=occl.FLAG_SYNC)
        base = ctx.occl_workspace_bytes()
        ctx.occl_set_workspace_cap(base + (1 << 20))  # the c1 lists need about 40 MB
        M = torch.full((sc.n_views, sc.H, sc.W), 7, dtype=torch.uint8, device="cuda")
        with pytest.raises(occl.OcclError) as ei:
            ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
        assert ei.value.status == -2  # OCCL_ERR_OUT_OF_MEMORY
        torch.cuda.synchronize()
        assert bool((M == 7).all())  # nothing was enqueued
        assert ctx.occl_workspace_bytes() == base
        ctx.occl_set_workspace_cap(0)  # unlimited again: the same call now runs
        ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
        M_ref, _, _ = ref.detect_scene(sc)
        assert np.array_equal(M.cpu().numpy(), M_ref)
    finally:
        ctx.occl_release()


def test_null_stream_gives_the_context_its_own_stream(torch, ref):
    from paper_2408_14050_amd import occl
    lib = occl.lib()
    h = C.c_void_p()
    assert lib.occl_init(C.byref(h), 0, None, 0, 0) == occl.OCCL_OK
    try:
        sc = scenes.make_scene("c0", 11)
        D = torch.from_numpy(sc.D).cuda()
        M = torch.full((1, sc.H, sc.W), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()  # D is written before the context's stream reads it
        a = np.ascontiguousarray(sc.angles, np.float64)
        r = np.ascontiguousarray(sc.ratios, np.float32)
        prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len)
        st = lib.occl_detect(h, C.c_void_p(D.data_ptr()), sc.H, sc.W, 1,
                             a.ctypes.data_as(C.POINTER(C.c_double)),
                             r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm),
                             C.c_void_p(M.data_ptr()))
        assert st == occl.OCCL_OK
        assert lib.occl_sync(h) == occl.OCCL_OK
        M_ref, _, _ = ref.detect_scene(sc)
        assert np.array_equal(M.cpu().numpy(), M_ref)
    finally:
        assert lib.occl_release(h) == occl.OCCL_OK


def test_quality_ratios_from_the_library(torch, ref):
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        rng = np.random.default_rng(5)
        a = (rng.random(300_001) < 0.3).astype(np.uint8)
        b = (rng.random(300_001) < 0.2).astype(np.uint8)
        q = ctx.occl_quality(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        qr = ref.quality(a, b)
        for k in ("tp", "fp", "fn", "tn"):
            assert q[k] == qr[k]
        for k in ("precision", "recall", "f1", "iou"):
            assert q[k] == pytest.approx(qr[k], rel=1e-15, abs=0)
        # empty masks: no errors to count
        z = torch.zeros(1000, dtype=torch.uint8, device="cuda")
        q0 = ctx.occl_quality(z, z)
        assert (q0["precision"], q0["recall"], q0["iou"]) == (1.0, 1.0, 1.0)
    finally:
        ctx.occl_release()


def test_binding_refuses_bad_tensors_on_the_device(torch):
    from paper_2408_14050_amd import occl
    ctx = occl.Context(0)
    try:
        prm = occl.params(scan_len=10)
        D = torch.zeros((32, 80), device="cuda")
        with pytest.raises(ValueError, match="contiguous"):
            ctx.occl_detect(D[:, ::2], [0.0], [1.0], prm)
        with pytest.raises(ValueError, match="shape"):
            ctx.occl_detect(D, [0.0, 90.0], [1.0, 1.0], prm,
                            M=torch.zeros((1, 32, 80), dtype=torch.uint8, device="cuda"))
        with pytest.raises(ValueError, match="float32"):
            ctx.occl_detect(D.double(), [0.0], [1.0], prm)
        with pytest.raises(ValueError, match="device tensor"):
            ctx.occl_detect(D.cpu(), [0.0], [1.0], prm)
    finally:
        ctx.occl_release()
