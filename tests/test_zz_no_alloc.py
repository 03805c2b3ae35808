"""occl_detect_noalloc, the exact path with its workspace in the library's
static device array, called through the C ABI and compared with
occl_detect's masks (bit for bit) on two calls in a row, the second with a
smaller frame; a frame too large for the array is refused with nothing
written."""
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


def _noalloc(lib, h, D, angles, ratios, prm, M):
    a = np.ascontiguousarray(angles, dtype=np.float64)
    r = np.ascontiguousarray(ratios, dtype=np.float32)
    return lib.occl_detect_noalloc(h, C.c_void_p(D.data_ptr()), int(D.shape[0]), int(D.shape[1]),
                                   int(a.shape[0]), a.ctypes.data_as(C.POINTER(C.c_double)),
                                   r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm),
                                   C.c_void_p(M.data_ptr()))


def test_noalloc_matches_detect(torch, ref):
    from paper_2408_14050_amd import occl
    lib = occl.lib()
    ctx = occl.Context(0)
    try:
        # two calls in a row, the second with a smaller frame (fewer views,
        # smaller lists: the array keeps the first call's contents)
        for name, seed in (("c1", 1002), ("c0", 3)):
            sc = scenes.make_scene(name, seed)
            print(f"noalloc {name} seed {seed} {sc.W}x{sc.H} x{sc.n_views}", flush=True)
            D = torch.from_numpy(sc.D).cuda()
            prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len)
            M_ref = ctx.occl_detect(D, sc.angles, sc.ratios, prm)
            M = torch.full((sc.n_views, sc.H, sc.W), 7, dtype=torch.uint8, device="cuda")
            st = _noalloc(lib, ctx.h, D, sc.angles, sc.ratios, prm, M)
            assert st == occl.OCCL_OK, lib.occl_last_error(ctx.h)
            torch.cuda.synchronize()
            assert torch.equal(M, M_ref), f"{name}: {int((M != M_ref).sum())} bytes differ"
            M_or, _, _ = ref.detect_scene(sc)
            assert np.array_equal(M.cpu().numpy(), M_or)
        # the automatic scan length reads D's statistics through the array
        sc = scenes.make_scene("c1", 1003)
        D = torch.from_numpy(sc.D).cuda()
        prm = occl.params(**sc.params, scan_len=0)
        M_ref = ctx.occl_detect(D, sc.angles, sc.ratios, prm)
        M = torch.full_like(M_ref, 7)
        assert _noalloc(lib, ctx.h, D, sc.angles, sc.ratios, prm, M) == occl.OCCL_OK
        torch.cuda.synchronize()
        assert torch.equal(M, M_ref)
    finally:
        ctx.occl_release()


def test_noalloc_refuses_oversize_frame(torch):
    from paper_2408_14050_amd import occl
    lib = occl.lib()
    ctx = occl.Context(0)
    try:
        H, W = 2048, 4096  # 8 views: about 256 MiB of lists
        angles, ratios = scenes.views_3x3()
        D = torch.zeros((H, W), dtype=torch.float32, device="cuda")
        M = torch.full((8, H, W), 7, dtype=torch.uint8, device="cuda")
        prm = occl.params(scan_len=50)
        st = _noalloc(lib, ctx.h, D, angles, ratios, prm, M)
        assert st == -4  # OCCL_ERR_UNSUPPORTED
        assert b"scratch" in lib.occl_last_error(ctx.h)
        torch.cuda.synchronize()
        assert bool((M == 7).all())  # nothing written
        # a frame that fits still works after the refusal
        sc = scenes.make_scene("c0", 5)
        Ds = torch.from_numpy(sc.D).cuda()
        p0 = occl.params(**sc.params, scan_len_per_view=sc.scan_len)
        Ms = torch.full((1, sc.H, sc.W), 7, dtype=torch.uint8, device="cuda")
        assert _noalloc(lib, ctx.h, Ds, sc.angles, sc.ratios, p0, Ms) == occl.OCCL_OK
        torch.cuda.synchronize()
        assert torch.equal(Ms, ctx.occl_detect(Ds, sc.angles, sc.ratios, p0))
    finally:
        ctx.occl_release()
