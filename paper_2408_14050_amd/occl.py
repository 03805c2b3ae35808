"""Thin ctypes binding of libocclusion.so (include/occl.h).

Argument marshalling only: every step of the detector runs in the HIP
kernels of the library.  Tensors are torch tensors on a ROCm device; torch
provides the device memory and the stream, nothing else.  There is no CPU
fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocclusion.so")

OCCL_OK = 0
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "HIP", -4: "UNSUPPORTED",
          -5: "NO_MODEL", -6: "STATE"}
OCCL_MAX_VIEWS = 64
OCCL_MAX_SCAN_LEN = 1023
FLAG_SYNC = 1
FLAG_VALIDATE_INPUT = 2
FLAG_USE_CNN = 4
FLAG_BILINEAR = 8
FLAG_THIN = 16


class OcclError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class occl_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("edge_thr", C.c_float),
        ("disp_thr", C.c_float),
        ("dist_thr", C.c_float),
        ("neighbours", C.c_int32),
        ("scan_len", C.c_int32),
        ("scan_len_per_view", C.POINTER(C.c_int32)),
        ("flags", C.c_uint32),
        ("cnn_lo", C.c_float),
        ("cnn_hi", C.c_float),
    ]


class occl_frame(C.Structure):
    _fields_ = [
        ("D", C.c_void_p),
        ("H", C.c_int32),
        ("W", C.c_int32),
        ("M", C.c_void_p),
        ("scan_len_per_view", C.POINTER(C.c_int32)),
    ]


class occl_tune(C.Structure):
    _fields_ = [("edge_rows", C.c_int32), ("scan_blocks_per_cu", C.c_int32), ("ms", C.c_float)]


_lib = None

# name -> (restype, argtypes); the same names as the C ABI
_SIGS = {
    "occl_params_default": (None, [C.POINTER(occl_params)]),
    "occl_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_size_t, C.c_int32]),
    "occl_detect": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                              C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(occl_params),
                              C.c_void_p]),
    "occl_detect_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_float),
                                      C.POINTER(occl_params), C.c_void_p]),
    "occl_detect_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(occl_frame), C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_float),
                                      C.POINTER(occl_params)]),
    "occl_last_candidate_counts": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int32]),
    "occl_edges": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "occl_quality": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                               C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "occl_set_workspace_cap": (C.c_int, [C.c_void_p, C.c_size_t]),
    "occl_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "occl_confusion": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.POINTER(C.c_uint64)]),
    "occl_zbuffer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                               C.POINTER(C.c_double), C.POINTER(C.c_float), C.c_float, C.c_void_p]),
    "occl_median_fuse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "occl_sync": (C.c_int, [C.c_void_p]),
    "occl_release": (C.c_int, [C.c_void_p]),
    "occl_status_string": (C.c_char_p, [C.c_int]),
    "occl_last_error": (C.c_char_p, [C.c_void_p]),
    "occl_direction": (C.c_int, [C.c_double, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "occl_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "occl_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "occl_time_scanlines": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "occl_time_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "occl_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(occl_params),
                                C.c_void_p, C.c_int32, C.POINTER(occl_tune)]),
    "occl_autotune_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(occl_frame), C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_float),
                                        C.POINTER(occl_params), C.c_int32, C.POINTER(occl_tune)]),
    "occl_detect_routed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_double), C.POINTER(C.c_float),
                                     C.POINTER(occl_params), C.c_void_p, C.c_void_p, C.c_void_p]),
    "occl_cnn_num_params": (C.c_size_t, []),
    "occl_cnn_init": (C.c_int, [C.c_void_p, C.c_uint64]),
    "occl_cnn_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_size_t]),
    "occl_cnn_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_int64), C.c_size_t]),
    "occl_cnn_pack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                C.c_void_p]),
    "occl_cnn_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_void_p]),
    "occl_cnn_propose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                   C.c_void_p]),
    "occl_cnn_activation": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "occl_cnn_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "occl_cnn_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_float, C.POINTER(C.c_double)]),
    "occl_cnn_tile_targets": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_void_p]),
    "occl_tune_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "occl_tune_load": (C.c_int, [C.c_void_p, C.c_char_p]),
}
STAGES = ("edges", "scanlines", "cnn", "fallback", "batched")


def exported_symbols():
    return list(_SIGS)


def lib():
    """Loads libocclusion.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OcclError(-3, f"{LIB_PATH} is missing: run __graft_entry__.build() "
                                "(python -m paper_2408_14050_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def params(edge_thr=1.0, disp_thr=0.5, dist_thr=1.0, neighbours=1, scan_len=0,
           scan_len_per_view=None, flags=0, cnn_lo=0.05, cnn_hi=0.95):
    p = occl_params()
    lib().occl_params_default(C.byref(p))
    p.edge_thr, p.disp_thr, p.dist_thr = float(edge_thr), float(disp_thr), float(dist_thr)
    p.neighbours, p.scan_len, p.flags = int(neighbours), int(scan_len), int(flags)
    p.cnn_lo, p.cnn_hi = float(cnn_lo), float(cnn_hi)
    keep = None
    if scan_len_per_view is not None:
        keep = np.ascontiguousarray(np.atleast_1d(scan_len_per_view), dtype=np.int32)
        p.scan_len_per_view = keep.ctypes.data_as(C.POINTER(C.c_int32))
    p._keep = keep  # keep the host array alive as long as the struct
    return p


def direction(angle_deg: float):
    c, s = C.c_float(), C.c_float()
    st = lib().occl_direction(float(angle_deg), C.byref(c), C.byref(s))
    if st != OCCL_OK:
        raise OcclError(st, "occl_direction")
    return np.float32(c.value), np.float32(s.value)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def check_tensor(t, name: str, dtype, shape=None, dim=None, device=None):
    """Raises ValueError unless `t` is a contiguous tensor of `dtype` (with
    `dim` dimensions and the given `shape` where stated) on ROCm device
    `device`.  The C ABI receives a bare device pointer and assumes exactly
    that layout: a strided view, another dtype, a host tensor or a short
    buffer would be misread or written out of bounds."""
    if t is None:
        raise ValueError(f"{name} is None")
    if dim is not None and t.dim() != dim:
        raise ValueError(f"{name} must have {dim} dimensions, got shape {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(int(x) for x in t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major, no strides)")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a ROCm device tensor, got device {t.device}")
    if device is not None and t.device.index != int(device):
        raise ValueError(f"{name} is on device {t.device.index}, the context on {device}")
    return t


def check_frame(D, M, n_views: int, device=None):
    """D float32 [H, W] and M uint8 [n_views, H, W], both contiguous on the
    context's device (the layout occl_detect reads and writes)."""
    import torch
    check_tensor(D, "D", torch.float32, dim=2, device=device)
    H, W = int(D.shape[0]), int(D.shape[1])
    check_tensor(M, "M", torch.uint8, shape=(n_views, H, W), device=device)
    return H, W


class Context:
    """An occl_ctx bound to one ROCm device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None, max_pixels_hint: int = 0,
                 max_views_hint: int = 0):
        import torch
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().occl_init(C.byref(h), int(device), C.c_void_p(stream.cuda_stream),
                             int(max_pixels_hint), int(max_views_hint))
        if st != OCCL_OK:
            raise OcclError(st, "occl_init")
        self.h = h
        self.device = device

    # -- helpers -----------------------------------------------------------
    def _check(self, st, what):
        if st != OCCL_OK:
            msg = lib().occl_last_error(self.h)
            raise OcclError(st, f"{what}: {msg.decode() if msg else ''}")

    @staticmethod
    def _views(angles, ratios):
        a = np.ascontiguousarray(np.atleast_1d(angles), dtype=np.float64)
        r = np.ascontiguousarray(np.atleast_1d(ratios), dtype=np.float32)
        if a.shape != r.shape:
            raise ValueError("angles and ratios differ in length")
        return a, r

    # -- API ---------------------------------------------------------------
    def occl_detect(self, D, angles, ratios, prm: occl_params, M=None):
        """D: float32 [H, W] device tensor; returns M uint8 [V, H, W]."""
        torch = self._torch
        a, r = self._views(angles, ratios)
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        H, W = int(D.shape[0]), int(D.shape[1])
        if M is None:
            M = torch.empty((a.shape[0], H, W), dtype=torch.uint8, device=D.device)
        check_frame(D, M, int(a.shape[0]), self.device)
        st = lib().occl_detect(self.h, _ptr(D), H, W, int(a.shape[0]),
                               a.ctypes.data_as(C.POINTER(C.c_double)),
                               r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm), _ptr(M))
        self._check(st, "occl_detect")
        return M

    def occl_detect_noalloc(self, D, angles, ratios, prm: occl_params, M):
        """occl_detect with the workspace in the library's static device
        array (the call allocates no device memory): M must be given."""
        a, r = self._views(angles, ratios)
        H, W = check_frame(D, M, int(a.shape[0]), self.device)
        st = lib().occl_detect_noalloc(self.h, _ptr(D), H, W, int(a.shape[0]),
                                       a.ctypes.data_as(C.POINTER(C.c_double)),
                                       r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm), _ptr(M))
        self._check(st, "occl_detect_noalloc")
        return M

    def occl_detect_prepared(self, angles, ratios, prm: occl_params):
        """occl_detect with the views and parameters marshalled once: returns
        f(D, M) that calls the library with only the frame pointers and sizes
        per call (for tight loops over many frames of the same views)."""
        a, r = self._views(angles, ratios)
        ap = a.ctypes.data_as(C.POINTER(C.c_double))
        rp = r.ctypes.data_as(C.POINTER(C.c_float))
        pr = C.byref(prm)
        L, h, nv = lib(), self.h, int(a.shape[0])
        keep = (a, r, prm)
        seen = [None]  # the last (D, M) pair that passed the checks

        def detect(D, M):
            key = (D.data_ptr(), M.data_ptr(), tuple(D.shape), tuple(M.shape), D.dtype, M.dtype)
            if key != seen[0]:
                check_frame(D, M, nv, self.device)
                seen[0] = key
            st = L.occl_detect(h, C.c_void_p(D.data_ptr()), int(D.shape[0]), int(D.shape[1]), nv,
                               ap, rp, pr, C.c_void_p(M.data_ptr()))
            if st != OCCL_OK:
                self._check(st, "occl_detect")
            return M

        detect._keep = keep  # the marshalled arrays live as long as the function
        return detect

    def _frames(self, frames, n_views):
        arr = (occl_frame * max(1, len(frames)))()
        keep = []
        for i, (D, M, Ls) in enumerate(frames):
            check_frame(D, M, n_views, self.device)
            arr[i].D = D.data_ptr()
            arr[i].H, arr[i].W = int(D.shape[0]), int(D.shape[1])
            arr[i].M = M.data_ptr()
            if Ls is not None:
                l = np.ascontiguousarray(Ls, dtype=np.int32)
                keep.append(l)
                arr[i].scan_len_per_view = l.ctypes.data_as(C.POINTER(C.c_int32))
        return arr, keep

    def occl_detect_batched(self, frames, angles, ratios, prm: occl_params):
        """frames: list of (D, M, scan_len_per_view or None)."""
        a, r = self._views(angles, ratios)
        arr, keep = self._frames(frames, int(a.shape[0]))
        st = lib().occl_detect_batched(self.h, len(frames), arr, int(a.shape[0]),
                                       a.ctypes.data_as(C.POINTER(C.c_double)),
                                       r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm))
        self._check(st, "occl_detect_batched")

    def occl_autotune(self, D, angles, ratios, prm: occl_params, M, reps: int = 10):
        a, r = self._views(angles, ratios)
        check_frame(D, M, int(a.shape[0]), self.device)
        out = occl_tune()
        st = lib().occl_autotune(self.h, _ptr(D), int(D.shape[0]), int(D.shape[1]), int(a.shape[0]),
                                 a.ctypes.data_as(C.POINTER(C.c_double)),
                                 r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm), _ptr(M),
                                 int(reps), C.byref(out))
        self._check(st, "occl_autotune")
        return {"edge_rows": out.edge_rows, "scan_blocks_per_cu": out.scan_blocks_per_cu, "ms": out.ms}

    def occl_autotune_batched(self, frames, angles, ratios, prm: occl_params, reps: int = 5):
        a, r = self._views(angles, ratios)
        arr, keep = self._frames(frames, int(a.shape[0]))
        out = occl_tune()
        st = lib().occl_autotune_batched(self.h, len(frames), arr, int(a.shape[0]),
                                         a.ctypes.data_as(C.POINTER(C.c_double)),
                                         r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm),
                                         int(reps), C.byref(out))
        self._check(st, "occl_autotune_batched")
        return {"edge_rows": out.edge_rows, "scan_blocks_per_cu": out.scan_blocks_per_cu, "ms": out.ms}

    def occl_tune_save(self, path: str):
        self._check(lib().occl_tune_save(self.h, path.encode()), "occl_tune_save")

    def occl_tune_load(self, path: str):
        self._check(lib().occl_tune_load(self.h, path.encode()), "occl_tune_load")

    def occl_last_candidate_counts(self, n_views: int):
        out = np.zeros(n_views, np.int64)
        st = lib().occl_last_candidate_counts(self.h, out.ctypes.data_as(C.POINTER(C.c_int64)),
                                              int(n_views))
        self._check(st, "occl_last_candidate_counts")
        return out

    def occl_edges(self, D, E=None, A=None):
        torch = self._torch
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        for name, t in (("E", E), ("A", A)):
            if t is not None:
                check_tensor(t, name, torch.float32, shape=D.shape, device=self.device)
        st = lib().occl_edges(self.h, _ptr(D), int(D.shape[0]), int(D.shape[1]), _ptr(E), _ptr(A))
        self._check(st, "occl_edges")
        return E, A

    def occl_confusion(self, pred, ref):
        torch = self._torch
        check_tensor(pred, "pred", torch.uint8, device=self.device)
        check_tensor(ref, "ref", torch.uint8, shape=pred.shape, device=self.device)
        out = np.zeros(4, np.uint64)
        st = lib().occl_confusion(self.h, _ptr(pred), _ptr(ref), int(pred.numel()),
                                  out.ctypes.data_as(C.POINTER(C.c_uint64)))
        self._check(st, "occl_confusion")
        return {"tp": int(out[0]), "fp": int(out[1]), "fn": int(out[2]), "tn": int(out[3])}

    def occl_zbuffer(self, D, angles, ratios, beta: float = 0.5, M=None):
        """Forward-warping ground truth masks uint8 [V, H, W] (Eq. (7) reference)."""
        torch = self._torch
        a, r = self._views(angles, ratios)
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        H, W = int(D.shape[0]), int(D.shape[1])
        if M is None:
            M = torch.empty((a.shape[0], H, W), dtype=torch.uint8, device=D.device)
        check_frame(D, M, int(a.shape[0]), self.device)
        st = lib().occl_zbuffer(self.h, _ptr(D), H, W, int(a.shape[0]),
                                a.ctypes.data_as(C.POINTER(C.c_double)),
                                r.ctypes.data_as(C.POINTER(C.c_float)), float(beta), _ptr(M))
        self._check(st, "occl_zbuffer")
        return M

    def occl_median_fuse(self, maps, D=None):
        """maps: float32 [K, H, W] device tensor -> fused D [H, W] (NaN-ignoring median)."""
        torch = self._torch
        check_tensor(maps, "maps", torch.float32, dim=3, device=self.device)
        K, H, W = int(maps.shape[0]), int(maps.shape[1]), int(maps.shape[2])
        if D is None:
            D = torch.empty((H, W), dtype=torch.float32, device=maps.device)
        check_tensor(D, "D", torch.float32, shape=(H, W), device=self.device)
        st = lib().occl_median_fuse(self.h, _ptr(maps), K, H, W, _ptr(D))
        self._check(st, "occl_median_fuse")
        return D

    def occl_quality(self, pred, ref):
        """Eq. (7) from the library: precision, recall, F1, IoU and the counts."""
        torch = self._torch
        check_tensor(pred, "pred", torch.uint8, device=self.device)
        check_tensor(ref, "ref", torch.uint8, shape=pred.shape, device=self.device)
        q = np.zeros(4, np.float64)
        c = np.zeros(4, np.uint64)
        st = lib().occl_quality(self.h, _ptr(pred), _ptr(ref), int(pred.numel()),
                                q.ctypes.data_as(C.POINTER(C.c_double)),
                                c.ctypes.data_as(C.POINTER(C.c_uint64)))
        self._check(st, "occl_quality")
        return {"precision": float(q[0]), "recall": float(q[1]), "f1": float(q[2]), "iou": float(q[3]),
                "tp": int(c[0]), "fp": int(c[1]), "fn": int(c[2]), "tn": int(c[3])}

    def occl_set_workspace_cap(self, nbytes: int):
        self._check(lib().occl_set_workspace_cap(self.h, int(nbytes)), "occl_set_workspace_cap")

    def occl_workspace_bytes(self) -> int:
        n = C.c_size_t()
        self._check(lib().occl_workspace_bytes(self.h, C.byref(n)), "occl_workspace_bytes")
        return int(n.value)

    def occl_profile_enable(self, enable: bool = True):
        self._check(lib().occl_profile_enable(self.h, int(bool(enable))), "occl_profile_enable")

    def occl_profile_read(self):
        """{stage: (total_ms, launches)} since the last enable."""
        ms = np.zeros(len(STAGES), np.float64)
        n = np.zeros(len(STAGES), np.int64)
        st = lib().occl_profile_read(self.h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                     n.ctypes.data_as(C.POINTER(C.c_int64)))
        self._check(st, "occl_profile_read")
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def occl_time_scanlines(self, reps: int = 100):
        """Mean ms per scanline pass of the last occl_detect, re-run `reps`
        times back to back (synchronises; the masks do not change)."""
        ms = C.c_double()
        self._check(lib().occl_time_scanlines(self.h, int(reps), C.byref(ms)), "occl_time_scanlines")
        return ms.value

    def occl_time_batched(self, reps: int = 20):
        """Mean ms per batch of the two stages of the last
        occl_detect_batched (edge and scanline passes, or mask fill and
        fused pass), re-run `reps` times outside the graph."""
        ms = np.zeros(2, np.float64)
        form = C.c_int32()
        self._check(lib().occl_time_batched(self.h, int(reps), ms.ctypes.data_as(C.POINTER(C.c_double)),
                                            C.byref(form)), "occl_time_batched")
        if form.value == 1:
            return {"form": "fused", "clear": float(ms[0]), "fused": float(ms[1])}
        return {"form": "two-pass", "edges": float(ms[0]), "scanlines": float(ms[1])}

    def occl_detect_routed(self, D, angles, ratios, prm: occl_params, logits, M=None,
                           tile_state=None):
        """Exact path on the tiles the logits leave uncertain; fills the rest.
        logits: float32 [V, ceil(H/16), ceil(W/16)] device tensor."""
        torch = self._torch
        a, r = self._views(angles, ratios)
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        H, W = int(D.shape[0]), int(D.shape[1])
        if M is None:
            M = torch.empty((a.shape[0], H, W), dtype=torch.uint8, device=D.device)
        check_frame(D, M, int(a.shape[0]), self.device)
        tshape = (int(a.shape[0]), (H + 15) // 16, (W + 15) // 16)
        check_tensor(logits, "logits", torch.float32, shape=tshape, device=self.device)
        if tile_state is not None:
            check_tensor(tile_state, "tile_state", torch.uint8, shape=tshape, device=self.device)
        st = lib().occl_detect_routed(self.h, _ptr(D), H, W, int(a.shape[0]),
                                      a.ctypes.data_as(C.POINTER(C.c_double)),
                                      r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(prm),
                                      _ptr(logits), _ptr(M), _ptr(tile_state))
        self._check(st, "occl_detect_routed")
        return M

    # -- learned tile proposal ----------------------------------------------
    @staticmethod
    def occl_cnn_num_params():
        return int(lib().occl_cnn_num_params())

    def occl_cnn_init(self, seed: int):
        self._check(lib().occl_cnn_init(self.h, C.c_uint64(int(seed))), "occl_cnn_init")

    def occl_cnn_set_state(self, theta, m=None, v=None, step: int = 0):
        n = self.occl_cnn_num_params()
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in (theta, m, v)]
        for a in arrs:
            if a is not None and a.size != n:
                raise ValueError(f"expected {n} parameters")
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        st = lib().occl_cnn_set_state(self.h, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), int(step), n)
        self._check(st, "occl_cnn_set_state")

    def occl_cnn_get_state(self):
        n = self.occl_cnn_num_params()
        th, m, v = (np.zeros(n, np.float32) for _ in range(3))
        step = C.c_int64()
        st = lib().occl_cnn_get_state(self.h, th.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                      v.ctypes.data_as(C.c_void_p), C.byref(step), n)
        self._check(st, "occl_cnn_get_state")
        return th, m, v, int(step.value)

    def occl_cnn_pack(self, D, angles, ratios, scan_len, X=None):
        """Network input of every view: bf16 [V, H, W, 8] (returned as int16 storage)."""
        torch = self._torch
        a, r = self._views(angles, ratios)
        Ls = np.ascontiguousarray(np.atleast_1d(scan_len), dtype=np.int32)
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        H, W = int(D.shape[0]), int(D.shape[1])
        if X is None:
            X = torch.empty((a.shape[0], H, W, 8), dtype=torch.int16, device=D.device)
        st = lib().occl_cnn_pack(self.h, _ptr(D), H, W, int(a.shape[0]),
                                 a.ctypes.data_as(C.POINTER(C.c_double)),
                                 r.ctypes.data_as(C.POINTER(C.c_float)),
                                 Ls.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(X))
        self._check(st, "occl_cnn_pack")
        return X

    def occl_cnn_forward(self, X, Z=None):
        torch = self._torch
        N, H, W = int(X.shape[0]), int(X.shape[1]), int(X.shape[2])
        if Z is None:
            Z = torch.empty((N, (H + 15) // 16, (W + 15) // 16), dtype=torch.float32, device=X.device)
        st = lib().occl_cnn_forward(self.h, _ptr(X), N, H, W, _ptr(Z))
        self._check(st, "occl_cnn_forward")
        return Z

    def occl_cnn_propose(self, D, angles, ratios, scan_len, Z=None):
        """Logits [V, ceil(H/16), ceil(W/16)] of every view straight from D."""
        torch = self._torch
        a, r = self._views(angles, ratios)
        Ls = np.ascontiguousarray(np.atleast_1d(scan_len), dtype=np.int32)
        check_tensor(D, "D", torch.float32, dim=2, device=self.device)
        H, W = int(D.shape[0]), int(D.shape[1])
        if Z is None:
            Z = torch.empty((a.shape[0], (H + 15) // 16, (W + 15) // 16), dtype=torch.float32,
                            device=D.device)
        st = lib().occl_cnn_propose(self.h, _ptr(D), H, W, int(a.shape[0]),
                                    a.ctypes.data_as(C.POINTER(C.c_double)),
                                    r.ctypes.data_as(C.POINTER(C.c_float)),
                                    Ls.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(Z))
        self._check(st, "occl_cnn_propose")
        return Z

    def occl_cnn_activation(self, layer: int, N: int, H: int, W: int):
        """Output of hidden layer `layer` of the last forward pass on an
        [N, H, W, 8] input: bf16 [N, H_l, W_l, 32] (int16 storage)."""
        torch = self._torch
        h, w = H, W
        for l in range(layer + 1):
            if l < 4:
                h, w = (h + 1) // 2, (w + 1) // 2
        out = torch.empty((N, h, w, 32), dtype=torch.int16, device=f"cuda:{self.device}")
        st = lib().occl_cnn_activation(self.h, int(layer), _ptr(out), out.numel())
        self._check(st, "occl_cnn_activation")
        return out

    def occl_cnn_backward(self, X, T, want_grad=True):
        N, H, W = int(X.shape[0]), int(X.shape[1]), int(X.shape[2])
        loss = C.c_double()
        g = np.zeros(self.occl_cnn_num_params(), np.float32) if want_grad else None
        st = lib().occl_cnn_backward(self.h, _ptr(X), N, H, W, _ptr(T), C.byref(loss),
                                     None if g is None else g.ctypes.data_as(C.c_void_p))
        self._check(st, "occl_cnn_backward")
        return float(loss.value), g

    def occl_cnn_train_step(self, X, T, lr: float, want_loss=True):
        N, H, W = int(X.shape[0]), int(X.shape[1]), int(X.shape[2])
        loss = C.c_double()
        st = lib().occl_cnn_train_step(self.h, _ptr(X), N, H, W, _ptr(T), float(lr),
                                       C.byref(loss) if want_loss else None)
        self._check(st, "occl_cnn_train_step")
        return float(loss.value) if want_loss else None

    def occl_cnn_tile_targets(self, M, T=None):
        torch = self._torch
        n, H, W = int(M.shape[0]), int(M.shape[1]), int(M.shape[2])
        if T is None:
            T = torch.empty((n, (H + 15) // 16, (W + 15) // 16), dtype=torch.float32, device=M.device)
        st = lib().occl_cnn_tile_targets(self.h, _ptr(M), n, H, W, _ptr(T))
        self._check(st, "occl_cnn_tile_targets")
        return T

    def occl_sync(self):
        self._check(lib().occl_sync(self.h), "occl_sync")

    def occl_release(self):
        if self.h:
            st = lib().occl_release(self.h)
            self.h = None
            if st != OCCL_OK:
                raise OcclError(st, "occl_release")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().occl_release(self.h)
        except Exception:
            pass


@dataclass
class SceneRun:
    M: object
    n_cand: np.ndarray


def detect_scene(ctx: Context, sc, D=None, want_counts=False, flags=FLAG_SYNC):
    """Runs one generated scene (paper_2408_14050_amd.scenes.Scene) on the GPU."""
    import torch
    if D is None:
        D = torch.from_numpy(sc.D).to(f"cuda:{ctx.device}")
    p = params(**sc.params, scan_len_per_view=sc.scan_len, flags=flags)
    M = ctx.occl_detect(D, sc.angles, sc.ratios, p)
    nc = ctx.occl_last_candidate_counts(sc.n_views) if want_counts else None
    return SceneRun(M, nc)
