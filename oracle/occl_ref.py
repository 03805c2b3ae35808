"""ctypes wrapper of the C++ CPU oracle (liboccl_ref.so) -- TEST INFRASTRUCTURE.

Every function mirrors one ``occl_ref_*`` entry point of ``occl_ref.cpp``;
arrays are numpy host arrays.  See the C++ file for the readings of the
paper each step follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=True)
        L = C.CDLL(path)
        fp = C.POINTER(C.c_float)
        u8 = C.POINTER(C.c_ubyte)
        i64 = C.POINTER(C.c_longlong)
        i32 = C.POINTER(C.c_int)
        dp = C.POINTER(C.c_double)
        L.occl_ref_direction.argtypes = [C.c_double, fp, fp]
        L.occl_ref_edges.argtypes = [fp, C.c_int, C.c_int, fp, fp, fp, fp]
        L.occl_ref_candidates.argtypes = [fp, C.c_int, C.c_int, C.c_double, C.c_float, u8, i64]
        L.occl_ref_line.argtypes = [C.c_int, fp, u8, C.c_int, C.c_float, C.c_float, C.c_float,
                                    C.c_int, u8]
        L.occl_ref_scan_len.argtypes = [fp, C.c_int, C.c_int, C.c_int, fp, C.c_int, i32]
        L.occl_ref_detect.argtypes = [fp, C.c_int, C.c_int, C.c_int, dp, fp, i32, C.c_float,
                                      C.c_float, C.c_float, C.c_int, u8, u8, i64]
        L.occl_ref_confusion.argtypes = [u8, u8, C.c_longlong, i64]
        L.occl_ref_zbuffer.argtypes = [fp, C.c_int, C.c_int, C.c_int, dp, fp, C.c_float, u8]
        L.occl_ref_median_fuse.argtypes = [fp, C.c_int, C.c_longlong, fp]
        L.occl_ref_detect_ex.argtypes = [fp, C.c_int, C.c_int, C.c_int, dp, fp, i32, C.c_float,
                                         C.c_float, C.c_float, C.c_int, u8, u8, i64, C.c_int]
        L.occl_ref_sample.argtypes = [fp, C.c_int, C.c_int, C.c_float, C.c_float, C.c_int, fp]
        L.occl_ref_scanline_pixels.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                               C.c_int, i32, i32, C.c_int]
        L.occl_ref_detect_window.argtypes = [fp, C.c_int, C.c_int, C.c_int, dp, fp, i32, C.c_float,
                                             C.c_float, C.c_float, C.c_int, C.c_int, C.c_int,
                                             C.c_int, C.c_int, u8]
        L.occl_ref_detect_window.restype = C.c_int
        for f in ("occl_ref_direction", "occl_ref_edges", "occl_ref_candidates", "occl_ref_line",
                  "occl_ref_scan_len", "occl_ref_detect", "occl_ref_confusion",
                  "occl_ref_scanline_pixels"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def direction(angle_deg: float):
    c, s = C.c_float(), C.c_float()
    rc = lib().occl_ref_direction(float(angle_deg), C.byref(c), C.byref(s))
    if rc != 0:
        raise ValueError("invalid angle")
    return np.float32(c.value), np.float32(s.value)


def edges(D):
    D = _f32(D)
    H, W = D.shape
    ex, ey, E, A = (np.empty((H, W), np.float32) for _ in range(4))
    rc = lib().occl_ref_edges(_p(D, C.c_float), H, W, _p(ex, C.c_float), _p(ey, C.c_float),
                              _p(E, C.c_float), _p(A, C.c_float))
    assert rc == 0
    return ex, ey, E, A


def candidates(D, angle_deg: float, gamma: float):
    D = _f32(D)
    H, W = D.shape
    out = np.empty((H, W), np.uint8)
    n = C.c_longlong()
    rc = lib().occl_ref_candidates(_p(D, C.c_float), H, W, float(angle_deg), float(gamma),
                                   _p(out, C.c_ubyte), C.byref(n))
    assert rc == 0
    return out


def line(V, r: float, zeta: float, beta: float, neighbours: int = 1, g0: int | None = None,
         valid=None):
    V = _f32(V)
    n = V.shape[0]
    if g0 is None:
        g0 = -(n // 2)
    hit = np.zeros(n, np.uint8)
    vd = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    rc = lib().occl_ref_line(n, _p(V, C.c_float), _p(vd, C.c_ubyte), int(g0), float(r),
                             float(zeta), float(beta), int(neighbours), _p(hit, C.c_ubyte))
    if rc != 0:
        raise ValueError("invalid argument")
    return hit


def scanline_pixels(cx, cy, angle_deg, L, H, W):
    """(xy [n, 2], g [n]) of the in-frame samples of one scanline."""
    cap = 2 * (L // 2) + 1
    xy = np.zeros((cap, 2), np.int32)
    g = np.zeros(cap, np.int32)
    n = lib().occl_ref_scanline_pixels(int(cx), int(cy), float(angle_deg), int(L), int(H), int(W),
                                       _p(xy, C.c_int), _p(g, C.c_int), cap)
    if n < 0:
        raise ValueError("invalid argument")
    return xy[:n], g[:n]


def scan_len(D, ratios, mode: int = 0):
    D = _f32(D)
    H, W = D.shape
    r = _f32(np.atleast_1d(ratios))
    out = np.empty(r.shape[0], np.int32)
    rc = lib().occl_ref_scan_len(_p(D, C.c_float), H, W, r.shape[0], _p(r, C.c_float), int(mode),
                                 _p(out, C.c_int))
    assert rc == 0
    return out


def detect(D, angles, ratios, scan_len, edge_thr=1.0, disp_thr=0.5, dist_thr=1.0,
           neighbours=1, want_tight=False, bilinear=False, thin=False):
    """Returns (M [V,H,W] uint8, tight or None, n_cand [V] int64).
    bilinear: the bilinear-V variant (occl_ref_detect_ex flag 1).
    thin: the candidate-thinning variant (flag 2; no tight map)."""
    D = _f32(D)
    H, W = D.shape
    a = np.ascontiguousarray(np.atleast_1d(angles), dtype=np.float64)
    r = _f32(np.atleast_1d(ratios))
    Ls = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(scan_len), a.shape), dtype=np.int32)
    V = a.shape[0]
    M = np.empty((V, H, W), np.uint8)
    T = np.empty((V, H, W), np.uint8) if want_tight else None
    nc = np.zeros(V, np.int64)
    rc = lib().occl_ref_detect_ex(_p(D, C.c_float), H, W, V, _p(a, C.c_double), _p(r, C.c_float),
                                  _p(Ls, C.c_int), float(edge_thr), float(disp_thr), float(dist_thr),
                                  int(neighbours), _p(M, C.c_ubyte), _p(T, C.c_ubyte),
                                  _p(nc, C.c_longlong), (1 if bilinear else 0) | (2 if thin else 0))
    if rc != 0:
        raise ValueError("invalid argument to occl_ref_detect")
    return M, T, nc


def detect_window(D, angles, ratios, scan_len, x0, y0, x1, y1, edge_thr=1.0, disp_thr=0.5,
                  dist_thr=1.0, neighbours=1):
    """Mask of the window [y0:y1, x0:x1] only, shape [V, y1-y0, x1-x0]."""
    D = _f32(D)
    H, W = D.shape
    a = np.ascontiguousarray(np.atleast_1d(angles), dtype=np.float64)
    r = _f32(np.atleast_1d(ratios))
    Ls = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(scan_len), a.shape), dtype=np.int32)
    Mw = np.empty((a.shape[0], y1 - y0, x1 - x0), np.uint8)
    rc = lib().occl_ref_detect_window(_p(D, C.c_float), H, W, a.shape[0], _p(a, C.c_double),
                                      _p(r, C.c_float), _p(Ls, C.c_int), float(edge_thr),
                                      float(disp_thr), float(dist_thr), int(neighbours), int(x0),
                                      int(y0), int(x1), int(y1), _p(Mw, C.c_ubyte))
    if rc != 0:
        raise ValueError("invalid argument to occl_ref_detect_window")
    return Mw


def detect_scene(sc, want_tight=False):
    p = sc.params
    return detect(sc.D, sc.angles, sc.ratios, sc.scan_len, p["edge_thr"], p["disp_thr"],
                  p["dist_thr"], p["neighbours"], want_tight=want_tight)


def confusion(pred, ref):
    pred = np.ascontiguousarray(pred, dtype=np.uint8).ravel()
    ref = np.ascontiguousarray(ref, dtype=np.uint8).ravel()
    assert pred.shape == ref.shape
    out = np.zeros(4, np.int64)
    rc = lib().occl_ref_confusion(_p(pred, C.c_ubyte), _p(ref, C.c_ubyte), pred.shape[0],
                                  _p(out, C.c_longlong))
    assert rc == 0
    return {"tp": int(out[0]), "fp": int(out[1]), "fn": int(out[2]), "tn": int(out[3])}


def zbuffer(D, angles, ratios, beta=0.5):
    """Forward-warping ground truth occlusion masks [V, H, W] (occl_ref_zbuffer)."""
    D = _f32(D)
    H, W = D.shape
    a = np.ascontiguousarray(np.atleast_1d(angles), dtype=np.float64)
    r = _f32(np.atleast_1d(ratios))
    M = np.empty((a.shape[0], H, W), np.uint8)
    rc = lib().occl_ref_zbuffer(_p(D, C.c_float), H, W, a.shape[0], _p(a, C.c_double),
                                _p(r, C.c_float), float(beta), _p(M, C.c_ubyte))
    if rc != 0:
        raise ValueError("invalid argument to occl_ref_zbuffer")
    return M


def quality(pred, ref):
    """Eq. (7): precision, recall, F1 and IoU of a predicted mask against a
    reference mask (pooled counts)."""
    c = confusion(pred, ref)
    tp, fp, fn = c["tp"], c["fp"], c["fn"]
    P = tp / (tp + fp) if tp + fp else 1.0
    R = tp / (tp + fn) if tp + fn else 1.0
    F = 2 * P * R / (P + R) if P + R else 0.0
    return {"precision": P, "recall": R, "f1": F, "iou": tp / (tp + fp + fn) if tp + fp + fn else 1.0, **c}


def median_fuse(maps):
    """Pixel-wise NaN-ignoring median of K maps [K, H, W] (occl_ref_median_fuse)."""
    maps = _f32(maps)
    K = maps.shape[0]
    out = np.empty(maps.shape[1:], np.float32)
    rc = lib().occl_ref_median_fuse(_p(maps, C.c_float), K, int(out.size), _p(out, C.c_float))
    if rc != 0:
        raise ValueError("invalid argument to occl_ref_median_fuse")
    return out


def sample(D, px, py, bilinear=True):
    """V of one scanline sample at real position (px, py) (occl_ref_sample)."""
    D = _f32(D)
    H, W = D.shape
    v = C.c_float()
    rc = lib().occl_ref_sample(_p(D, C.c_float), H, W, float(px), float(py), int(bilinear), C.byref(v))
    if rc != 0:
        raise ValueError("sample outside the frame")
    return np.float32(v.value)
