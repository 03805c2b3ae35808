"""Occlusion ground truth from every painted surface of a scene -- TEST
INFRASTRUCTURE (the reference for the limitation cases of Sec. 5; it is not
the method).

The method, like any forward warp of the centre disparity map D alone, only
sees the surfaces D holds.  The paper names three situations where the true
occlusion needs more (Sec. 5): an object that only one camera sees, objects
just outside the centre frame, and occluders that are themselves occluded in
the centre view.  Given the list of every painted surface (its pixels in
centre-view coordinates, inside or outside the frame, hidden parts
included), the true mask of view v marks a visible centre pixel p when some
surface point lands on the same nearest target pixel of view v with a
disparity larger than D(p) by more than beta.

Targets follow the rule of the D-only z-buffer of occl_ref.cpp (the reading
that p lands at p - r*D(p)*u): t = fp32(r * d), tx = rint(x - t*c),
ty = rint(y - t*s), each product and difference rounded to fp32, halves to
even; (c, s) is the octant-exact direction of the view.  With the visible
surface as the only layer this is exactly that z-buffer (pinned in
tests/test_limitations.py).
"""
from __future__ import annotations

import numpy as np

from . import occl_ref


def zbuffer_layers(D, layers, angles, ratios, beta=0.5):
    """D: visible centre map float32 [H, W]; layers: objects with int arrays
    x, y and float32 array d (centre-view coordinates, possibly outside the
    frame); returns uint8 [V, H, W]."""
    D = np.ascontiguousarray(D, dtype=np.float32)
    H, W = D.shape
    xs = np.concatenate([np.asarray(l.x, np.int64) for l in layers])
    ys = np.concatenate([np.asarray(l.y, np.int64) for l in layers])
    ds = np.concatenate([np.asarray(l.d, np.float32) for l in layers])
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.zeros((len(angles), H, W), np.uint8)
    beta = np.float32(beta)
    for v, (a, r) in enumerate(zip(angles, ratios)):
        c, s = occl_ref.direction(float(a))
        r = np.float32(r)

        def target(x, y, d):
            t = (r * d).astype(np.float32)
            tx = np.rint(x.astype(np.float32) - (t * c).astype(np.float32)).astype(np.int64)
            ty = np.rint(y.astype(np.float32) - (t * s).astype(np.float32)).astype(np.int64)
            return tx, ty

        lx, ly = target(xs, ys, ds)
        px, py = target(xx.ravel(), yy.ravel(), D.ravel())
        x0 = min(lx.min(), px.min())
        y0 = min(ly.min(), py.min())
        gw = int(max(lx.max(), px.max()) - x0 + 1)
        gh = int(max(ly.max(), py.max()) - y0 + 1)
        best = np.full(gw * gh, -np.inf, np.float32)
        np.maximum.at(best, (ly - y0) * gw + (lx - x0), ds)
        top = best[(py - y0) * gw + (px - x0)]
        out[v] = ((top - D.ravel()).astype(np.float32) > beta).reshape(H, W)
    return out
