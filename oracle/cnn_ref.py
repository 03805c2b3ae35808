"""CPU oracle of the learned tile proposal's network -- TEST INFRASTRUCTURE.

Plain numpy, fp64 arithmetic on bf16-rounded operands, written from the
textbook definitions of the operations (only the tests and the benchmark's
checks use it; the GPU library never calls it):

* 3x3 convolution, zero padding 1, stride s:
    y[n, oy, ox, co] = b[co] + sum_{ky, kx, ci} x[n, oy*s + ky - 1, ox*s + kx - 1, ci] * w[co, ky, kx, ci]
  (NHWC activations, weights [Cout][3][3][Cin]); output size ceil(H / s).
* its gradients with respect to x, w and b (the adjoint of the sum above);
* ReLU, the logistic function and the binary cross-entropy with a soft
  target t in [0, 1]:  loss(z, t) = softplus(z) - t * z, d loss / dz = sigmoid(z) - t;
* Adam (Kingma & Ba 2015) with bias correction;
* the network: 6 layers (8->32 s2, 32->32 s2, 32->32 s2, 32->32 s2,
  32->32 s1, 32->1 s1), ReLU after all but the last; activations and
  activation gradients are rounded to bf16 between layers, logits and their
  gradient stay fp32 -- the same storage precisions as the GPU kernels;
* tile routing: a tile whose occlusion probability sigmoid(z) lies below the
  band [lo, hi] is filled with 0, above it with 1, and otherwise takes the
  exact path (a NaN logit too).
"""
from __future__ import annotations

import numpy as np

LAYERS = [(8, 32, 2, True), (32, 32, 2, True), (32, 32, 2, True), (32, 32, 2, True),
          (32, 32, 1, True), (32, 1, 1, False)]
TILE = 16
IN_CH = 8


def n_params():
    return sum(co * 9 * ci + co for ci, co, _, _ in LAYERS)


def bf16(x):
    """Round to the nearest bf16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = r.astype(np.uint32)
    nan = np.isnan(a)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def out_size(n, stride):
    return (n + stride - 1) // stride


def conv3x3(x, w, b, stride):
    """x [N,H,W,Cin], w [Cout,3,3,Cin], b [Cout] -> y [N,Ho,Wo,Cout] (fp64)."""
    N, H, W, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    y = np.zeros((N, Ho, Wo, Co)) + b.reshape(1, 1, 1, Co)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            y += np.tensordot(patch, w[:, ky, kx, :], axes=([3], [1]))
    return y


def conv3x3_backward(x, w, gy, stride):
    """Gradients of sum(gy * conv3x3(x, w, b)) w.r.t. x, w, b."""
    N, H, W, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = gy.shape[1], gy.shape[2]
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride), slice(None))
            patch = xp[sl]
            gw[:, ky, kx, :] = np.tensordot(gy, patch, axes=([0, 1, 2], [0, 1, 2]))
            gxp[sl] += np.tensordot(gy, w[:, ky, kx, :], axes=([3], [0]))
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:H + 1, 1:W + 1, :], gw, gb


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def bce(z, t):
    """Mean soft binary cross-entropy and its gradient w.r.t. the logits."""
    loss = np.logaddexp(0.0, z) - t * z
    return float(loss.mean()), (sigmoid(z) - t) / z.size


def unflatten(theta):
    """Flat parameter vector (layer order, weights then bias) -> [(w, b)]."""
    out, k = [], 0
    for ci, co, _, _ in LAYERS:
        nw = co * 9 * ci
        w = np.asarray(theta[k:k + nw], dtype=np.float64).reshape(co, 3, 3, ci)
        k += nw
        b = np.asarray(theta[k:k + co], dtype=np.float64)
        k += co
        out.append((w, b))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def forward(theta, x, round_bf16=True):
    """Logits [N, Ht, Wt] (fp64) and the per-layer activations.  Weights and
    activations are bf16-rounded as on the GPU; biases and logits are not."""
    params = unflatten(theta)
    acts = [bf16(x) if round_bf16 else np.asarray(x, np.float64)]
    for li, ((w, b), (_, _, s, relu)) in enumerate(zip(params, LAYERS)):
        wq = bf16(w) if round_bf16 else w
        y = conv3x3(acts[-1], wq, b, s)
        if relu:
            y = np.maximum(y, 0.0)
            y = bf16(y) if round_bf16 else y
        acts.append(y)
    return acts[-1][..., 0], acts


def backward(theta, x, t, round_bf16=True):
    """Loss and the flat gradient of the mean BCE loss w.r.t. theta, with the
    activation gradients rounded to bf16 between layers (as on the GPU)."""
    params = unflatten(theta)
    z, acts = forward(theta, x, round_bf16)
    loss, gz = bce(z, t)
    g = gz[..., None]
    grads = [None] * len(LAYERS)
    for li in range(len(LAYERS) - 1, -1, -1):
        w, _ = params[li]
        wq = bf16(w) if round_bf16 else w
        _, _, s, relu = LAYERS[li]
        if relu:
            g = g * (acts[li + 1] > 0)
        gx, gw, gb = conv3x3_backward(acts[li], wq, g, s)
        grads[li] = (gw, gb)
        g = bf16(gx) if round_bf16 else gx
    return loss, flatten(grads)


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def pack(D, c, s, ratio, L):
    """Input channels of one view: D*r/L, E/8, cos A, sin A, cos alpha,
    sin alpha, r/2, 0 (A = atan2(E_y, E_x); E, E_x, E_y of Eq. (1);
    (c, s) = (cos alpha, sin alpha), the view's direction vector) -> bf16."""
    D = np.asarray(D, np.float64)
    H, W = D.shape
    ex = np.zeros_like(D)
    ey = np.zeros_like(D)
    ex[:, :-1] = D[:, 1:] - D[:, :-1]
    ey[:-1, :] = D[1:, :] - D[:-1, :]
    E = np.sqrt(ex * ex + ey * ey)
    # cos A and sin A of A = atan2(E_y, E_x), written as E_x / E and E_y / E
    # (A = 0 where E = 0, as atan2(0, 0) = 0)
    safe = np.where(E > 0, E, 1.0)
    cosA = np.where(E > 0, ex / safe, 1.0)
    sinA = np.where(E > 0, ey / safe, 0.0)
    x = np.zeros((H, W, IN_CH))
    x[..., 0] = D * (ratio / L)
    x[..., 1] = E / 8.0
    x[..., 2] = cosA
    x[..., 3] = sinA
    x[..., 4] = c
    x[..., 5] = s
    x[..., 6] = ratio / 2.0
    return bf16(x)


def tile_fraction(M, tile=TILE):
    """Occluded fraction of every tile x tile block (edge tiles partial)."""
    M = np.asarray(M, np.float64)
    H, W = M.shape[-2:]
    Ht, Wt = out_size(H, tile), out_size(W, tile)
    out = np.zeros(M.shape[:-2] + (Ht, Wt))
    for ty in range(Ht):
        for tx in range(Wt):
            blk = M[..., ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile]
            out[..., ty, tx] = blk.mean(axis=(-2, -1))
    return out


def logit_bound(p):
    """The logit of a probability bound, evaluated in double and rounded to
    fp32 (p <= 0 -> -inf, p >= 1 -> +inf): sigmoid(z) < p  <=>  z < logit(p)
    since the logistic function is strictly increasing."""
    if p <= 0:
        return np.float32(-np.inf)
    if p >= 1:
        return np.float32(np.inf)
    return np.float32(np.log(p / (1.0 - p)))


def tile_states(z, lo, hi):
    """Routing state of every tile from its logit z (fp32): 0 (fill 0) if
    z < logit(lo), 1 (fill 1) if z > logit(hi), else 2 (exact path); a NaN
    logit compares false both ways and takes the exact path."""
    z = np.asarray(z, np.float32)
    zl, zh = logit_bound(lo), logit_bound(hi)
    s = np.full(z.shape, 2, np.uint8)
    s[z < zl] = 0
    s[z > zh] = 1
    return s

