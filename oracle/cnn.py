"""FP64 CPU oracle for the learned tile/theta-band proposal -- TEST
INFRASTRUCTURE ONLY (tests, smoke, benchmark baseline).

The paper has no learned component; the network, labels, mask rule and
agreement metric are the task's additions and are specified here:

  network  four 3x3 convolutions with zero padding 1:
             conv1  1 -> 16, stride 2, ReLU
             conv2 16 -> 16, stride 2, ReLU
             conv3 16 -> 16, stride 2, ReLU
             head  16 ->  9, stride 1        (logits at 1/8 resolution)
           input: gray / 255.  Output channel 0 = keep logit of the 8x8 tile,
           channels 1..8 = logits of the 8 theta bands.
  loss     mean over tiles of BCE(keep) + mean over keep-labelled tiles of
           the mean over bands of BCE(band)
  labels   from the plain Hough pipeline: a tile is "keep" iff it holds an
           edge pixel whose r for the angle of one of the top-k peaks lies
           within 1 of that peak's r; its band label is the union of the
           bands of those peaks
  mask     per tile, from float32 logits: keep >= t_hi -> the bands with
           logit >= 0 (at least the largest); keep <= -t_hi -> nothing;
           otherwise every band (fallback to the full Hough).  t_hi =
           float32(log(c / (1 - c))), c = float32(conf).
  agreement  fraction of plain top-k peaks with a pruned top-k peak within
           +-1 theta bin and +-1 r bin (theta wrapping, r mirrored per half
           turn, as in the peak suppression)

Everything is written as plain loops over kernel taps with numpy
vectorisation over pixels only.
"""
from __future__ import annotations

import math

import numpy as np

# (c_in, c_out, stride, relu)
LAYERS = ((1, 16, 2, True), (16, 16, 2, True), (16, 16, 2, True), (16, 9, 1, False))


def param_shapes():
    return [((co, ci, 3, 3), (co,)) for ci, co, _, _ in LAYERS]


def n_params() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def init_params(seed: int = 0):
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    ps = []
    for (wshape, bshape) in param_shapes():
        fan_in = wshape[1] * 9
        lim = math.sqrt(6.0 / fan_in)
        ps.append((rng.uniform(-lim, lim, size=wshape), np.zeros(bshape)))
    return ps


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(vec: np.ndarray):
    out, o = [], 0
    for wshape, bshape in param_shapes():
        nw, nb = int(np.prod(wshape)), int(np.prod(bshape))
        out.append((vec[o:o + nw].reshape(wshape).astype(np.float64),
                    vec[o + nw:o + nw + nb].astype(np.float64)))
        o += nw + nb
    return out


def out_size(n: int, stride: int) -> int:
    return (n + 2 - 3) // stride + 1


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """x [C_in][H][W] -> [C_out][Ho][Wo]; cross-correlation, zero pad 1:
    out[o][y][x] = b[o] + sum_{c,ky,kx} w[o][c][ky][kx] * x[c][s*y+ky-1][s*x+kx-1]."""
    ci, H, W = x.shape
    co = w.shape[0]
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((ci, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.zeros((co, Ho, Wo)) + b[:, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += np.tensordot(w[:, :, ky, kx], patch, axes=([1], [0]))
    return out


def conv2d_backward(x, w, dout, stride):
    """Gradients of conv2d w.r.t. x, w, b given dL/dout."""
    ci, H, W = x.shape
    co, Ho, Wo = dout.shape
    xp = np.zeros((ci, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dw[:, :, ky, kx] = np.tensordot(dout, xp[sl], axes=([1, 2], [1, 2]))
            dxp[sl] += np.tensordot(w[:, :, ky, kx], dout, axes=([0], [0]))
    db = dout.sum(axis=(1, 2))
    return dxp[:, 1:H + 1, 1:W + 1], dw, db


def forward(img_u8: np.ndarray, params):
    """Returns (logits [9][th][tw], cache for backward)."""
    x = img_u8.astype(np.float64)[None] / 255.0
    acts = [x]
    for (w, b), (_, _, s, relu) in zip(params, LAYERS):
        y = conv2d(acts[-1], w, b, s)
        if relu:
            y = np.maximum(y, 0.0)
        acts.append(y)
    return acts[-1], acts


def backward(acts, params, dlogits):
    """Analytic backward through the four layers; returns [(dw, db)]."""
    grads = [None] * len(LAYERS)
    d = dlogits
    for li in range(len(LAYERS) - 1, -1, -1):
        w, _ = params[li]
        _, _, s, relu = LAYERS[li]
        if relu:
            d = d * (acts[li + 1] > 0)
        dx, dw, db = conv2d_backward(acts[li], w, d, s)
        grads[li] = (dw, db)
        d = dx
    return grads


def bce_with_logits(z, y):
    return np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss_and_grad(logits, keep, bands):
    """logits [9][th][tw]; keep [th][tw] in {0,1}; bands [th][tw] uint8 bits.
    Returns (loss, dL/dlogits)."""
    n = keep.size
    zk = logits[0]
    yk = keep.astype(np.float64)
    loss = bce_with_logits(zk, yk).mean()
    g = np.zeros_like(logits)
    g[0] = (sigmoid(zk) - yk) / n
    npos = int(keep.sum())
    if npos:
        for b in range(8):
            yb = ((bands >> b) & 1).astype(np.float64)
            zb = logits[1 + b]
            loss += (bce_with_logits(zb, yb) * yk).sum() / (npos * 8)
            g[1 + b] = (sigmoid(zb) - yb) * yk / (npos * 8)
    return loss, g


def tile_labels(edges: np.ndarray, C, S, D: int, theta_idx, r_idx, count: int):
    """keep / band labels per 8x8 tile from the plain top-k peaks."""
    from oracle import band_bits

    H, W = edges.shape
    th, tw = (H + 7) // 8, (W + 7) // 8
    keep = np.zeros((th, tw), np.uint8)
    bands = np.zeros((th, tw), np.uint8)
    bb = band_bits(len(C))
    ys, xs = np.nonzero(edges == 255)
    for p in range(count):
        t, rp = int(theta_idx[p]), int(r_idx[p]) - D
        v = xs.astype(np.int64) * int(C[t]) + ys.astype(np.int64) * int(S[t])
        r = np.floor_divide(v + 8192, 16384)
        hit = np.abs(r - rp) <= 1
        ty, tx = ys[hit] // 8, xs[hit] // 8
        keep[ty, tx] = 1
        bands[ty, tx] |= bb[t]
    return keep, bands


def mask_from_logits(logits32: np.ndarray, conf: float = 0.9) -> np.ndarray:
    """Decision rule on float32 logits (the GPU compares the same float32
    values against the same float32 threshold)."""
    z = logits32.astype(np.float32)
    c = float(np.float32(conf))  # the confidence as the float32 the GPU call receives
    t_hi = np.float32(math.log(c / (1.0 - c)))
    _, th, tw = z.shape
    m = np.zeros((th, tw), np.uint8)
    for y in range(th):
        for x in range(tw):
            k = z[0, y, x]
            if k >= t_hi:
                bz = z[1:, y, x]
                bits = 0
                for b in range(8):
                    if bz[b] >= np.float32(0.0):
                        bits |= 1 << b
                if bits == 0:
                    bits = 1 << int(np.argmax(bz))  # first largest
                m[y, x] = bits
            elif k <= -t_hi:
                m[y, x] = 0
            else:
                m[y, x] = 0xFF
    return m


def same_line(t1, r1, t2, r2, n_theta: int, D: int, tol: int = 1) -> bool:
    """(t1, r1) within +-tol bins of (t2, r2), theta wrapping with r mirrored."""
    for q in (-1, 0, 1):
        tt = t2 + q * n_theta
        rr = (2 * D - r2) if q % 2 else r2
        if abs(tt - t1) <= tol and abs(rr - r1) <= tol:
            return True
    return False


def agreement(plain_t, plain_r, plain_n, pr_t, pr_r, pr_n, n_theta: int, D: int) -> float:
    if plain_n == 0:
        return 1.0
    hit = 0
    for i in range(plain_n):
        if any(same_line(int(plain_t[i]), int(plain_r[i]), int(pr_t[j]), int(pr_r[j]), n_theta, D)
               for j in range(pr_n)):
            hit += 1
    return hit / plain_n
