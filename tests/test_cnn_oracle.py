"""Pins of the FP64 proposal-network oracle: a library convolution and
autograd (torch, CPU, float64), central finite differences, closed-form
loss values, and hand-built label / mask / agreement cases."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F


@pytest.fixture(scope="module")
def cnn():
    import oracle.cnn as c

    return c


@pytest.mark.parametrize("shape,stride,ci,co", [((9, 13), 2, 1, 16), ((10, 12), 2, 16, 16),
                                                ((7, 5), 1, 16, 9), ((1, 1), 2, 16, 16),
                                                ((6, 11), 1, 1, 16)])
def test_conv_matches_library(cnn, shape, stride, ci, co):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(ci,) + shape)
    w = rng.normal(size=(co, ci, 3, 3))
    b = rng.normal(size=co)
    ours = cnn.conv2d(x, w, b, stride)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b),
                   stride=stride, padding=1)[0].numpy()
    assert ours.shape == ref.shape
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-12)
    # backward against autograd
    xt = torch.from_numpy(x)[None].requires_grad_(True)
    wt = torch.from_numpy(w).requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    dout = rng.normal(size=ref.shape)
    F.conv2d(xt, wt, bt, stride=stride, padding=1).backward(torch.from_numpy(dout)[None])
    dx, dw, db = cnn.conv2d_backward(x, w, dout, stride)
    assert np.allclose(dx, xt.grad[0].numpy(), rtol=1e-11, atol=1e-11)
    assert np.allclose(dw, wt.grad.numpy(), rtol=1e-11, atol=1e-11)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_output_is_one_eighth(cnn):
    for H, W in [(1080, 1920), (720, 1280), (480, 640), (17, 33)]:
        h, w = H, W
        for _, _, s, _ in cnn.LAYERS:
            h, w = cnn.out_size(h, s), cnn.out_size(w, s)
        assert (h, w) == ((H + 7) // 8, (W + 7) // 8)


def test_bce_closed_forms(cnn):
    assert math.isclose(cnn.bce_with_logits(np.array(0.0), 1.0), math.log(2))
    z = np.linspace(-30, 30, 13)
    for y in (0.0, 1.0):
        ref = F.binary_cross_entropy_with_logits(torch.from_numpy(z), torch.full((13,), y, dtype=torch.float64),
                                                 reduction="none").numpy()
        assert np.allclose(cnn.bce_with_logits(z, y), ref, rtol=1e-12, atol=1e-12)


def _full_loss(cnn, img, params, keep, bands):
    logits, _ = cnn.forward(img, params)
    return cnn.loss_and_grad(logits, keep, bands)[0]


def test_backward_finite_differences(cnn):
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, size=(20, 28), dtype=np.uint8)
    params = cnn.init_params(3)
    params = [(w, rng.normal(scale=0.1, size=b.shape)) for w, b in params]
    th, tw = 3, 4
    keep = rng.integers(0, 2, size=(th, tw)).astype(np.uint8)
    keep[0, 0] = 1
    bands = rng.integers(0, 256, size=(th, tw)).astype(np.uint8)
    logits, acts = cnn.forward(img, params)
    assert logits.shape == (9, th, tw)
    _, g = cnn.loss_and_grad(logits, keep, bands)
    grads = cnn.backward(acts, params, g)
    eps = 1e-6
    checked = 0
    for li in range(4):
        w, b = params[li]
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(4)]:
            wp = [(ww.copy(), bb) for ww, bb in params]
            wp[li][0][idx] += eps
            wm = [(ww.copy(), bb) for ww, bb in params]
            wm[li][0][idx] -= eps
            num = (_full_loss(cnn, img, wp, keep, bands) - _full_loss(cnn, img, wm, keep, bands)) / (2 * eps)
            ana = grads[li][0][idx]
            if abs(num) > 1e-9 or abs(ana) > 1e-9:
                assert abs(num - ana) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (li, idx, num, ana)
                checked += 1
        j = int(rng.integers(0, b.shape[0]))
        bp = [(ww, bb.copy()) for ww, bb in params]
        bp[li][1][j] += eps
        bm = [(ww, bb.copy()) for ww, bb in params]
        bm[li][1][j] -= eps
        num = (_full_loss(cnn, img, bp, keep, bands) - _full_loss(cnn, img, bm, keep, bands)) / (2 * eps)
        assert abs(num - grads[li][1][j]) <= 1e-6 * max(1.0, abs(num)) + 1e-9
    assert checked >= 8


def test_loss_grad_matches_autograd(cnn):
    rng = np.random.default_rng(5)
    logits = rng.normal(size=(9, 4, 6)) * 3
    keep = rng.integers(0, 2, size=(4, 6)).astype(np.uint8)
    bands = rng.integers(0, 256, size=(4, 6)).astype(np.uint8)
    loss, g = cnn.loss_and_grad(logits, keep, bands)
    z = torch.from_numpy(logits).requires_grad_(True)
    yk = torch.from_numpy(keep.astype(np.float64))
    lt = F.binary_cross_entropy_with_logits(z[0], yk)
    npos = keep.sum()
    yb = torch.from_numpy(np.stack([(bands >> b) & 1 for b in range(8)]).astype(np.float64))
    lt = lt + (F.binary_cross_entropy_with_logits(z[1:], yb, reduction="none") * yk).sum() / (npos * 8)
    lt.backward()
    assert math.isclose(loss, lt.item(), rel_tol=1e-12)
    assert np.allclose(g, z.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_tile_labels_drawn_line(cnn, synth, oracle):
    W, H, n_theta = 64, 40, 360
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    e = np.zeros((H, W), np.uint8)
    e[:, 20] = 255          # vertical line x = 20: theta 0, r = 20
    e[5, 50] = 255          # a stray pixel far away
    t = np.array([0], np.int32)
    r = np.array([20 + D], np.int32)
    keep, bands = cnn.tile_labels(e, C, S, D, t, r, 1)
    want = np.zeros_like(keep)
    want[:, 20 // 8] = 1
    assert (keep == want).all()
    bb = oracle.band_bits(n_theta)
    assert (bands[:, 2] == bb[0]).all() and bands[:, 0].sum() == 0 and bands[0, 6] == 0


def test_mask_rule_cases(cnn):
    t = np.float32(math.log(9.0))
    z = np.zeros((9, 1, 6), np.float32)
    z[0, 0, 0] = t                     # confident keep: bands >= 0 (all zero -> all)
    z[1:, 0, 0] = -1
    z[3, 0, 0] = 0.0
    z[5, 0, 0] = 2.0
    z[0, 0, 1] = t + 1                 # keep, no band >= 0 -> first largest
    z[1:, 0, 1] = -5
    z[4, 0, 1] = -0.5
    z[6, 0, 1] = -0.5
    z[0, 0, 2] = -t                    # confident skip
    z[0, 0, 3] = np.nextafter(t, np.float32(0))  # just below: fallback
    z[0, 0, 4] = 0.0                   # unsure: fallback
    z[0, 0, 5] = -t - 3
    m = cnn.mask_from_logits(z, 0.9)
    assert m[0, 0] == (1 << 2) | (1 << 4)
    assert m[0, 1] == 1 << 3
    assert m[0, 2] == 0 and m[0, 5] == 0
    assert m[0, 3] == 0xFF and m[0, 4] == 0xFF


def test_agreement_cases(cnn):
    n, D = 360, 100
    assert cnn.agreement([10], [50], 1, [11], [51], 1, n, D) == 1.0
    assert cnn.agreement([10], [50], 1, [12], [50], 1, n, D) == 0.0
    # wrap: theta 0 vs 359 with r mirrored (2D - r)
    assert cnn.agreement([0], [120], 1, [359], [2 * D - 120], 1, n, D) == 1.0
    assert cnn.agreement([0], [120], 1, [359], [120], 1, n, D) == 0.0
    assert cnn.agreement([1, 2], [5, 9], 2, [1], [5], 1, n, D) == 0.5
