"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test names the passage of the paper it follows.  None of them re-types
the oracle's own formula as the expectation: they use closed forms of the
Sobel operator (Sec. 2.1 Eq. 1), invariants of the vote (Sec. 2.3 Eq. 3),
the real-valued line equation with its Q14 error bound, a library
correlation, and brute force on tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

# Sobel kernels written out (Sec. 2.1; coefficients only take the forms
# 0, 1 and 2 per Sec. 3.1).  Correlation (not convolution) orientation; the
# absolute values in Eq. (1) make the orientation irrelevant.
KX = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], np.int64)
KY = KX.T.copy()


def lib_sobel(img):
    a = img.astype(np.int64)
    gx = ndimage.correlate(a, KX, mode="constant", cval=0)
    gy = ndimage.correlate(a, KY, mode="constant", cval=0)
    return np.abs(gx) + np.abs(gy)


# ------------------------------------------------------------ Sobel (P1-P4)

@pytest.mark.parametrize("c", [0, 1, 7, 40, 63, 64, 90, 200, 255])
def test_constant_image_closed_form(oracle, c):
    H, W = 9, 13
    img = np.full((H, W), c, np.uint8)
    edges, mag, n = oracle.sobel_binarize(img, threshold=128, border_mode=0)
    # interior gradient is zero
    assert (mag[1:-1, 1:-1] == 0).all()
    # zero padding: sides see 4c, corners 6c (gx = gy = 3c)
    side = min(4 * c, 255)
    corner = min(6 * c, 255)
    assert (mag[0, 1:-1] == side).all() and (mag[-1, 1:-1] == side).all()
    assert (mag[1:-1, 0] == side).all() and (mag[1:-1, -1] == side).all()
    for y, x in [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1)]:
        assert mag[y, x] == corner
    assert (edges[1:-1, 1:-1] == 0).all()
    assert (edges[0, 1:-1] == (255 if 4 * c > 128 else 0)).all()
    # mode 1 forces the ring to non-edge but keeps the magnitude
    e1, m1, n1 = oracle.sobel_binarize(img, threshold=128, border_mode=1)
    assert n1 == 0 and (e1 == 0).all() and (m1 == mag).all()


@pytest.mark.parametrize("a,b,c0", [(1, 0, 3), (0, 2, 5), (3, 4, 0), (-2, 1, 120), (5, -3, 150)])
def test_linear_ramp_closed_form(oracle, a, b, c0):
    H, W = 12, 15
    y, x = np.mgrid[0:H, 0:W]
    v = a * x + b * y + c0
    assert v.min() >= 0 and v.max() <= 255
    img = v.astype(np.uint8)
    _, mag, _ = oracle.sobel_binarize(img, threshold=255, border_mode=0)
    assert (mag[1:-1, 1:-1] == min(8 * (abs(a) + abs(b)), 255)).all()


@pytest.mark.parametrize("h", [1, 10, 31, 32, 33, 60])
def test_vertical_step(oracle, h):
    H, W, x0 = 10, 16, 7
    img = np.full((H, W), 50, np.uint8)
    img[:, x0:] += h
    edges, mag, _ = oracle.sobel_binarize(img, threshold=128, border_mode=1)
    g = np.zeros((H, W), np.int64)
    g[:, x0 - 1] = 4 * h
    g[:, x0] = 4 * h
    assert (mag[1:-1, 1:-1] == np.minimum(g, 255)[1:-1, 1:-1]).all()
    # threshold is strict: 4*32 = 128 is not an edge, 4*33 = 132 is
    want = 255 if 4 * h > 128 else 0
    assert (edges[1:-1, x0 - 1] == want).all() and (edges[1:-1, x0] == want).all()
    others = np.delete(edges[1:-1, 1:-1], [x0 - 2, x0 - 1], axis=1)
    assert (others == 0).all()


def test_step_threshold_boundary(oracle):
    img = np.zeros((5, 6), np.uint8)
    img[:, 3:] = 32
    e, _, _ = oracle.sobel_binarize(img, threshold=128, border_mode=1)
    assert (e == 0).all()
    img[:, 3:] = 33
    e, _, _ = oracle.sobel_binarize(img, threshold=128, border_mode=1)
    assert (e[1:-1, 2:4] == 255).all()


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (3, 3), (8, 8), (13, 29), (32, 32)])
@pytest.mark.parametrize("seed", [0, 1])
def test_sobel_vs_library_correlation(oracle, shape, seed):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=shape, dtype=np.uint8)
    g = lib_sobel(img)
    for T in (0, 100, 128, 254):
        for mode in (0, 1):
            e, m, n = oracle.sobel_binarize(img, threshold=T, border_mode=mode)
            want_e = np.where(g > T, 255, 0)
            if mode == 1:
                want_e[0, :] = 0
                want_e[-1, :] = 0
                want_e[:, 0] = 0
                want_e[:, -1] = 0
            assert (m == np.minimum(g, 255)).all()
            assert (e == want_e).all()
            assert n == int((want_e == 255).sum())


def test_sobel_pitch(oracle):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(11, 20), dtype=np.uint8)
    e0, m0, _ = oracle.sobel_binarize(img[:, :17].copy(), threshold=128)
    e1, m1, _ = oracle.sobel_binarize(img, W=17, threshold=128)
    assert (e0 == e1).all() and (m0 == m1).all()


# ------------------------------------------------------------ vote (P5-P9)

def test_trig_table_spot_values(synth):
    c, s = synth.trig_q14(180)
    assert c[0] == 16384 and s[0] == 0          # theta = 0
    assert c[90] == 0 and s[90] == 16384        # theta = 90 deg
    assert c[60] == 8192 and s[30] == 8192      # cos 60 = sin 30 = 1/2
    assert c[45] == 11585 and s[45] == 11585    # 2^14/sqrt(2) = 11585.24
    assert c[135] == -11585 and s[135] == 11585
    # symmetry of Eq. (4)-(5): sin(180-t) = sin t, cos(180-t) = -cos t
    for k in range(1, 180):
        assert s[180 - k] == s[k] and c[180 - k] == -c[k]


def _single_point(W, H, x, y):
    e = np.zeros((H, W), np.uint8)
    e[y, x] = 255
    return e


@pytest.mark.parametrize("n_theta", [4, 180, 360])
@pytest.mark.parametrize("pt", [(0, 0), (5, 3), (39, 29), (17, 0), (0, 22)])
def test_one_point_one_vote_per_theta(oracle, synth, n_theta, pt):
    W, H = 40, 30
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, cast, dropped = oracle.hough_vote(_single_point(W, H, *pt), C, S, D, 2 * D + 1)
    assert dropped == 0 and cast == n_theta
    assert (acc.sum(axis=1) == 1).all()
    x, y = pt
    # theta = 0 gives r = x, theta = 90 deg gives r = y (Eq. 3 exactly)
    assert acc[0, x + D] == 1
    if n_theta % 2 == 0:
        assert acc[n_theta // 2, y + D] == 1
    # every vote lies within the Q14 error bound of the real-valued Eq. (3)
    ks, ii = np.nonzero(acc)
    th = ks * math.pi / n_theta
    r_true = x * np.cos(th) + y * np.sin(th)
    assert (np.abs((ii - D) - r_true) <= 0.5 + (x + y) / 2 ** 15 + 1e-9).all()


def test_total_votes_invariant(oracle, synth):
    rng = np.random.default_rng(11)
    W, H = 53, 37
    e = np.where(rng.random((H, W)) < 0.2, 255, 0).astype(np.uint8)
    n_e = int((e == 255).sum())
    for n_theta in (180, 360, 7):
        C, S = synth.trig_q14(n_theta)
        D = synth.r_offset(W, H)
        acc, cast, dropped = oracle.hough_vote(e, C, S, D, 2 * D + 1)
        assert dropped == 0
        assert acc.sum() + dropped == n_e * n_theta
        assert (acc.sum(axis=1) == n_e).all()


def test_dropped_counted_when_range_too_small(oracle, synth):
    rng = np.random.default_rng(5)
    W, H = 30, 20
    e = np.where(rng.random((H, W)) < 0.3, 255, 0).astype(np.uint8)
    n_e = int((e == 255).sum())
    C, S = synth.trig_q14(90)
    acc, cast, dropped = oracle.hough_vote(e, C, S, 3, 11)
    assert dropped > 0 and acc.sum() == cast and cast + dropped == n_e * 90


def test_extremes_at_corners(oracle, synth):
    """r is monotone in x and y, so per theta the extreme r of a full frame
    is reached at one of the four corners."""
    W, H = 31, 17
    e = np.full((H, W), 255, np.uint8)
    C, S = synth.trig_q14(180)
    D = synth.r_offset(W, H)
    acc, _, dropped = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    assert dropped == 0
    corners = np.zeros((H, W), np.uint8)
    for (x, y) in [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1)]:
        corners[y, x] = 255
    accc, _, _ = oracle.hough_vote(corners, C, S, D, 2 * D + 1)
    for k in range(180):
        nz = np.nonzero(acc[k])[0]
        nzc = np.nonzero(accc[k])[0]
        assert nz.min() == nzc.min() and nz.max() == nzc.max()


@pytest.mark.parametrize("k0,r0", [(0, 20), (30, 25), (45, 60), (90, 12), (120, 5), (150, -8),
                                   (179, -3), (100, 40), (60, 90)])
def test_drawn_line_peaks_at_its_own_bin(oracle, synth, k0, r0):
    """Mark the pixels on the real line x cos t + y sin t = r0 (within 0.3 px;
    the Q14 error is far below the remaining 0.2 px), vote, and the cell
    (k0, r0) must count every marked pixel and be the strict maximum (the
    frame is large enough that no neighbouring bin holds the whole line)."""
    W, H, n_theta = 220, 160, 180
    th = k0 * math.pi / n_theta
    y, x = np.mgrid[0:H, 0:W]
    on = np.abs(x * math.cos(th) + y * math.sin(th) - r0) < 0.3
    if on.sum() < 8:
        pytest.skip("line too short in this frame")
    e = np.where(on, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, _, dropped = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    assert dropped == 0
    assert acc[k0, r0 + D] == on.sum()
    flat = acc.ravel()
    assert flat.max() == on.sum()
    assert (flat == flat.max()).sum() == 1
    t, r, v, n = oracle.hough_peaks(acc, D, 1)
    assert n == 1 and t[0] == k0 and r[0] == r0 + D and v[0] == on.sum()


def test_band_bits_cover_each_theta_twice(oracle):
    for n in (8, 180, 360):
        bb = oracle.band_bits(n)
        assert all(bin(int(b)).count("1") == 2 for b in bb)
    bb = oracle.band_bits(360)
    # band b = [45b, 45b+90) mod 360 for 360 bins
    for b in range(8):
        ks = [k for k in range(360) if bb[k] >> b & 1]
        assert len(ks) == 90
        assert set(ks) == {(45 * b + j) % 360 for j in range(90)}


def test_mask_all_ones_zero_and_subset(oracle, synth):
    rng = np.random.default_rng(2)
    W, H = 45, 27
    e = np.where(rng.random((H, W)) < 0.25, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(180)
    D = synth.r_offset(W, H)
    plain, cast, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    th, tw = (H + 7) // 8, (W + 7) // 8
    full = np.full((th, tw), 0xFF, np.uint8)
    a1, c1, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1, full)
    assert (a1 == plain).all() and c1 == cast
    zero = np.zeros((th, tw), np.uint8)
    a0, c0, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1, zero)
    assert a0.sum() == 0 and c0 == 0
    m = rng.integers(0, 256, size=(th, tw), dtype=np.uint8)
    am, cm, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1, m)
    assert (am <= plain).all()
    # brute-force count of the pruned votes from the band definition
    bb = oracle.band_bits(180)
    ys, xs = np.nonzero(e == 255)
    want = sum(int(((m[y // 8, x // 8] & bb) != 0).sum()) for y, x in zip(ys, xs))
    assert cm == want


def test_vote_vs_brute_force_histogram(oracle, synth):
    """Independent formulation: for every theta, a histogram (np.bincount) of
    the rounded r of all edge pixels, with r rounded by real division."""
    rng = np.random.default_rng(9)
    W, H = 33, 21
    e = np.where(rng.random((H, W)) < 0.3, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(60)
    D = synth.r_offset(W, H)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    ys, xs = np.nonzero(e == 255)
    for k in range(60):
        v = xs.astype(np.int64) * int(C[k]) + ys.astype(np.int64) * int(S[k])
        r = np.array([math.floor(val / 16384 + 0.5) for val in v.tolist()])
        hist = np.bincount(r + D, minlength=2 * D + 1)
        assert (hist == acc[k]).all()


# ------------------------------------------------------------ peaks (P10)

def _brute_peaks(acc, D, k, ht, hr, min_votes=1):
    """Greedy NMS stated on lines rather than rows/columns: cell (t, i) is the
    line (theta_t, r = i - D), and (t + n, i) is the same line as
    (t, 2D - i) because (r, theta + 180) == (-r, theta).  A cell is
    suppressed if some selected line lies within the window after unfolding
    theta by any whole number of half turns."""
    n_theta, n_r = acc.shape
    sel = []
    alive = np.ones_like(acc, dtype=bool)
    out = []
    for _ in range(k):
        best = None
        for t in range(n_theta):
            for i in range(n_r):
                if alive[t, i] and (best is None or acc[t, i] > acc[best]):
                    best = (t, i)
        if best is None or acc[best] < max(1, min_votes):
            break
        out.append((best[0], best[1], int(acc[best])))
        sel.append(best)
        t0, i0 = best
        for t in range(n_theta):
            for i in range(n_r):
                for q in range(-3, 4):
                    tt = t + q * n_theta
                    ii = (2 * D - i) if q % 2 else i
                    if abs(tt - t0) <= ht and abs(ii - i0) <= hr:
                        alive[t, i] = False
    return out


@pytest.mark.parametrize("seed", range(6))
def test_peaks_vs_brute_force(oracle, seed):
    rng = np.random.default_rng(seed)
    n_theta, D = int(rng.integers(3, 9)), int(rng.integers(2, 6))
    n_r = 2 * D + 1
    acc = rng.integers(0, 6, size=(n_theta, n_r)).astype(np.int32)
    for k in (1, 3, 6):
        for ht, hr in ((0, 0), (1, 1), (2, 1), (1, 3)):
            t, r, v, n = oracle.hough_peaks(acc, D, k, ht, hr)
            want = _brute_peaks(acc, D, k, ht, hr)
            assert n == len(want)
            got = [(int(t[j]), int(r[j]), int(v[j])) for j in range(n)]
            assert got == want
            assert (t[n:] == -1).all() and (r[n:] == -1).all() and (v[n:] == -1).all()


def test_peaks_tie_and_wrap_cases(oracle):
    D = 3
    acc = np.zeros((5, 7), np.int32)
    # two equal maxima: the smaller theta-major index wins
    acc[1, 2] = 9
    acc[3, 5] = 9
    t, r, v, n = oracle.hough_peaks(acc, D, 1, 0, 0)
    assert (t[0], r[0], v[0]) == (1, 2, 9)
    # wrap: a peak in the last row suppresses mirrored columns of row 0
    acc = np.zeros((5, 7), np.int32)
    acc[4, 1] = 10
    acc[0, 5] = 8      # mirror of column 1 is 2*3 - 1 = 5 -> suppressed
    acc[0, 1] = 7      # same column, not mirrored -> survives
    t, r, v, n = oracle.hough_peaks(acc, D, 3, 1, 0)
    assert n == 2
    assert (t[0], r[0]) == (4, 1) and (t[1], r[1], v[1]) == (0, 1, 7)
    # min_votes stops early
    t, r, v, n = oracle.hough_peaks(acc, D, 3, 0, 0, min_votes=9)
    assert n == 1 and t[1] == -1
    # all-zero accumulator: no peaks
    t, r, v, n = oracle.hough_peaks(np.zeros((4, 7), np.int32), D, 2)
    assert n == 0 and (t == -1).all()


def test_r_offset_matches_integer_sqrt(oracle, synth):
    for W, H in [(1, 1), (2, 1), (640, 480), (1920, 1080), (3840, 2160), (1280, 720), (8192, 8192)]:
        assert oracle.r_offset(W, H) == synth.r_offset(W, H)
        d = oracle.r_offset(W, H)
        q = (W - 1) ** 2 + (H - 1) ** 2
        assert d * d >= q and (d - 1) * (d - 1) < q or q == 0


# ------------------------------------------------- line segments (Sec. 1 step 4, Sec. 5)
# Drawn segments with known end points: the expected output is the drawing,
# not a re-typed formula.

def _trig(n_theta):
    from paper_2212_09460_amd import synth as s

    return s.trig_q14(n_theta)


def _lines(oracle, e, n_theta, t, r, **kw):
    C, S = _trig(n_theta)
    H, W = e.shape
    D = oracle.r_offset(W, H)
    segs, counts, npts = oracle.hough_lines(e, C, S, D, np.array([t], np.int32),
                                            np.array([r + D], np.int32), **kw)
    got = [tuple(int(v) for v in segs[0, s]) for s in range(min(int(counts[0]), segs.shape[1]))]
    return got, int(counts[0]), int(npts[0])


def test_lines_horizontal_and_vertical_runs(oracle):
    e = np.zeros((48, 64), np.uint8)
    e[17, 5:51] = 255          # row 17, x = 5..50
    e[3:40, 33] = 255          # column 33, y = 3..39 (crosses the row)
    # theta = 90 deg (bin 90 of 180): r = y; the row plus the column's pixel on it
    got, n, npts = _lines(oracle, e, 180, 90, 17, fill_gap=20, min_length=10)
    assert got == [(5, 17, 50, 17)] and n == 1 and npts == 46
    # theta = 0: r = x; ordered by y
    got, n, npts = _lines(oracle, e, 180, 0, 33, fill_gap=20, min_length=10)
    assert got == [(33, 3, 33, 39)] and npts == 37


def test_lines_gap_fill_and_min_length(oracle):
    e = np.zeros((32, 96), np.uint8)
    e[10, 2:21] = 255          # x = 2..20
    e[10, 31:61] = 255         # x = 31..60: gap of 11 between 20 and 31
    e[10, 80:84] = 255         # x = 80..83: a 3-px piece 20 away from 60
    got, n, _ = _lines(oracle, e, 180, 90, 10, fill_gap=20, min_length=10)
    assert got == [(2, 10, 83, 10)]                           # every gap <= 20 joins
    got, n, _ = _lines(oracle, e, 180, 90, 10, fill_gap=10, min_length=10)
    assert got == [(2, 10, 20, 10), (31, 10, 60, 10)] and n == 2   # the 3-px piece is dropped
    got, n, _ = _lines(oracle, e, 180, 90, 10, fill_gap=10, min_length=3)
    assert got == [(2, 10, 20, 10), (31, 10, 60, 10), (80, 10, 83, 10)]
    got, n, _ = _lines(oracle, e, 180, 90, 10, fill_gap=10, min_length=3, max_seg=2)
    assert got == [(2, 10, 20, 10), (31, 10, 60, 10)] and n == 3   # count beyond the slots


def test_lines_diagonal_and_off_line_pixels(oracle):
    e = np.zeros((64, 64), np.uint8)
    for x in range(10, 41):
        e[x, x] = 255          # y = x
    e[30, 20] = 255            # 10 px off the line
    e[25, 27] = 255            # distance 2/sqrt(2) off the line
    # theta = 135 deg: x cos + y sin = (y - x)/sqrt(2) = 0 on the diagonal
    got, n, npts = _lines(oracle, e, 180, 135, 0, fill_gap=5, min_length=5)
    assert got == [(10, 10, 40, 40)] and npts == 31
    assert _lines(oracle, e, 180, 135, 7, fill_gap=5, min_length=0)[2] == 1   # (20, 30): r = 10/sqrt(2)


def test_lines_points_are_the_peak_voters(oracle):
    rng = np.random.default_rng(5)
    e = np.where(rng.random((40, 56)) < 0.2, 255, 0).astype(np.uint8)
    n_theta = 64
    C, S = _trig(n_theta)
    D = oracle.r_offset(56, 40)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    t = np.repeat(np.arange(n_theta, dtype=np.int32), 3)
    r = np.array([D, D + 7, D - 11] * n_theta, np.int32)
    _, counts, npts = oracle.hough_lines(e, C, S, D, t, r, fill_gap=1000, min_length=0)
    assert (npts == acc[t, r]).all()                  # exactly the cell's voters
    assert (counts == (npts > 0)).all()               # one segment when no gap splits


def test_lines_padding_peak_is_empty(oracle):
    e = np.full((8, 8), 255, np.uint8)
    C, S = _trig(16)
    segs, counts, npts = oracle.hough_lines(e, C, S, oracle.r_offset(8, 8), np.array([-1], np.int32),
                                            np.array([-1], np.int32))
    assert counts[0] == 0 and npts[0] == 0 and (segs == -1).all()


# --------------------------------------------------------------- Canny (Sec. 7)
# The detector the paper proposes instead of Sobel + binarization.  Pinned by
# library routines (blur and gradient by scipy correlation, the hysteresis by
# scipy connected-component labelling) and by drawn steps whose thinned edge
# is known.

W5 = np.array([1, 4, 6, 4, 1], np.int64)


def lib_canny_mag(img):
    a = img.astype(np.int64)
    b = (ndimage.correlate(a, np.outer(W5, W5), mode="nearest") + 128) >> 8
    gx = ndimage.correlate(b, KX, mode="nearest")
    gy = ndimage.correlate(b, KY, mode="nearest")
    return np.abs(gx) + np.abs(gy)


@pytest.mark.parametrize("seed", range(4))
def test_canny_gradient_matches_library(oracle, seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    _, mag, _ = oracle.canny(img, t_low=50, t_high=100)
    assert (mag == np.minimum(lib_canny_mag(img), 255)).all()


def test_canny_constant_and_steps(oracle):
    H, W = 30, 40
    assert oracle.canny(np.full((H, W), 77, np.uint8))[2] == 0
    img = np.full((H, W), 50, np.uint8)
    img[:, 20:] = 200                      # vertical step between columns 19 and 20
    e, _, n = oracle.canny(img, t_low=64, t_high=128)
    want = np.zeros((H, W), np.uint8)
    want[1:H - 1, 19] = 255                # one column: the left of the two equal maxima
    assert (e == want).all() and n == H - 2
    e, _, _ = oracle.canny(img.T.copy(), t_low=64, t_high=128)
    assert (e == want.T).all()             # horizontal step: one row
    # a step below the high threshold and above the low one has no strong pixel
    weak = np.full((H, W), 100, np.uint8)
    weak[:, 20:] = 118
    _, mag, _ = oracle.canny(weak, t_low=10, t_high=200)
    assert 10 < mag[5, 19] <= 200
    assert oracle.canny(weak, t_low=10, t_high=200)[2] == 0


def test_canny_diagonal_step_is_thin_and_continuous(oracle):
    H = W = 48
    yy, xx = np.mgrid[0:H, 0:W]
    img = np.where(xx + yy > 47, 210, 60).astype(np.uint8)
    e, _, _ = oracle.canny(img, t_low=64, t_high=128)
    ys, xs = np.nonzero(e)
    assert len(ys) > 0
    assert set((xs + ys).tolist()) <= {47, 48}      # within half a pixel of the boundary
    for y in range(3, H - 3):                       # an unbroken 8-connected line
        assert e[y].any()


def textbook_kept(img, boundary_deg=22.5):
    """Thinning step of Canny with the gradient direction quantised by its
    angle (atan2 in double precision, folded into [0, 90] degrees): below the
    boundary the neighbours along x, above 90 - boundary those along y, else
    the diagonal the signs of gx, gy point along.  Returns (kept, angle)."""
    a = img.astype(np.int64)
    b = (ndimage.correlate(a, np.outer(W5, W5), mode="nearest") + 128) >> 8
    gx = ndimage.correlate(b, KX, mode="nearest")
    gy = ndimage.correlate(b, KY, mode="nearest")
    m = np.abs(gx) + np.abs(gy)
    ang = np.degrees(np.arctan2(np.abs(gy), np.abs(gx)))
    H, W = img.shape
    mp = np.pad(m, 1)                                    # zero outside the frame

    def nb(dx, dy):
        return mp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]

    m1 = np.where(ang < boundary_deg, nb(-1, 0),
                  np.where(ang > 90 - boundary_deg, nb(0, -1),
                           np.where(gx * gy > 0, nb(-1, -1), nb(1, -1))))
    m2 = np.where(ang < boundary_deg, nb(1, 0),
                  np.where(ang > 90 - boundary_deg, nb(0, 1),
                           np.where(gx * gy > 0, nb(1, 1), nb(-1, 1))))
    return (m > m1) & (m >= m2) & (m > 0), ang


def sector_images():
    H = W = 64
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    out = []
    for phi in (20, 25, 65, 70, 110, 115, 155, 160):      # step normals either side of each boundary
        t = np.radians(phi)
        d = (xx - 31.3) * np.cos(t) + (yy - 32.6) * np.sin(t)
        out.append(np.where(d > 0, 205, 55).astype(np.uint8))
    for seed in range(6):                               # every direction, smoothly varying
        rng = np.random.default_rng(90 + seed)
        f = ndimage.gaussian_filter(rng.integers(0, 256, (H, W)).astype(float), 2.5)
        out.append(np.clip((f - f.mean()) * 8 + 128, 0, 255).astype(np.uint8))
    return out


def test_canny_sectors_match_the_angle(oracle):
    """Pins the sector boundary tan(22.5 deg) = 13573 / 2^15 of the integer
    definition: on step edges whose normals lie at 20/25 (and 65/70, ...)
    degrees and on smooth random images, the thinned pixels (thresholds 0,
    no ring) equal those of the textbook quantisation of the angle itself.
    Pixels within 1e-4 degrees of a boundary (where the rounded constant and
    the exact angle may disagree) are left out; the images hold hundreds of
    pixels within a degree of each side of 22.5, so a constant off by a few
    hundredths of a degree already changes the result (checked below with
    the boundary moved to 22.3 degrees)."""
    near_lo = near_hi = 0
    moved_differs = False
    for img in sector_images():
        got = oracle.canny(img, t_low=0, t_high=0, border_mode=0)[0] == 255
        want, ang = textbook_kept(img)
        exact = (np.abs(ang - 22.5) > 1e-4) & (np.abs(ang - 67.5) > 1e-4)
        assert (got == want)[exact].all()
        near_lo += int(((ang > 21.5) & (ang < 22.5)).sum())
        near_hi += int(((ang > 22.5) & (ang < 23.5)).sum())
        moved, _ = textbook_kept(img, 22.3)
        moved_differs |= bool((moved != want)[exact].any())
    assert near_lo > 100 and near_hi > 100
    assert moved_differs


@pytest.mark.parametrize("seed", range(5))
def test_canny_hysteresis_is_connected_components(oracle, seed):
    rng = np.random.default_rng(50 + seed)
    H, W = 60, 80
    img = ndimage.gaussian_filter(rng.integers(0, 256, (H, W)).astype(float), 2.0)
    img = np.clip((img - img.mean()) * 6 + 128, 0, 255).astype(np.uint8)
    lo, hi = 40, 120
    cand = oracle.canny(img, t_low=lo, t_high=lo)[0] == 255     # kept and above low
    strong = oracle.canny(img, t_low=hi, t_high=hi)[0] == 255   # kept and above high
    assert strong.any() and (cand & ~strong).any()
    lab, _ = ndimage.label(cand, structure=np.ones((3, 3), int))
    keep = np.unique(lab[strong])
    want = np.isin(lab, keep[keep > 0])
    got = oracle.canny(img, t_low=lo, t_high=hi)[0] == 255
    assert (got == want).all()


# ------------------------------------------- coarse-to-fine Hough (Sec. 4.3, ref. [9])
# The progressive transform is pinned against the plain vote and peaks
# (themselves pinned above): with no coarsening it must reduce to them, its
# coarse accumulator must be the binned fine rows it samples, its windows
# must be cells of the fine accumulator (with the half-turn mirror), its
# final peaks the brute-force greedy selection over the candidates, and it
# must find drawn lines at their own cells.

def _prog(f=4, w=9, kc=8, hct=1, hcr=2, minc=1, mt=2, mr=6, k=4, ht=1, hr=2, mv=1):
    return dict(theta_step=f, r_width=w, k_coarse=kc, h_theta_coarse=hct, h_r_coarse=hcr,
                min_votes_coarse=minc, margin_theta=mt, margin_r=mr, k=k, h_theta=ht, h_r=hr,
                min_votes=mv)


def _random_edges(seed, H, W, p):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((H, W)) < p, 255, 0).astype(np.uint8)


@pytest.mark.parametrize("seed", range(4))
def test_progressive_without_coarsening_is_the_plain_hough(oracle, synth, seed):
    """theta_step 1, r_width 1, no margins: the coarse accumulator is the
    fine one, each window is its coarse peak's own cell, and the final
    peaks are the brute-force greedy peaks of the fine accumulator."""
    H, W, n_theta = 24 + seed, 30 + 3 * seed, [8, 12, 9, 16][seed]
    e = _random_edges(seed, H, W, 0.15)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    for k, ht, hr in ((1, 0, 0), (3, 1, 1), (6, 2, 3)):
        out = oracle.hough_progressive(e, C, S, D, **_prog(1, 1, k, ht, hr, 1, 0, 0, k, ht, hr, 1))
        assert out["n_c"] == n_theta and out["n_rc"] == 2 * D + 1 and out["Dc"] == D
        assert (out["coarse_acc"] == acc).all()
        want = _brute_peaks(acc, D, k, ht, hr)
        got = [(int(out["theta_idx"][j]), int(out["r_idx"][j]), int(out["votes"][j]))
               for j in range(out["count"])]
        assert got == want
        for j in range(out["coarse_count"]):
            assert out["windows"][j].shape == (1, 1)
            assert out["windows"][j][0, 0] == acc[out["coarse_theta"][j], out["coarse_r"][j]]


@pytest.mark.parametrize("f,w", [(2, 3), (4, 9), (3, 5), (6, 1), (1, 7), (12, 15)])
def test_progressive_coarse_rows_are_binned_fine_rows(oracle, synth, f, w):
    """Coarse row c is fine row c*f + f/2 with odd-width r bins centred on
    r = 0: every coarse cell is the sum of w fine cells of that row."""
    H, W, n_theta = 41, 57, 36
    e = _random_edges(7 + f + w, H, W, 0.2)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, cast, dropped = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    assert dropped == 0
    out = oracle.hough_progressive(e, C, S, D, **_prog(f, w))
    q, Dc = (w - 1) // 2, out["Dc"]
    assert Dc * w + q >= D and (Dc - 1) * w + q < D   # the outer bins reach +-D
    want = np.zeros((n_theta // f, 2 * Dc + 1), np.int64)
    for c in range(n_theta // f):
        row = acc[c * f + f // 2]
        for i in range(2 * D + 1):
            r = i - D
            b = math.floor((r + q) / w)
            assert b * w - q <= r <= b * w + q
            want[c, b + Dc] += row[i]
    assert (out["coarse_acc"] == want).all()
    assert (out["coarse_acc"].sum(axis=1) == int((e == 255).sum())).all()


def _unfolded_cell(u, rr, n_theta, D):
    """Fine accumulator cell of the line at unfolded row u and r = rr."""
    h = u // n_theta
    t = u - h * n_theta
    r = -rr if h % 2 else rr
    return t, r + D


@pytest.mark.parametrize("case", ["vertical", "near_180", "random"])
def test_progressive_windows_are_fine_cells(oracle, synth, case):
    """Every window cell equals the fine accumulator at the cell's line,
    including rows that run past 0 or 180 degrees (where the line's r is
    mirrored), and the candidate is the first largest in window order."""
    H, W, n_theta = 64, 80, 72
    e = _random_edges(3, H, W, 0.02)
    if case == "vertical":
        e[:, 37] = 255                       # theta = 0, r = 37
    elif case == "near_180":
        yy, xx = np.mgrid[0:H, 0:W]
        th = 70 * math.pi / 72               # 175 degrees
        e[np.abs(xx * math.cos(th) + yy * math.sin(th) + 20) < 0.4] = 255
    else:
        e = _random_edges(4, H, W, 0.25)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    f, w, mt, mr = 4, 5, 3, 4
    out = oracle.hough_progressive(e, C, S, D, **_prog(f, w, 6, 1, 1, 1, mt, mr, 3, 1, 2, 1))
    q, Dc, R, Wc = (w - 1) // 2, out["Dc"], out["R"], out["Wc"]
    wraps = 0
    for j in range(out["coarse_count"]):
        c, bi = int(out["coarse_theta"][j]), int(out["coarse_r"][j])
        best, where = -1, None
        for a in range(R):
            u = c * f - mt + a
            wraps += u < 0 or u >= n_theta
            for ee in range(Wc):
                t, i = _unfolded_cell(u, (bi - Dc) * w - q - mr + ee, n_theta, D)
                inside = 0 <= i <= 2 * D
                assert out["windows"][j, a, ee] == (acc[t, i] if inside else 0)
                if inside and acc[t, i] > best:
                    best, where = int(acc[t, i]), (t, i)
        assert tuple(out["cand"][j]) == (where[0], where[1], best)
    for j in range(out["coarse_count"], 6):
        assert (out["windows"][j] == 0).all() and (out["cand"][j] == -1).all()
    if case != "random":
        assert wraps > 0


@pytest.mark.parametrize("seed", range(3))
def test_progressive_final_is_greedy_over_candidates(oracle, synth, seed):
    H, W, n_theta = 50, 70, 36
    e = _random_edges(20 + seed, H, W, 0.3)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    for k, ht, hr, mv in ((4, 1, 2, 1), (8, 3, 5, 1), (8, 0, 0, 60)):
        out = oracle.hough_progressive(e, C, S, D, **_prog(3, 7, 12, 1, 1, 1, 1, 3, k, ht, hr, mv))
        sparse = np.zeros((n_theta, 2 * D + 1), np.int32)
        for j in range(out["coarse_count"]):
            t, i, v = out["cand"][j]
            sparse[t, i] = v
        want = _brute_peaks(sparse, D, k, ht, hr, mv)
        got = [(int(out["theta_idx"][j]), int(out["r_idx"][j]), int(out["votes"][j]))
               for j in range(out["count"])]
        assert got == want


def test_progressive_finds_drawn_lines(oracle, synth):
    """Three real lines drawn at angles between the coarse samples over
    faint salt: the final peaks are exactly their own cells, with every
    drawn pixel counted (Sec. 2.3: the peak cell is the line)."""
    H, W, n_theta = 240, 320, 180
    yy, xx = np.mgrid[0:H, 0:W]
    e = _random_edges(5, H, W, 0.003)
    lines = [(33, 60), (91, 150), (150, -40)]
    on_all = []
    for k0, r0 in lines:
        th = k0 * math.pi / n_theta
        on = np.abs(xx * math.cos(th) + yy * math.sin(th) - r0) < 0.3
        e[on] = 255
        on_all.append(on)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    out = oracle.hough_progressive(e, C, S, D, **_prog(2, 5, 8, 1, 2, 1, 1, 6, 3, 2, 6, 1))
    got = {(int(out["theta_idx"][j]), int(out["r_idx"][j])) for j in range(out["count"])}
    assert got == {(k0, r0 + D) for k0, r0 in lines}
    for j in range(out["count"]):
        t, i = int(out["theta_idx"][j]), int(out["r_idx"][j])
        assert out["votes"][j] == acc[t, i]
    for (k0, r0), on in zip(lines, on_all):
        assert acc[k0, r0 + D] >= on.sum()
