"""C ABI contract checks that need no GPU: the library loads, exports every
function include/lane.h declares, its host helpers agree with the inputs
module / the mathematics, and bad arguments are rejected before any launch.
(No call here reaches a kernel: each one fails validation first.)"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lane.h")
LIB = os.environ.get("LANE_LIB_PATH") or os.path.join(ROOT, "paper_2212_09460_amd", "liblane.so")

E_ARG, E_SIZE, E_RANGE, E_WS, E_UNSUP = -1, -2, -3, -4, -6


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(lane_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblane.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    import paper_2212_09460_amd.lane as lane

    assert sorted(lane.EXPORTS) == declared()


def test_abi_version_and_strerror(lib):
    assert lib.lane_abi_version() == 2
    lib.lane_strerror.restype = ctypes.c_char_p
    assert lib.lane_strerror(0) == b"ok"
    assert b"workspace" in lib.lane_strerror(E_WS)


def test_trig_table_matches_inputs_module(lib, synth):
    for n in (1, 7, 180, 360, 1024):
        c = np.zeros(n, np.int16)
        s = np.zeros(n, np.int16)
        assert lib.lane_make_trig_q14(n, c.ctypes.data_as(ctypes.c_void_p),
                                      s.ctypes.data_as(ctypes.c_void_p)) == 0
        c2, s2 = synth.trig_q14(n)
        assert (c == c2).all() and (s == s2).all()
    assert lib.lane_make_trig_q14(0, None, None) == E_ARG


def test_r_offset(lib, oracle):
    d = ctypes.c_int32(0)
    for W, H in [(1, 1), (3, 1), (640, 480), (1920, 1080), (3840, 2160), (8192, 8192), (8192, 3)]:
        assert lib.lane_r_offset(W, H, ctypes.byref(d)) == 0
        assert d.value == oracle.r_offset(W, H)
    assert lib.lane_r_offset(8193, 4, ctypes.byref(d)) == E_SIZE
    assert lib.lane_r_offset(0, 4, ctypes.byref(d)) == E_ARG


def test_edge_list_size(lib):
    n = ctypes.c_size_t(0)
    assert lib.lane_edge_list_size(1920, 1080, ctypes.byref(n)) == 0
    th, tw, nchunk = 135, 240, 2
    nseg = th * nchunk
    off_ent = (nseg + th * tw + 3) // 4 * 4
    assert n.value == 4 * (off_ent + nseg * 8192)
    assert lib.lane_edge_list_size(9000, 4, ctypes.byref(n)) == E_SIZE


def test_argument_errors_before_launch(lib):
    P = ctypes.c_void_p(16)  # never dereferenced: every call below fails validation
    P1 = ctypes.c_void_p(17)
    f = lib.lane_sobel_binarize
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    assert f(None, 8, 8, 8, 128, 1, P, None, None, None, None) == E_ARG
    assert f(P, 8, 8, 7, 128, 1, P, None, None, None, None) == E_ARG        # pitch < W
    assert f(P, 8, 8, 8, 256, 1, P, None, None, None, None) == E_ARG        # threshold
    assert f(P, 9000, 8, 9000, 128, 1, P, None, None, None, None) == E_SIZE
    assert f(P, 8, 8, 8, 128, 7, P, None, None, None, None) == E_UNSUP
    assert f(P, 8, 8, 8, 128, 1, P, None, P1, None, None) == E_ARG          # misaligned list
    v = lib.lane_hough_vote
    v.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert v(P, 8, 8, P, P, 0, 5, 11, None, P, None, None) == E_ARG
    assert v(P, 8, 8, P, P, 180, 5, 0, None, P, None, None) == E_ARG
    assert v(P, 8, 8, P, P, 90, 5, 11, P, P, None, None) == E_UNSUP        # mask needs n%4==0
    pk = lib.lane_hough_peaks
    pk.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    assert pk(P, 180, 11, 5, 0, 1, 1, 1, P, P, P, P, P, 1 << 20, None) == E_ARG   # k < 1
    assert pk(P, 180, 12, 5, 2, 1, 1, 1, P, P, P, P, P, 1 << 20, None) == E_RANGE  # n_r != 2D+1
    assert pk(P, 180, 11, 5, 2, 1, 1, 1, P, P, P, P, P, 8, None) == E_WS
    pn = lib.lane_hough_peaks_noalloc
    pn.argtypes = pk.argtypes[:12] + [ctypes.c_void_p]
    assert pn(P, 180, 11, 5, 0, 1, 1, 1, P, P, P, P, None) == E_ARG    # k < 1
    assert pn(None, 180, 11, 5, 2, 1, 1, 1, P, P, P, P, None) == E_ARG  # no accumulator
    assert pn(P, 180, 12, 5, 2, 1, 1, 1, P, P, P, P, None) == E_RANGE  # n_r != 2D+1
    assert pn(P, 1 << 16, 11, 5, 2, 1, 1, 1, P, P, P, P, None) == E_SIZE
    lib.lane_hough_peaks_noalloc_max_bytes.restype = ctypes.c_size_t
    assert lib.lane_hough_peaks_noalloc_max_bytes() == 8192 * 8
    ln = lib.lane_hough_lines
    ln.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p]
    ok = (P, 64, 48, P, P, 180, 79, P, P, None, 8, 20, 40, 16, P, P, None, None)
    def lines_with(i, val):
        a = list(ok)
        a[i] = val
        return ln(*a)
    assert lines_with(0, None) == E_ARG            # no edge map
    assert lines_with(10, 0) == E_ARG              # k < 1
    assert lines_with(10, 5000) == E_ARG           # k > 4096
    assert lines_with(11, -1) == E_ARG             # fill_gap
    assert lines_with(12, 70000) == E_ARG          # min_length
    assert lines_with(13, 0) == E_ARG              # max_segments
    assert lines_with(1, 9000) == E_SIZE
    assert lines_with(6, 200000) == E_RANGE        # r_offset


def test_progressive_layout_geometry_and_limits(oracle):
    """Layout of the coarse-to-fine Hough: geometry equal to the oracle's,
    sections in order inside the reported size, and the documented limits
    rejected (no device involved)."""
    import paper_2212_09460_amd.lane as lane

    for (W, H, n_theta, over) in [(1920, 1080, 360, {}), (1, 1, 8, dict(theta_step=2, k_coarse=2, k=1)),
                                  (8192, 8192, 180, dict(r_width=1, margin_r=0)),
                                  (640, 480, 180, dict(theta_step=6, r_width=15, margin_theta=0))]:
        D = oracle.r_offset(W, H)
        p = lane.progressive_params(n_theta, 2 * D + 1, **over)
        lay = lane.progressive_layout(W, H, n_theta, D, p)
        f, w = p["theta_step"], p["r_width"]
        q = (w - 1) // 2
        assert lay["n_coarse_theta"] == n_theta // f
        assert lay["coarse_r_offset"] == (D + q) // w
        assert lay["n_coarse_r"] == 2 * lay["coarse_r_offset"] + 1
        assert lay["win_rows"] == f + 2 * p["margin_theta"]
        assert lay["win_cols"] == w + 2 * p["margin_r"]
        kc = p["k_coarse"]
        assert lay["coarse_acc"] == 0
        assert lay["windows"] >= 4 * lay["n_coarse_theta"] * lay["n_coarse_r"]
        assert lay["coarse_peaks"] >= lay["windows"] + 4 * kc * lay["win_rows"] * lay["win_cols"]
        assert lay["candidates"] >= lay["coarse_peaks"] + 4 * (3 * kc + 1)
        assert lay["bytes"] > lay["candidates"] + 12 * kc
    D = oracle.r_offset(1920, 1080)
    good = lane.progressive_params(360, 2 * D + 1)
    bad = [dict(theta_step=7), dict(theta_step=0), dict(r_width=8), dict(r_width=65),
           dict(k_coarse=65), dict(k=17), dict(k=0), dict(h_theta=360), dict(h_theta=-1),
           dict(margin_theta=513), dict(margin_r=-1), dict(h_r_coarse=-1)]
    for over in bad:
        with pytest.raises(lane.LaneError) as ei:
            lane.progressive_layout(1920, 1080, 360, D, {**good, **over})
        assert ei.value.code == E_ARG, over
    with pytest.raises(lane.LaneError) as ei:   # window cells beyond the LDS budget
        lane.progressive_layout(1920, 1080, 360, D, {**good, "margin_theta": 100, "margin_r": 200})
    assert ei.value.code == E_SIZE
    with pytest.raises(lane.LaneError) as ei:
        lane.progressive_layout(1920, 1080, 360, 16385, good)
    assert ei.value.code == E_RANGE


def test_progressive_argument_errors_before_launch(lib):
    import paper_2212_09460_amd.lane as lane

    p = lane._prog_struct(lane.progressive_params(360, 4407))
    buf = (ctypes.c_uint8 * 64)()
    a16 = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 16
    f = lib.lane_hough_progressive
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p] + [ctypes.c_void_p] * 5 + \
                 [ctypes.c_size_t, ctypes.c_void_p]
    args = [a16, 1920, 1080, a16, a16, 360, 2203, ctypes.addressof(p), a16, a16, a16, a16, a16, 1 << 30, None]
    for i in (0, 3, 4, 7, 8, 9, 10, 11, 12):
        bad = list(args)
        bad[i] = None
        assert f(*bad) == E_ARG, i
    bad = list(args)
    bad[0] = a16 + 4           # list not 16-byte aligned
    assert f(*bad) == E_ARG
    bad = list(args)
    bad[13] = 16               # workspace too small
    assert f(*bad) == E_WS


def test_coarse_bin_division_by_float_reciprocal_is_exact():
    """The coarse vote finds floor(n / w) as trunc(fma(n, float(1/w),
    float(1/w) / 2)) in single precision; checked for every n in [0, 2^16)
    and every odd w <= 63 (the products are exact in double, so rounding
    the double sum to float is the one rounding of the fused multiply-add)."""
    n = np.arange(0, 1 << 16, dtype=np.int64)
    for w in range(1, 64, 2):
        iw = np.float32(1.0 / w)
        hiw = np.float32(0.5) * iw
        t = (n.astype(np.float64) * np.float64(iw) + np.float64(hiw)).astype(np.float32)
        assert (np.trunc(t).astype(np.int64) == n // w).all(), w


def test_paired_vote_argument_errors_before_launch(lib):
    f = lib.lane_hough_vote_paired
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    f.argtypes = [vp, i32, i32, vp, vp, i32, i32, i32, i32, vp, vp, vp]
    buf = (ctypes.c_uint8 * 64)()
    a16 = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 16
    good = [a16, 1920, 1080, a16, a16, 360, 2203, 4407, 1, a16, None, None]
    for i in (0, 3, 4, 9):
        bad = list(good)
        bad[i] = None
        assert f(*bad) == E_ARG, i
    for i, v in ((8, 2), (8, -1), (5, 0), (7, 0), (1, 0)):
        bad = list(good)
        bad[i] = v
        assert f(*bad) == E_ARG, (i, v)
    bad = list(good)
    bad[0] = a16 + 4
    assert f(*bad) == E_ARG
    bad = list(good)
    bad[6] = -1
    assert f(*bad) == E_RANGE
    bad = list(good)
    bad[1] = 8193
    assert f(*bad) == E_SIZE
