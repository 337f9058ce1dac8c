"""GPU parity of the coarse-to-fine Hough transform (lane_hough_progressive)
with the CPU oracle: the coarse accumulator, the coarse peaks, every window
cell, the candidates and the final peaks, bit-exact, on road frames (Sobel
and Canny edges), random edge maps of odd sizes across every coarse layout
(4, 2 and 1 rows per workgroup), windows that run past 0 and 180 degrees,
table rows that throw r out of range, early stops, and the largest frame."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lane():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2212_09460_amd.lane as lane_mod

    return lane_mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print("[case]", *a, flush=True)


def check(lane, oracle, e, C, S, D, params, lst=None, ws=None):
    """Run both sides on edge map e (uint8 [H][W], 255 = edge) and compare
    every output; returns the oracle's result."""
    H, W = e.shape
    if lst is None:
        lst, _ = lane.edges_to_list(dev(e))
    t, r, v, c, det = lane.hough_progressive(lst, W, H, dev(C), dev(S), D, params, ws=ws)
    o = oracle.hough_progressive(e, C, S, D, **params)
    kc = params["k_coarse"]
    assert (host(det["coarse_acc"]) == o["coarse_acc"]).all(), "coarse accumulator"
    cp = host(det["coarse_peaks"])
    assert (cp[:kc] == o["coarse_theta"]).all() and (cp[kc:2 * kc] == o["coarse_r"]).all()
    assert (cp[2 * kc:3 * kc] == o["coarse_votes"]).all() and cp[3 * kc] == o["coarse_count"]
    assert (host(det["windows"]) == o["windows"]).all(), "windows"
    assert (host(det["candidates"]) == o["cand"]).all(), "candidates"
    assert (host(t) == o["theta_idx"]).all() and (host(r) == o["r_idx"]).all()
    assert (host(v) == o["votes"]).all() and int(host(c)[0]) == o["count"]
    return o


@pytest.mark.parametrize("which", ["640", "1080", "4k"])
def test_progressive_road_frames_sobel(lane, synth, oracle, which):
    say("progressive road sobel", which)
    if which == "640":
        img, n_theta = synth.plain_640(0), 180
    elif which == "1080":
        img, n_theta = synth.plain_1080(0), 360
    else:
        img, n_theta = synth.gen_frame(synth.scene_road(3840, 2160), 7), 360
    H, W = img.shape
    C, S = synth.trig_q14(n_theta)
    D = oracle.r_offset(W, H)
    e, _, lst, _ = lane.sobel_binarize(dev(img), W, 128, 1)
    eo, _, _ = oracle.sobel_binarize(img, W, 128, 1)
    assert (host(e) == eo).all()
    o = check(lane, oracle, eo, C, S, D, lane.progressive_params(n_theta, 2 * D + 1), lst=lst)
    assert o["count"] > 0


def test_progressive_road_frame_canny(lane, synth, oracle):
    say("progressive road canny 1080")
    img = synth.plain_1080(2)
    H, W = img.shape
    C, S = synth.trig_q14(360)
    D = oracle.r_offset(W, H)
    _, _, lst, _ = lane.canny(dev(img), W, 64, 128, 1)
    eo, _, _ = oracle.canny(img, W, 64, 128, 1)
    for over in ({}, dict(theta_step=8, r_width=15, margin_theta=4, margin_r=10, k_coarse=32, k=16),
                 dict(theta_step=2, r_width=3, margin_theta=1, margin_r=2)):
        say("  params", over)
        check(lane, oracle, eo, C, S, D, lane.progressive_params(360, 2 * D + 1, **over), lst=lst)


@pytest.mark.parametrize("W,H,n_theta,p,seed,over", [
    (1, 1, 8, 1.0, 0, dict(theta_step=2, k_coarse=2, k=1)),
    (7, 13, 12, 0.6, 1, dict(theta_step=3, r_width=3, margin_theta=1, margin_r=1, k_coarse=6, k=4)),
    (63, 17, 36, 0.3, 2, dict(theta_step=1, r_width=1, margin_theta=0, margin_r=0, k_coarse=8, k=8,
                              h_theta_coarse=1, h_r_coarse=1, h_theta=1, h_r=1)),
    (997, 41, 360, 0.2, 3, dict(theta_step=6, r_width=15, margin_theta=4, margin_r=9, k_coarse=64, k=64)),
    (300, 200, 180, 0.1, 4, dict(theta_step=4, r_width=63, margin_theta=3, margin_r=40)),
    (33, 600, 90, 0.5, 5, dict(theta_step=5, r_width=7, k_coarse=20, k=10, h_theta=0, h_r=0)),
    (1920, 1080, 360, 0.05, 6, dict(r_width=1, margin_r=3)),                  # 2 rows per group
    (3840, 2160, 180, 0.01, 7, dict(r_width=1, margin_r=2, theta_step=2)),    # 1 row per group
])
def test_progressive_random_edges(lane, synth, oracle, W, H, n_theta, p, seed, over):
    say("progressive random", W, H, n_theta, p, seed, over)
    rng = np.random.default_rng(seed)
    e = np.where(rng.random((H, W)) < p, 255, 0).astype(np.uint8)
    e[rng.random((H, W)) < 0.02] = 7     # not 255: not an edge
    C, S = synth.trig_q14(n_theta)
    D = oracle.r_offset(W, H)
    params = lane.progressive_params(n_theta, 2 * D + 1, **over)
    lay = lane.progressive_layout(W, H, n_theta, D, params)
    say("  layout", lay["n_coarse_theta"], lay["n_coarse_r"], lay["win_rows"], lay["win_cols"])
    check(lane, oracle, e, C, S, D, params)


@pytest.mark.parametrize("angle", [0, 1, 175, 179])
def test_progressive_windows_past_the_half_turn(lane, synth, oracle, angle):
    """A strong line near 0 or 180 degrees: its coarse peak sits in the first
    or last coarse row and its window reads mirrored rows."""
    say("progressive wrap", angle)
    H, W, n_theta = 240, 320, 180
    rng = np.random.default_rng(angle)
    e = np.where(rng.random((H, W)) < 0.01, 255, 0).astype(np.uint8)
    yy, xx = np.mgrid[0:H, 0:W]
    th = angle * math.pi / n_theta
    for r0 in (40, -30, 150):
        e[np.abs(xx * math.cos(th) + yy * math.sin(th) - r0) < 0.45] = 255
    C, S = synth.trig_q14(n_theta)
    D = oracle.r_offset(W, H)
    params = lane.progressive_params(n_theta, 2 * D + 1, theta_step=4, r_width=5, margin_theta=5,
                                     margin_r=6, k_coarse=8, k=4, h_theta=3, h_r=4)
    o = check(lane, oracle, e, C, S, D, params)
    assert o["count"] >= 1


def test_progressive_out_of_range_rows_and_early_stops(lane, synth, oracle):
    say("progressive odd table / min_votes")
    H, W, n_theta = 90, 140, 48
    rng = np.random.default_rng(11)
    e = np.where(rng.random((H, W)) < 0.2, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(n_theta)
    C, S = C.copy(), S.copy()
    C[5], S[5] = 30000, 30000        # r far beyond +-D: not counted
    C[23], S[23] = -32000, 1000
    C[31], S[31] = 100, -200         # small values: r near 0
    D = oracle.r_offset(W, H)
    base = dict(theta_step=2, r_width=5, margin_theta=3, margin_r=4, k_coarse=10, k=6)
    check(lane, oracle, e, C, S, D, lane.progressive_params(n_theta, 2 * D + 1, **base))
    # coarse min_votes above every count: no coarse peak, nothing downstream
    o = check(lane, oracle, e, C, S, D,
              lane.progressive_params(n_theta, 2 * D + 1, **base, min_votes_coarse=10 ** 7))
    assert o["coarse_count"] == 0 and o["count"] == 0
    # final min_votes between the candidates' counts: fewer final peaks
    o = check(lane, oracle, e, C, S, D, lane.progressive_params(n_theta, 2 * D + 1, **base))
    cv = sorted(int(x) for x in o["cand"][:, 2] if x > 0)
    mid = cv[len(cv) // 2]
    o2 = check(lane, oracle, e, C, S, D,
               lane.progressive_params(n_theta, 2 * D + 1, **base, min_votes=mid))
    assert 0 < o2["count"] <= o["count"]


def test_progressive_workspace_reuse_and_empty_list(lane, synth, oracle):
    """The same workspace serves two frames in a row (every section is
    rewritten); an empty edge map gives no peak."""
    say("progressive workspace reuse")
    n_theta = 180
    C, S = synth.trig_q14(n_theta)
    W, H = 400, 300
    D = oracle.r_offset(W, H)
    params = lane.progressive_params(n_theta, 2 * D + 1)
    ws = torch.empty(lane.progressive_layout(W, H, n_theta, D, params)["bytes"] // 8 + 2,
                     dtype=torch.int64, device="cuda")
    rng = np.random.default_rng(3)
    e1 = np.where(rng.random((H, W)) < 0.3, 255, 0).astype(np.uint8)
    check(lane, oracle, e1, C, S, D, params, ws=ws)
    o = check(lane, oracle, np.zeros((H, W), np.uint8), C, S, D, params, ws=ws)
    assert o["count"] == 0 and o["coarse_count"] == 0
    e2 = np.where(rng.random((H, W)) < 0.05, 255, 0).astype(np.uint8)
    check(lane, oracle, e2, C, S, D, params, ws=ws)


def test_progressive_largest_frame(lane, synth, oracle):
    say("progressive 8192 x 8192")
    W = H = 8192
    e = np.zeros((H, W), np.uint8)
    e[4000, 100:8100] = 255
    e[10:8180, 7000] = 255
    idx = np.arange(50, 8150)
    e[idx, idx] = 255
    rng = np.random.default_rng(9)
    e[rng.integers(0, H, 100000), rng.integers(0, W, 100000)] = 255
    C, S = synth.trig_q14(180)
    D = oracle.r_offset(W, H)
    for over in (dict(theta_step=4, r_width=9), dict(theta_step=2, r_width=1, margin_r=2)):
        say("  params", over)
        params = lane.progressive_params(180, 2 * D + 1, k_coarse=8, k=4, **over)
        o = check(lane, oracle, e, C, S, D, params)
        assert o["votes"][0] >= 8000
