"""GPU parity of the line segments along peaks (lane_hough_lines) with the
CPU oracle: segments, counts and point counts equal element by element on
road frames (peaks from the GPU path, which equal the oracle's), random edge
maps with peaks at every angle, odd shapes, truncation, padding, the largest
frame, and a table row that is not a rotation."""
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


def both(lane, oracle, e, C, S, D, t, r, count=None, **kw):
    segs, cnt, npts = lane.hough_lines(dev(e), dev(C), dev(S), D, dev(t), dev(r),
                                       None if count is None else dev(np.array([count], np.int32)), **kw)
    tt = t.copy()
    if count is not None:
        tt[count:] = -1
    okw = dict(kw)
    if "max_segments" in okw:
        okw["max_seg"] = okw.pop("max_segments")
    so, co, no = oracle.hough_lines(e, C, S, D, tt, r, **okw)
    return (host(segs), host(cnt), host(npts)), (so, co, no)


def check(g, o):
    (sg, cg, ng), (so, co, no) = g, o
    assert (cg == co).all(), (cg, co)
    assert (ng == no).all(), (ng, no)
    assert (sg == so).all()


@pytest.mark.parametrize("which", ["640", "1080", "4k"])
def test_lines_road_frames(lane, synth, oracle, which):
    say("lines on road frame", which)
    if which == "640":
        img, n_theta, k = synth.plain_640(0), 180, 2
    elif which == "1080":
        img, n_theta, k = synth.plain_1080(0), 360, 8
    else:
        img, n_theta, k = synth.gen_frame(synth.scene_road(3840, 2160), 5), 360, 8
    H, W = img.shape
    C, S = synth.trig_q14(n_theta)
    want = oracle.pipeline(img, C, S, k)
    D = want["D"]
    got = lane.pipeline(dev(img), dev(C), dev(S), k)
    t, r, c = host(got["theta_idx"]), host(got["r_idx"]), int(host(got["count"])[0])
    assert (t == want["theta_idx"]).all() and (r == want["r_idx"]).all() and c == want["count"]
    # the chain on the device: the GPU edge map and the GPU peaks feed the lines
    segs, cnt, npts = lane.hough_lines(got["edges"], dev(C), dev(S), D, got["theta_idx"],
                                       got["r_idx"], got["count"])
    g = (host(segs), host(cnt), host(npts))
    o = oracle.hough_lines(want["edges"], C, S, D, want["theta_idx"], want["r_idx"])
    check(g, o)
    # the points of a peak are exactly the voters of its cell
    acc = want["acc"]
    assert (g[2][:c] == acc[t[:c], r[:c]]).all()
    assert (g[1][:c] >= 1).all()


@pytest.mark.parametrize("W,H,n_theta,p,seed", [(64, 48, 64, 0.3, 0), (200, 150, 180, 0.05, 1),
                                                (997, 41, 360, 0.2, 2), (33, 600, 90, 0.5, 3),
                                                (1, 1, 16, 1.0, 4), (7, 13, 7, 0.6, 5),
                                                (1280, 720, 360, 0.02, 6)])
def test_lines_random_edges_every_angle(lane, synth, oracle, W, H, n_theta, p, seed):
    say("lines random", W, H, n_theta, p, seed)
    rng = np.random.default_rng(seed)
    e = np.where(rng.random((H, W)) < p, 255, 0).astype(np.uint8)
    e[rng.random((H, W)) < 0.02] = 9  # not 255: not an edge
    C, S = synth.trig_q14(n_theta)
    D = oracle.r_offset(W, H)
    k = int(min(4096, 3 * n_theta, max(16, 2e8 // (W * H))))  # bounded oracle time
    t = np.repeat(np.arange(n_theta, dtype=np.int32), 3)[:k]
    r = rng.integers(0, 2 * D + 1, size=k).astype(np.int32)
    r[1::3] = D  # lines through the origin
    for fg, ml, ms in [(20, 40, 16), (1, 0, 4), (3, 5, 2), (0, 0, 64)]:
        g, o = both(lane, oracle, e, C, S, D, t, r, fill_gap=fg, min_length=ml, max_segments=ms)
        check(g, o)


def test_lines_drawn_segments(lane, synth, oracle):
    say("lines drawn segments")
    e = np.zeros((96, 128), np.uint8)
    e[40, 5:60] = 255
    e[40, 75:120] = 255
    for x in range(10, 80):
        e[x // 2 + 10, x] = 255   # a slope-1/2 staircase
    e[:, 100] = 255
    C, S = synth.trig_q14(180)
    D = oracle.r_offset(128, 96)
    acc, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
    t, r, v, n = oracle.hough_peaks(acc, D, 6)
    g, o = both(lane, oracle, e, C, S, D, t, r, count=n, fill_gap=5, min_length=10)
    check(g, o)
    assert g[1][:n].max() >= 2  # the split row gives two segments


def test_lines_padding_count_and_bad_table_row(lane, synth, oracle):
    say("lines padding / count / table row")
    rng = np.random.default_rng(11)
    e = np.where(rng.random((50, 70)) < 0.3, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(32)
    D = oracle.r_offset(70, 50)
    t = np.array([3, -1, 7, 9, 12], np.int32)
    r = np.array([D + 4, -1, D, D - 3, D + 10], np.int32)
    g, o = both(lane, oracle, e, C, S, D, t, r, count=3)   # peaks 3, 4 switched off
    check(g, o)
    assert g[1][1] == 0 and g[1][3] == 0 and g[1][4] == 0
    C2, S2 = C.copy(), S.copy()
    C2[7], S2[7] = 100, -200   # not a rotation: refused
    segs, cnt, npts = lane.hough_lines(dev(e), dev(C2), dev(S2), D, dev(t), dev(r))
    assert int(host(cnt)[2]) == -1 and int(host(npts)[2]) == 0


def test_lines_largest_frame(lane, synth, oracle):
    say("lines 8192 x 8192")
    W = H = 8192
    e = np.zeros((H, W), np.uint8)
    e[4000, 100:8100] = 255
    e[10:8180, 7000] = 255
    idx = np.arange(50, 8150)
    e[idx, idx] = 255
    rng = np.random.default_rng(3)
    ys, xs = rng.integers(0, H, 200000), rng.integers(0, W, 200000)
    e[ys, xs] = 255
    C, S = synth.trig_q14(180)
    D = oracle.r_offset(W, H)
    t = np.array([90, 0, 135, 45], np.int32)
    r = np.array([D + 4000, D + 7000, D, D + 5000], np.int32)
    g, o = both(lane, oracle, e, C, S, D, t, r, fill_gap=20, min_length=40)
    check(g, o)
    assert g[2].max() > 8000


def test_lines_in_batch_graph(lane, synth, oracle):
    """The batch's fifth stage: frames that ask for segments get them after
    their peaks, in the same graph launch, equal to the oracle on every
    replay; frames switched off by select keep their previous outputs."""
    say("lines in the batch graph")
    n_theta, k = 360, 8
    C, S = synth.trig_q14(n_theta)
    Cd, Sd = dev(C), dev(S)
    specs = [(640, 480, 640, 21, 16), (1280, 720, 1280, 22, 4), (1920, 1080, 1920, 23, 16),
             (997, 41, 1000, 24, 2), (3840, 2160, 3840, 25, 16), (640, 480, 640, 26, 0)]
    frames, wants = [], []
    for (Wf, Hf, pitch, seed, ms) in specs:
        img = synth.gen_frame(synth.scene_road(Wf, Hf), seed, pitch=pitch)
        fb = lane.FrameBuffers(dev(img), Wf, n_theta, k, Cd, Sd, lines_max_seg=ms,
                               lines_fill_gap=15, lines_min_length=30)
        frames.append(fb)
        w = oracle.pipeline(img[:, :Wf].copy(), C, S, k)
        if ms:
            w["lines"] = oracle.hough_lines(w["edges"], C, S, w["D"], w["theta_idx"], w["r_idx"],
                                            fill_gap=15, min_length=30, max_seg=ms)
        wants.append(w)

    def check_all(which):
        torch.cuda.synchronize()
        for i in which:
            f, w = frames[i], wants[i]
            assert (host(f.theta_idx()) == w["theta_idx"]).all(), i
            if f.lines is None:
                continue
            so, co, no = w["lines"]
            assert (host(f.seg_count()) == co).all(), i
            assert (host(f.line_npts()) == no).all(), i
            assert (host(f.segments()) == so).all(), i

    b = lane.Batch(frames)
    for rep in range(3):
        say("replay", rep)
        b.launch()
        check_all(range(len(frames)))
        for f in frames:
            if f.lines is not None:
                f.lines.fill_(-9)
        torch.cuda.synchronize()
    # only frames 1 and 4 run: their segments come back, the others keep -9
    b.select([0, 1, 0, 0, 1, 0])
    b.launch()
    check_all([1, 4])
    for i in (0, 2, 3):
        assert (host(frames[i].lines) == -9).all(), i
    b.select([1] * len(frames))
    b.launch_stage(4)   # the stage alone recomputes the segments from the kept peaks
    check_all(range(len(frames)))
    b.close()
