"""Guard bands around every output buffer: each output (edge map, magnitude,
edge list, edge count, accumulator, dropped count, peaks, peak workspace,
line segments) sits between two 4 KiB bands of a sentinel byte, and after
every launch the bands must be untouched -- for the single-frame entry
points and for batch plans (mixed sizes, split votes, masks) -- while the
results equal the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GUARD = 4096
SENTINEL = 0xA5


@pytest.fixture(scope="module")
def lane():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2212_09460_amd.lane as lane_mod

    return lane_mod


def say(*a):
    print("[case]", *a, flush=True)


class Guarded:
    """A device buffer of `nbytes` between two sentinel bands."""

    def __init__(self, nbytes):
        self.n = int(nbytes)
        self.buf = torch.full((self.n + 2 * GUARD,), SENTINEL, dtype=torch.uint8, device="cuda")

    def view(self, shape, dtype):
        return self.buf[GUARD:GUARD + self.n].view(dtype).view(shape)

    def intact(self):
        return bool((self.buf[:GUARD] == SENTINEL).all()) and bool((self.buf[GUARD + self.n:] == SENTINEL).all())


def guarded(shape, dtype):
    n = int(np.prod(shape)) * torch.tensor([], dtype=dtype).element_size()
    g = Guarded(max(n, 4))
    return g, g.view((-1,), dtype)[:int(np.prod(shape))].view(shape)


def all_intact(gs, what):
    torch.cuda.synchronize()
    for name, g in gs.items():
        assert g.intact(), f"{what}: guard band of {name} overwritten"


@pytest.mark.parametrize("W,H,n_theta,k", [(1, 1, 7, 2), (17, 5, 180, 3), (997, 41, 360, 8),
                                           (640, 480, 180, 2), (1920, 1080, 360, 8),
                                           (4100, 37, 90, 4)])
def test_single_frame_calls_stay_in_bounds(lane, synth, oracle, W, H, n_theta, k):
    say("guard bands, single-frame calls", W, H, n_theta, k)
    img = synth.road(W, H, 77) if W >= 8 and H >= 8 else np.random.default_rng(1).integers(
        0, 256, (H, W)).astype(np.uint8)
    C, S = synth.trig_q14(n_theta)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    d_img = torch.from_numpy(img).cuda()
    want = oracle.pipeline(img, C, S, k)
    D, n_r = want["D"], want["n_r"]
    gs = {}
    gs["edges"], edges = guarded((H, W), torch.uint8)
    gs["mag"], mag = guarded((H, W), torch.uint8)
    gs["list"], lst = guarded((lane.edge_list_size(W, H) // 4,), torch.int32)
    gs["count"], cnt = guarded((1,), torch.int32)
    lane.sobel_binarize(d_img, W, 128, 1, edges=edges, mag=mag, edge_list=lst, edge_count=cnt)
    all_intact(gs, "sobel")
    assert (edges.cpu().numpy() == want["edges"]).all() and (mag.cpu().numpy() == want["mag"]).all()
    assert int(cnt.cpu()[0]) == want["n_edges"]
    gs["acc"], acc = guarded((n_theta, n_r), torch.int32)
    gs["dropped"], dropped = guarded((1,), torch.int32)
    lane.hough_vote(lst, W, H, Cd, Sd, D, n_r, acc=acc, dropped=dropped)
    all_intact(gs, "vote")
    assert (acc.cpu().numpy() == want["acc"]).all() and int(dropped.cpu()[0]) == want["dropped"]
    gs["peaks"], out = guarded((3 * k + 1,), torch.int32)
    gs["peaks_ws"], ws = guarded((lane.peaks_workspace_size(n_theta, n_r) // 8,), torch.int64)
    t, r, v, c = lane.hough_peaks(acc, D, k, out=out, ws=ws)
    all_intact(gs, "peaks")
    assert int(c.cpu()[0]) == want["count"] and (t.cpu().numpy() == want["theta_idx"]).all()
    assert (r.cpu().numpy() == want["r_idx"]).all() and (v.cpu().numpy() == want["votes"]).all()
    t2, r2, v2, c2 = lane.hough_peaks_noalloc(acc, D, k, out=out)
    all_intact(gs, "peaks without workspace")
    assert int(c2.cpu()[0]) == want["count"] and (v2.cpu().numpy() == want["votes"]).all()
    max_seg = 4
    gs["segments"], segs = guarded((k, max_seg, 4), torch.int32)
    gs["seg_count"], sc = guarded((k,), torch.int32)
    gs["npts"], npts = guarded((k,), torch.int32)
    lane.hough_lines(edges, Cd, Sd, D, t, r, c, max_segments=max_seg, segments=segs, seg_count=sc,
                     npts=npts)
    all_intact(gs, "lines")


def test_batch_plans_stay_in_bounds(lane, synth, oracle):
    """Mixed sizes with masks, plain and split votes, graph replays: every
    output of every frame keeps its guard bands."""
    specs = [(640, 480, 5, False), (1280, 720, 6, True), (997, 41, 7, False), (1920, 1080, 8, True),
             (33, 17, 9, False)]
    n_theta, k = 360, 8
    C, S = synth.trig_q14(n_theta)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    frames, wants, gs = [], [], {}
    for i, (W, H, seed, masked) in enumerate(specs):
        img = synth.road(W, H, seed)
        mask = None
        if masked:
            mask = np.random.default_rng(seed).integers(0, 256, ((H + 7) // 8, (W + 7) // 8)).astype(np.uint8)
        fb = lane.FrameBuffers(torch.from_numpy(img).cuda(), W, n_theta, k, Cd, Sd,
                               tile_mask=None if mask is None else torch.from_numpy(mask).cuda())
        gs[f"{i}.edges"], fb.edges = guarded((H, W), torch.uint8)
        gs[f"{i}.list"], fb.edge_list = guarded((lane.edge_list_size(W, H) // 4,), torch.int32)
        gs[f"{i}.acc"], fb.acc = guarded((fb.n_theta, fb.n_r), torch.int32)
        gs[f"{i}.peaks"], fb.peaks = guarded((3 * k + 1,), torch.int32)
        gs[f"{i}.counters"], fb.counters = guarded((2,), torch.int32)
        frames.append(fb)
        wants.append(oracle.pipeline(img, C, S, k, tile_mask=mask))
    for split in (0, 8):
        say("guard bands, batch plan, vote split", split)
        b = lane.Batch(frames, vote_rows=4 if split else 0, vote_split=split)
        for rep in range(2):
            b.launch()
            all_intact(gs, f"batch split {split} launch {rep}")
            for i, (f, w) in enumerate(zip(frames, wants)):
                assert (f.acc.cpu().numpy() == w["acc"]).all(), (split, i)
                assert int(f.count().cpu()) == w["count"], (split, i)
                assert (f.votes().cpu().numpy() == w["votes"]).all(), (split, i)
        b.close()
