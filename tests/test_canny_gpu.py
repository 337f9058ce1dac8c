"""GPU parity of the Canny detector (lane_canny) with the CPU oracle: edge
maps, blurred-gradient magnitudes, edge counts and the edge list, bit-exact,
on road frames, random smooth images of odd sizes across tile boundaries,
both border modes, threshold corner cases, a frame-spanning weak chain (a
long union-find component), and Canny edges through the vote and peaks."""
import numpy as np
import pytest
from scipy import ndimage

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


def list_points(lst, W, H):
    """(x, y) of every entry of the edge list (layout in include/lane.h)."""
    a = host(lst).view(np.uint32)
    th, tw, nchunk = (H + 7) // 8, (W + 7) // 8, (W + 1023) // 1024
    nseg = th * nchunk
    off_ent = (nseg + th * tw + 3) // 4 * 4
    pts = [a[off_ent + s * 8192: off_ent + s * 8192 + a[s]] for s in range(nseg)]
    e = np.concatenate(pts) if pts else np.zeros(0, np.uint32)
    return np.sort((e >> 16).astype(np.int64) * W + (e & 0xFFFF).astype(np.int64))


def run_both(lane, oracle, img, W, lo, hi, bm=1):
    H = img.shape[0]
    e, m, lst, cnt = lane.canny(dev(img), W, lo, hi, bm, want_mag=True)
    eo, mo, no = oracle.canny(img, W, lo, hi, bm)
    eg, mg = host(e), host(m)
    assert (mg == mo).all(), "magnitude"
    assert (eg == eo).all(), "edges"
    assert int(host(cnt)[0]) == no
    ys, xs = np.nonzero(eo == 255)
    assert (list_points(lst, W, H) == np.sort(ys.astype(np.int64) * W + xs)).all(), "edge list"
    return eo, no


@pytest.mark.parametrize("which", ["640", "1080", "4k"])
def test_canny_road_frames(lane, synth, oracle, which):
    say("canny road", which)
    if which == "640":
        img = synth.plain_640(0)
    elif which == "1080":
        img = synth.plain_1080(0)
    else:
        img = synth.gen_frame(synth.scene_road(3840, 2160), 9)
    H, W = img.shape
    _, n = run_both(lane, oracle, img, W, 64, 128)
    assert n > 0


def smooth_random(rng, H, W, sigma, gain):
    f = ndimage.gaussian_filter(rng.integers(0, 256, (H, W)).astype(float), sigma)
    return np.clip((f - f.mean()) * gain + 128, 0, 255).astype(np.uint8)


@pytest.mark.parametrize("W,H,pitch,seed", [(1, 1, 1, 0), (7, 13, 7, 1), (63, 17, 64, 2), (65, 33, 65, 3),
                                            (1000, 41, 1008, 4), (300, 200, 300, 5), (129, 47, 130, 6)])
def test_canny_random_shapes(lane, oracle, W, H, pitch, seed):
    say("canny random", W, H, pitch, seed)
    rng = np.random.default_rng(seed)
    img = np.zeros((H, pitch), np.uint8)
    img[:, :W] = smooth_random(rng, H, W, 1.5, 5)
    img[:, W:] = 255  # padding columns must not be read
    for lo, hi, bm in [(40, 120, 1), (40, 120, 0), (0, 0, 1), (90, 90, 0), (30, 5000, 1)]:
        run_both(lane, oracle, img, W, lo, hi, bm)


def test_canny_frame_spanning_weak_chain(lane, oracle):
    """A serpentine of faint bars over the whole frame (weak edges) whose
    last bar rises to a strong section: hysteresis must carry the strong
    label through one component of about half a million pixels."""
    say("canny serpentine 2048 x 1024")
    H, W = 1024, 2048
    img = np.full((H, W), 100, np.uint8)
    ys = list(range(4, H - 4, 8))
    for k, y in enumerate(ys):
        img[y:y + 3, 4:W - 4] = 118                     # a faint bar: weak edges
        x = W - 6 if k % 2 == 0 else 4                  # joined at alternate ends
        img[y:y + 11, x:x + 2] = 118
    # the middle of the last bar rises smoothly to a strong section, so its
    # edge lines stay unbroken and carry the strong label to every bar
    xs = np.arange(600, 1000)
    img[ys[-1]:ys[-1] + 3, 600:1000] = np.clip(250 - np.abs(xs - 800) * 132 // 150, 118, 250)
    e, n = run_both(lane, oracle, img, W, 10, 60)
    assert n > 500000


def test_canny_through_vote_and_peaks(lane, synth, oracle):
    say("canny -> vote -> peaks 1080p")
    img = synth.plain_1080(1)
    H, W = img.shape
    C, S = synth.trig_q14(360)
    eo, _, _ = oracle.canny(img, W, 64, 128, 1)
    D = oracle.r_offset(W, H)
    acc_o, _, _ = oracle.hough_vote(eo, C, S, D, 2 * D + 1)
    to, ro, vo, no = oracle.hough_peaks(acc_o, D, 8)
    _, _, lst, _ = lane.canny(dev(img), W, 64, 128, 1)
    acc, dropped = lane.hough_vote(lst, W, H, dev(C), dev(S), D, 2 * D + 1)
    assert (host(acc) == acc_o).all()
    t, r, v, c = lane.hough_peaks(acc, D, 8)
    assert (host(t) == to).all() and (host(r) == ro).all() and (host(v) == vo).all()
