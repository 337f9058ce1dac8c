"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, on seeded inputs.  Integer path, so every comparison is
bit-exact.  Each test prints the case it runs before touching the GPU."""
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


def decode_list(lst, W, H):
    """Parse the edge list (layout in include/lane.h); return (entries as an
    array of (x, y), per-segment counts, per-tile (count, start))."""
    a = host(lst).view(np.uint32)
    th, tw, nchunk = (H + 7) // 8, (W + 7) // 8, (W + 1023) // 1024
    nseg = th * nchunk
    off_info = nseg
    off_ent = (nseg + th * tw + 3) // 4 * 4
    seg_count = a[:nseg].astype(np.int64)
    info = a[off_info:off_info + th * tw].reshape(th, tw)
    xy = []
    for seg in range(nseg):
        ty, chunk = divmod(seg, nchunk)
        base = off_ent + seg * 8192
        ents = a[base:base + seg_count[seg]]
        # grouping: tiles of the segment in x order, counts/starts consistent
        pos = 0
        for tx in range(chunk * 128, min(tw, chunk * 128 + 128)):
            cnt, start = int(info[ty, tx] >> 16), int(info[ty, tx] & 0xFFFF)
            if cnt:
                assert start == pos, (seg, tx, start, pos)
                e = ents[start:start + cnt]
                xs, ys = e & 0xFFFF, e >> 16
                assert ((xs >> 3) == tx).all() and ((ys >> 3) == ty).all()
                key = (ys & 7) * 8 + (xs & 7)
                assert (np.diff(key.astype(np.int64)) > 0).all()  # row-major in tile
            pos += cnt
        assert pos == seg_count[seg]
        xy.append(np.stack([ents & 0xFFFF, ents >> 16], 1))
    xy = np.concatenate(xy) if xy else np.zeros((0, 2), np.uint32)
    return xy, seg_count, info


def check_list_matches_edges(lst, edges, W, H):
    xy, seg_count, _ = decode_list(lst, W, H)
    ys, xs = np.nonzero(edges[:, :W] == 255)
    got = np.sort(xy[:, 1].astype(np.int64) * W + xy[:, 0].astype(np.int64))
    want = np.sort(ys.astype(np.int64) * W + xs)
    assert got.shape == want.shape and (got == want).all()
    assert int(seg_count.sum()) == len(want)


FRAMES = {
    "plain_640": lambda s: s.plain_640(0),
    "plain_1080": lambda s: s.plain_1080(0),
}


@pytest.mark.parametrize("name", sorted(FRAMES))
@pytest.mark.parametrize("mode", [0, 1])
def test_sobel_frames(lane, synth, oracle, name, mode):
    say("sobel", name, "border", mode)
    img = FRAMES[name](synth)
    H, W = img.shape
    e_o, m_o, n_o = oracle.sobel_binarize(img, W, 128, mode)
    e, m, lst, cnt = lane.sobel_binarize(dev(img), W, 128, mode, want_mag=True)
    assert (host(e) == e_o).all()
    assert (host(m) == m_o).all()
    assert int(host(cnt)[0]) == n_o
    check_list_matches_edges(lst, e_o, W, H)


ODD = [(1, 1), (5, 1), (1, 5), (7, 13), (16, 16), (33, 17), (1030, 9), (1024, 24), (8192, 3),
       (3, 2000), (997, 41), (2049, 40)]


@pytest.mark.parametrize("W,H", ODD)
def test_sobel_odd_shapes(lane, oracle, W, H):
    rng = np.random.default_rng(W * 7919 + H)
    for pitch in sorted({W, W + 3, ((W + 15) // 16) * 16 + 16}):
        say("sobel odd", W, H, "pitch", pitch)
        img = rng.integers(0, 256, size=(H, pitch), dtype=np.uint8)
        for T, mode in ((128, 1), (40, 0), (254, 1)):
            e_o, m_o, n_o = oracle.sobel_binarize(img, W, T, mode)
            e, m, lst, cnt = lane.sobel_binarize(dev(img), W, T, mode, want_mag=True)
            assert (host(e) == e_o).all(), (W, H, pitch, T, mode)
            assert (host(m) == m_o).all()
            assert int(host(cnt)[0]) == n_o
            check_list_matches_edges(lst, e_o, W, H)


@pytest.mark.parametrize("W,H,p", [(37, 29, 0.3), (1500, 70, 0.1), (640, 480, 0.02), (8, 8, 1.0)])
def test_edges_to_list(lane, W, H, p):
    say("edges_to_list", W, H, p)
    rng = np.random.default_rng(W + H)
    e = np.where(rng.random((H, W)) < p, 255, 0).astype(np.uint8)
    e[rng.random((H, W)) < 0.05] = 7  # not 255: not an edge
    lst, cnt = lane.edges_to_list(dev(e), W)
    check_list_matches_edges(lst, e, W, H)
    assert int(host(cnt)[0]) == int((e == 255).sum())


@pytest.mark.parametrize("seed", range(3))
def test_edges_to_list_tile_patterns(lane, seed):
    """Edge maps built tile by tile from patterns that exercise the list
    writer's cases: empty tiles, single pixels, full first / last rows (a
    lane's run ending in a full row), full tiles, sparse and dense random
    tiles, and tile rows above and below the one-pass stage size (2048)."""
    rng = np.random.default_rng(100 + seed)
    W, H = 2048 + 8 * seed + 16, 96
    th, tw = H // 8, W // 8
    e = np.zeros((H, W), np.uint8)
    for ty in range(th):
        dense_row = ty % 4 == 3  # more than 2048 edges in some segments
        for tx in range(tw):
            kind = rng.integers(0, 8)
            t = np.zeros((8, 8), bool)
            if kind == 1:
                t[rng.integers(0, 8), rng.integers(0, 8)] = True
            elif kind == 2:
                t[7, :] = True
            elif kind == 3:
                t[0, :] = True
            elif kind == 4 and (dense_row or rng.random() < 0.1):
                t[:, :] = True
            elif kind == 5:
                t = rng.random((8, 8)) < 0.2
            elif kind == 6:
                t = rng.random((8, 8)) < (0.9 if dense_row else 0.4)
            elif kind == 7:
                t[7, rng.integers(0, 8):] = True
            e[ty * 8:ty * 8 + 8, tx * 8:tx * 8 + 8] = np.where(t, 255, 0)
    say("edges_to_list tile patterns", W, H, seed, int((e == 255).sum()))
    lst, cnt = lane.edges_to_list(dev(e), W)
    check_list_matches_edges(lst, e, W, H)
    assert int(host(cnt)[0]) == int((e == 255).sum())


def vote_both(lane, oracle, e, W, H, C, S, D, n_r, mask=None):
    lst, _ = lane.edges_to_list(dev(e), W)
    acc, dropped = lane.hough_vote(lst, W, H, dev(C), dev(S), D, n_r,
                                   None if mask is None else dev(mask))
    acc_o, cast_o, drop_o = oracle.hough_vote(e, C, S, D, n_r, mask, W)
    return host(acc), int(host(dropped)[0]), acc_o, drop_o


@pytest.mark.parametrize("name,n_theta", [("plain_640", 180), ("plain_1080", 360)])
def test_vote_frames(lane, synth, oracle, name, n_theta):
    say("vote", name, n_theta)
    img = FRAMES[name](synth)
    H, W = img.shape
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    e_o, _, n_e = oracle.sobel_binarize(img, W, 128, 1)
    e, _, lst, _ = lane.sobel_binarize(dev(img), W, 128, 1)
    acc, dropped = lane.hough_vote(lst, W, H, dev(C), dev(S), D, 2 * D + 1)
    acc_o, cast_o, drop_o = oracle.hough_vote(e_o, C, S, D, 2 * D + 1)
    a = host(acc)
    assert int(host(dropped)[0]) == drop_o == 0
    assert (a == acc_o).all()
    assert a.sum() == n_e * n_theta


@pytest.mark.parametrize("W,H,n_theta", [(1, 1, 180), (7, 13, 7), (33, 17, 64), (1030, 9, 1),
                                         (3, 600, 33), (200, 150, 360), (997, 41, 128)])
def test_vote_odd(lane, synth, oracle, W, H, n_theta):
    say("vote odd", W, H, n_theta)
    rng = np.random.default_rng(W * 31 + H)
    e = np.where(rng.random((H, W)) < 0.3, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    a, d, a_o, d_o = vote_both(lane, oracle, e, W, H, C, S, D, 2 * D + 1)
    assert d == d_o == 0 and (a == a_o).all()


@pytest.mark.parametrize("seed", range(4))
def test_vote_unusual_tables_and_ranges(lane, synth, oracle, seed):
    """Tables / r ranges that send votes outside [0, n_r): the exact
    fallback path, with the dropped count."""
    say("vote unusual", seed)
    rng = np.random.default_rng(100 + seed)
    W, H, n_theta = 120, 75, 40
    e = np.where(rng.random((H, W)) < 0.2, 255, 0).astype(np.uint8)
    if seed == 0:
        C = np.full(n_theta, 32767, np.int16)
        S = np.full(n_theta, -32768, np.int16)
        D, n_r = 100, 301
    elif seed == 1:
        C = rng.integers(-32768, 32768, n_theta).astype(np.int16)
        S = rng.integers(-32768, 32768, n_theta).astype(np.int16)
        D, n_r = 300, 500
    elif seed == 2:
        C, S = synth.trig_q14(n_theta)
        D, n_r = 20, 41     # too narrow for the frame
    else:
        C, S = synth.trig_q14(n_theta)
        C = C.copy()
        C[5] = 32767        # one row leaves the range, the rest is normal
        D = synth.r_offset(W, H)
        n_r = 2 * D + 1
    a, d, a_o, d_o = vote_both(lane, oracle, e, W, H, C, S, D, n_r)
    assert d == d_o and (a == a_o).all()
    assert a.sum() + d == int((e == 255).sum()) * n_theta


def _masked_frame(synth, which):
    if which == "640":
        return synth.plain_640(1)
    if which == "wide":   # three 1024-px chunks, the last one ragged
        return synth.road(2100, 96, 41)
    # noise-only background: many tiles without edges
    return synth.gen_frame(synth.Scene(W=1100, H=120, n_lanes=3), 5)


def _mask(rng, kind, th, tw):
    if kind == "random":
        return rng.integers(0, 256, (th, tw))
    if kind == "ones":
        return np.full((th, tw), 255)
    if kind == "zeros":
        return np.zeros((th, tw))
    if kind == "sparse":
        return np.where(rng.random((th, tw)) < 0.1, 1 << rng.integers(0, 8, (th, tw)), 0)
    # runs of equal bytes of random length, some of them zero
    m = np.zeros((th, tw), np.int64)
    for y in range(th):
        x = 0
        while x < tw:
            n = int(rng.integers(1, 90))
            v = 0 if rng.random() < 0.3 else int(rng.integers(1, 256))
            m[y, x:x + n] = v
            x += n
    return m


@pytest.mark.parametrize("which,kind", [("640", "random"), ("640", "ones"), ("640", "zeros"),
                                        ("640", "sparse"), ("640", "runs"), ("wide", "runs"),
                                        ("wide", "random"), ("wide", "sparse"), ("quiet", "runs"),
                                        ("quiet", "ones")])
def test_vote_masked(lane, synth, oracle, which, kind):
    say("vote masked", which, kind)
    img = _masked_frame(synth, which)
    H, W = img.shape
    n_theta = 180 if which == "640" else 360
    C, S = synth.trig_q14(n_theta)
    D = synth.r_offset(W, H)
    e, _, _ = oracle.sobel_binarize(img, W, 128, 1)
    rng = np.random.default_rng(7)
    th, tw = (H + 7) // 8, (W + 7) // 8
    mask = _mask(rng, kind, th, tw).astype(np.uint8)
    a, d, a_o, d_o = vote_both(lane, oracle, e, W, H, C, S, D, 2 * D + 1, mask)
    assert (a == a_o).all() and d == d_o == 0
    if kind == "ones":
        plain, _, _ = oracle.hough_vote(e, C, S, D, 2 * D + 1)
        assert (a == plain).all()


def test_vote_masked_unusual_table(lane, synth, oracle):
    say("vote masked unusual")
    rng = np.random.default_rng(3)
    W, H, n_theta = 90, 50, 36
    e = np.where(rng.random((H, W)) < 0.3, 255, 0).astype(np.uint8)
    C = rng.integers(-32768, 32768, n_theta).astype(np.int16)
    S = rng.integers(-32768, 32768, n_theta).astype(np.int16)
    mask = rng.integers(0, 256, ((H + 7) // 8, (W + 7) // 8)).astype(np.uint8)
    a, d, a_o, d_o = vote_both(lane, oracle, e, W, H, C, S, 200, 401, mask)
    assert (a == a_o).all() and d == d_o


def peaks_both(lane, oracle, acc, D, k, ht=None, hr=None, mv=1):
    t, r, v, c = lane.hough_peaks(dev(acc), D, k, ht, hr, mv)
    to, ro, vo, no = oracle.hough_peaks(acc, D, k, ht, hr, mv)
    assert int(host(c)[0]) == no
    assert (host(t) == to).all() and (host(r) == ro).all() and (host(v) == vo).all()
    return no


@pytest.mark.parametrize("name,n_theta,k", [("plain_640", 180, 2), ("plain_1080", 360, 8)])
def test_peaks_frames(lane, synth, oracle, name, n_theta, k):
    say("peaks", name)
    img = FRAMES[name](synth)
    H, W = img.shape
    C, S = synth.trig_q14(n_theta)
    r = oracle.pipeline(img, C, S, k)
    assert peaks_both(lane, oracle, r["acc"], r["D"], k) == k
    assert peaks_both(lane, oracle, r["acc"], r["D"], 50, 0, 0) == 50
    assert peaks_both(lane, oracle, r["acc"], r["D"], 20, 10, 200, 300) >= 1


@pytest.mark.parametrize("seed", range(8))
def test_peaks_random_small(lane, oracle, seed):
    say("peaks random", seed)
    rng = np.random.default_rng(seed)
    n_theta, D = int(rng.integers(1, 40)), int(rng.integers(0, 30))
    acc = rng.integers(0, 4, size=(n_theta, 2 * D + 1)).astype(np.int32)  # many ties
    for k, ht, hr in ((1, 0, 0), (5, 1, 1), (12, 3, 2), (30, 0, 5), (7, 50, 1)):
        peaks_both(lane, oracle, acc, D, k, ht, hr)
    peaks_both(lane, oracle, np.zeros_like(acc), D, 3)


def test_peaks_large_blocks(lane, oracle):
    """An accumulator large enough that blocks hold more than 256 cells."""
    say("peaks large")
    rng = np.random.default_rng(5)
    n_theta, D = 700, 2000
    acc = rng.integers(0, 50, size=(n_theta, 2 * D + 1)).astype(np.int32)
    acc[350, 10] = 999
    acc[0, 3995] = 998
    peaks_both(lane, oracle, acc, D, 10)


@pytest.mark.parametrize("case", ["frame_k32", "frame_k200", "sparse", "flat", "dense_top",
                                  "floor_above", "wide_window"])
def test_peaks_candidate_branches(lane, synth, oracle, case):
    """The peak search first works on the cells at or above a count tau
    that only a few hundred blocks reach, and redoes the frame with the
    general search when that set runs out above the vote floor or is too
    large.  One case per way through: the set suffices (a 1080p frame,
    k = 32); it runs out above the floor (k = 200); it runs out at the
    floor (a few isolated cells); more blocks than allowed share the top
    count (a flat accumulator); the set holds too many cells (a band of
    rows at one high count); nothing reaches min_votes; a window wider
    than the half-turn."""
    say("peaks candidate branch", case)
    n_theta = 360
    if case.startswith("frame") or case == "wide_window":
        img = synth.plain_1080(3)
        C, S = synth.trig_q14(n_theta)
        r = oracle.pipeline(img, C, S, 8)
        acc, D = r["acc"], r["D"]
    else:
        D = 2202
        acc = np.zeros((n_theta, 2 * D + 1), np.int32)
    if case == "frame_k32":
        assert peaks_both(lane, oracle, acc, D, 32) == 32
    elif case == "frame_k200":
        assert peaks_both(lane, oracle, acc, D, 200) == 200
    elif case == "sparse":
        for j, (t, i) in enumerate([(5, 100), (90, 2000), (200, 4000), (359, 7), (180, 2202)]):
            acc[t, i] = 10 + j
        assert peaks_both(lane, oracle, acc, D, 8) == 5
    elif case == "flat":
        acc[:] = 7
        assert peaks_both(lane, oracle, acc, D, 8) == 8
    elif case == "dense_top":
        rng = np.random.default_rng(4)
        acc[:] = rng.integers(0, 20, acc.shape)
        acc[10:14, :] = 100
        assert peaks_both(lane, oracle, acc, D, 8) == 8
    elif case == "floor_above":
        assert peaks_both(lane, oracle, acc + 5, D, 8, mv=6) == 0
    else:
        assert peaks_both(lane, oracle, acc, D, 12, 200, 30) >= 1


@pytest.mark.parametrize("idx", [0, 16, 32, 48])
def test_pipeline_mixed_sizes(lane, synth, oracle, idx):
    sc, seed = synth.mixed_batch_scene(idx)
    say("pipeline mixed", idx, sc.W, sc.H)
    img = synth.gen_frame(sc, seed)
    C, S = synth.trig_q14(360)
    want = oracle.pipeline(img, C, S, 8)
    got = lane.pipeline(dev(img), dev(C), dev(S), 8)
    assert (host(got["edges"]) == want["edges"]).all()
    assert (host(got["acc"]) == want["acc"]).all()
    assert int(host(got["dropped"])[0]) == 0
    assert int(host(got["count"])[0]) == want["count"]
    assert (host(got["theta_idx"]) == want["theta_idx"]).all()
    assert (host(got["r_idx"]) == want["r_idx"]).all()
    assert (host(got["votes"]) == want["votes"]).all()


def test_deterministic_repeat(lane, synth):
    say("determinism")
    img = dev(synth.plain_1080(2))
    C, S = synth.trig_q14(360)
    a = lane.pipeline(img, dev(C), dev(S), 8)
    b = lane.pipeline(img, dev(C), dev(S), 8)
    assert torch.equal(a["acc"], b["acc"]) and torch.equal(a["edges"], b["edges"])
    assert torch.equal(a["theta_idx"], b["theta_idx"]) and torch.equal(a["votes"], b["votes"])


def test_max_size_frame(lane, synth, oracle):
    """8192 x 8192, the largest frame the ABI accepts."""
    say("max size 8192x8192")
    rng = np.random.default_rng(1)
    W = H = 8192
    e = np.where(rng.random((H, W)) < 0.004, 255, 0).astype(np.uint8)
    C, S = synth.trig_q14(180)
    D = synth.r_offset(W, H)
    a, d, a_o, d_o = vote_both(lane, oracle, e, W, H, C, S, D, 2 * D + 1)
    assert d == d_o == 0 and (a == a_o).all()
    img = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    e_o, m_o, n_o = oracle.sobel_binarize(img, W, 250, 1)
    eg, mg, lst, cnt = lane.sobel_binarize(dev(img), W, 250, 1, want_mag=True)
    assert (host(eg) == e_o).all() and (host(mg) == m_o).all() and int(host(cnt)[0]) == n_o
