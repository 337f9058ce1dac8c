"""Batched plans (one HIP graph per launch) against the CPU oracle: every
frame's outputs in a mixed batch equal the oracle's, bit-exactly, on every
replay of the graph, with eager work between the replays."""
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


def say(*a):
    print("[case]", *a, flush=True)


def make_frames(lane, synth, oracle, specs, n_theta=360, k=8):
    frames, wants = [], []
    C, S = synth.trig_q14(n_theta)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    for (Wf, Hf, pitch, seed, masked) in specs:
        img = synth.gen_frame(synth.scene_road(Wf, Hf), seed, pitch=pitch)
        mask = None
        if masked:
            rng = np.random.default_rng(seed)
            mask = rng.integers(0, 256, ((Hf + 7) // 8, (Wf + 7) // 8)).astype(np.uint8)
        fb = lane.FrameBuffers(torch.from_numpy(img).cuda(), Wf, n_theta, k, Cd, Sd,
                               tile_mask=None if mask is None else torch.from_numpy(mask).cuda())
        frames.append(fb)
        want = oracle.pipeline(img[:, :Wf].copy(), C, S, k, tile_mask=mask)
        wants.append(want)
    return frames, wants


def check(frames, wants):
    torch.cuda.synchronize()
    for i, (f, w) in enumerate(zip(frames, wants)):
        assert (f.edges.cpu().numpy() == w["edges"]).all(), i
        assert (f.acc.cpu().numpy() == w["acc"]).all(), i
        c = f.counters.cpu().numpy()
        assert int(c[0]) == w["n_edges"] and int(c[1]) == w["dropped"], i
        assert int(f.count().cpu()) == w["count"], i
        assert (f.theta_idx().cpu().numpy() == w["theta_idx"]).all(), i
        assert (f.r_idx().cpu().numpy() == w["r_idx"]).all(), i
        assert (f.votes().cpu().numpy() == w["votes"]).all(), i


def scribble(frames):
    for f in frames:
        f.edges.fill_(3)
        f.acc.fill_(-7)
        f.peaks.fill_(-5)
        f.counters.fill_(99)
        f.edge_list.fill_(0x7FFF7FFF)


@pytest.mark.parametrize("queue", [-1, 0, 1, 2])
def test_mixed_batch_graph_replays(lane, synth, oracle, queue):
    say("mixed batch queue", queue)
    specs = [(640, 480, 640, 11, False), (1280, 720, 1280, 12, False), (1920, 1080, 1920, 13, False),
             (3840, 2160, 3840, 14, False), (997, 41, 1000, 15, False), (33, 17, 33, 16, False),
             (640, 480, 640, 17, True), (1920, 1080, 1920, 18, True)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, vote_queue=queue)
    for rep in range(3):
        say("replay", rep)
        b.launch()
        check(frames, wants)
        scribble(frames)
        torch.cuda.synchronize()
    b.launch()
    check(frames, wants)
    b.close()


def test_same_size_static_and_stages(lane, synth, oracle):
    say("same-size static")
    specs = [(640, 480, 640, 100 + i, False) for i in range(12)]
    frames, wants = make_frames(lane, synth, oracle, specs, n_theta=180, k=2)
    b = lane.Batch(frames, vote_queue=0)
    b.launch()
    check(frames, wants)
    scribble(frames)
    for st in range(4):
        b.launch_stage(st)
    check(frames, wants)
    b.close()


@pytest.mark.parametrize("rows", [1, 2, 4, 8, 16, 32, 64])
def test_vote_rows_override(lane, synth, oracle, rows):
    say("vote rows", rows)
    specs = [(1280, 720, 1280, 7, False), (640, 480, 640, 8, True)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, vote_rows=rows)
    b.launch()
    check(frames, wants)
    b.close()


@pytest.mark.parametrize("rows", [4, 8])
def test_vote_paired_cells_dense_edges(lane, synth, oracle, rows):
    """Every interior pixel an edge (columns 0, 0, 255, 255 repeating) on a
    4094 x 4094 frame.  With 16 angles the slices around 45 degrees span
    about 5800 r cells, too wide for one word per cell at 4 or 8 rows, so the
    paired layout votes them (the Q14 rows there bound a cell pair by
    3 x 4094 = 12282 < 2^14 pixels); a cell pair gets about 11600 votes."""
    W = H = 4094
    say("paired cells, dense edges", W, H, "rows", rows)
    img = np.tile(np.array([0, 0, 255, 255], np.uint8), (H, W // 4 + 1))[:, :W].copy()
    C, S = synth.trig_q14(16)
    want = oracle.pipeline(img, C, S, 4)
    assert want["n_edges"] == (W - 2) * (H - 2)
    assert want["acc"].max() > 5000
    fb = lane.FrameBuffers(torch.from_numpy(img).cuda(), W, 16, 4, torch.from_numpy(C).cuda(),
                           torch.from_numpy(S).cuda())
    b = lane.Batch([fb], vote_rows=rows)
    b.launch()
    check([fb], [want])
    b.close()


def test_batch_matches_single_frame_calls(lane, synth):
    """A frame gives the same bytes alone (single-frame entry points) and in
    a batch."""
    say("alone == in batch")
    img = torch.from_numpy(synth.plain_1080(5)).cuda()
    C, S = synth.trig_q14(360)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    alone = lane.pipeline(img, Cd, Sd, 8)
    others = [lane.FrameBuffers(torch.from_numpy(synth.road(1280, 720, 900 + i)).cuda(), None,
                                360, 8, Cd, Sd) for i in range(3)]
    fb = lane.FrameBuffers(img, None, 360, 8, Cd, Sd)
    b = lane.Batch(others[:2] + [fb] + others[2:])
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(fb.acc, alone["acc"]) and torch.equal(fb.edges, alone["edges"])
    assert torch.equal(fb.theta_idx(), alone["theta_idx"]) and torch.equal(fb.votes(), alone["votes"])
    b.close()


def test_autotuner_choice_is_valid_and_exact(lane, synth, oracle):
    """The tuner returns a setting within its search space, and a plan built
    with it gives the oracle's results."""
    say("autotuner")
    from paper_2212_09460_amd import tune as tuner

    img = torch.from_numpy(synth.road(1280, 720, 4242)).cuda()
    t, info = tuner.tuned(img, 360, 4, use_cache=False)
    assert t.vote_rows in (1, 2, 4, 8, 16, 32, 64) and t.vote_queue in (0, 1, 2)
    assert t.sobel_strip_rows in (8, 16, 24, 32, 64, 128) and t.sobel_groups_per_cu in (0, 1, 2)
    assert info["vote_ms"] > 0 and info["sobel_ms"] > 0
    specs = [(1280, 720, 1280, 50 + i, False) for i in range(3)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, tune=t)
    b.launch()
    check(frames, wants)
    b.close()


@pytest.mark.parametrize("strip", [8, 16, 64, 128])
def test_sobel_strip_heights(lane, synth, oracle, strip):
    say("strip", strip)
    specs = [(640, 480, 640, 70, False), (997, 41, 1000, 71, False), (1280, 720, 1280, 72, True)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, sobel_strip_rows=strip, sobel_groups_per_cu=1)
    b.launch()
    check(frames, wants)
    b.close()


@pytest.mark.parametrize("queue", [1, 0, 2])
def test_select_runs_only_selected_frames(lane, synth, oracle, queue):
    """lane_batch_select: selected frames are computed from their current
    images, the others keep every output and counter untouched; a later
    selection of all frames computes everything again (graph replays)."""
    say("select", queue)
    specs = [(640, 480, 640, 21, False), (1280, 720, 1280, 22, False), (333, 211, 352, 23, True),
             (1920, 1080, 1920, 24, False), (640, 480, 640, 25, True)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, vote_rows=2, vote_queue=queue, sobel_strip_rows=8)
    b.launch()
    check(frames, wants)
    # new images for the selected frames 0, 2, 3; sentinels in the others
    sel = [1, 0, 1, 1, 0]
    new_wants = list(wants)
    C, S = synth.trig_q14(360)
    for i in (0, 2, 3):
        Wf, Hf, pitch, seed, masked = specs[i]
        img = synth.gen_frame(synth.scene_road(Wf, Hf), seed + 100, pitch=pitch)
        frames[i].img.copy_(torch.from_numpy(img))
        mask = frames[i].tile_mask.cpu().numpy() if masked else None
        new_wants[i] = oracle.pipeline(img[:, :Wf].copy(), C, S, 8, tile_mask=mask)
    for i in (1, 4):
        frames[i].edges.fill_(3)
        frames[i].acc.fill_(-7)
        frames[i].peaks.fill_(-5)
        frames[i].counters.fill_(11)
    b.select(sel)
    for rep in range(2):
        b.launch()
        torch.cuda.synchronize()
        check([frames[i] for i in (0, 2, 3)], [new_wants[i] for i in (0, 2, 3)])
        for i in (1, 4):
            assert (frames[i].edges == 3).all() and (frames[i].acc == -7).all()
            assert (frames[i].peaks == -5).all() and (frames[i].counters == 11).all()
    b.select([1] * 5)
    b.launch()
    check(frames, new_wants)
    b.close()


@pytest.mark.parametrize("rows,split,queue", [(1, 2, 1), (4, 4, 1), (16, 3, 0), (2, 8, 1), (8, 64, 1), (4, 8, 2)])
def test_vote_split(lane, synth, oracle, rows, split, queue):
    """Edge-split vote: several workgroups per slice, each adding its share
    of the rows into the accumulator the plan clears first; exact on every
    replay (the clear and the vote's queue restart in every pass)."""
    say("vote split", rows, split, queue)
    specs = [(1280, 720, 1280, 31, False), (640, 480, 640, 32, True), (1100, 200, 1104, 33, False)]
    frames, wants = make_frames(lane, synth, oracle, specs)
    b = lane.Batch(frames, vote_rows=rows, vote_split=split, vote_queue=queue)
    for rep in range(3):
        scribble(frames)
        b.launch()
        check(frames, wants)
    b.close()


def test_vote_split_with_fallback_rows(lane, synth, oracle):
    """A table whose row leaves the accumulator sends that slice down the
    exact global-atomic path, which runs unsplit in the slice's first part."""
    say("vote split + fallback")
    W, H = 640, 480
    img = synth.road(W, H, 61)
    C, S = synth.trig_q14(360)
    C = C.copy()
    C[5] = 32767
    D = synth.r_offset(W, H)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    fb = lane.FrameBuffers(torch.from_numpy(img).cuda(), W, 360, 8, Cd, Sd)
    want = oracle.pipeline(img, C, S, 8)
    b = lane.Batch([fb], vote_rows=4, vote_split=4, vote_queue=1)
    for rep in range(2):
        scribble([fb])
        b.launch()
        torch.cuda.synchronize()
        assert (fb.acc.cpu().numpy() == want["acc"]).all()
        assert int(fb.counters.cpu().numpy()[1]) == want["dropped"] > 0
        assert (fb.theta_idx().cpu().numpy() == want["theta_idx"]).all()
    b.close()


def proposal_like_mask(rng, Hf, Wf, keep=0.07, restricted=0.01):
    """Tile masks shaped like the proposal network's: most tiles skipped
    (0), some voting every row (0xFF), a few restricted to some bands."""
    th, tw = (Hf + 7) // 8, (Wf + 7) // 8
    r = rng.random((th, tw))
    m = np.zeros((th, tw), np.uint8)
    m[r < keep] = 0xFF
    sel = (r >= keep) & (r < keep + restricted)
    m[sel] = rng.integers(1, 255, int(sel.sum()))
    return m


@pytest.mark.parametrize("rows,split,queue", [(4, 8, 1), (16, 2, 0), (1, 64, 1)])
def test_split_vote_pruned_lists(lane, synth, oracle, rows, split, queue):
    """Masked frames in a split plan vote from pruned copies of their edge
    lists (tiles that vote every row) plus a pass over the band-restricted
    tiles: exact on every replay, frames switched off keep their outputs,
    and mask contents changed between launches take effect."""
    say("split vote pruned lists", rows, split, queue)
    rng = np.random.default_rng(rows * 100 + split)
    C, S = synth.trig_q14(360)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    specs = [(1920, 1080, 1920, 81), (1280, 720, 1280, 82), (333, 211, 352, 83), (3840, 2160, 3840, 84)]
    frames, wants, masks = [], [], []
    for (Wf, Hf, pitch, seed) in specs:
        img = synth.gen_frame(synth.scene_road(Wf, Hf), seed, pitch=pitch)
        m = proposal_like_mask(rng, Hf, Wf)
        masks.append(m)
        frames.append(lane.FrameBuffers(torch.from_numpy(img).cuda(), Wf, 360, 8, Cd, Sd,
                                        tile_mask=torch.from_numpy(m).cuda()))
        wants.append(oracle.pipeline(img[:, :Wf].copy(), C, S, 8, tile_mask=m))
    # one unmasked frame in the same plan
    img = synth.gen_frame(synth.scene_road(640, 480), 85)
    frames.append(lane.FrameBuffers(torch.from_numpy(img).cuda(), 640, 360, 8, Cd, Sd))
    wants.append(oracle.pipeline(img, C, S, 8))
    b = lane.Batch(frames, vote_rows=rows, vote_split=split, vote_queue=queue)
    for rep in range(2):
        scribble(frames)
        b.launch()
        check(frames, wants)
    # new masks for frames 0 and 2 (every tile restricted in frame 2), frame 1 off
    masks[0] = proposal_like_mask(rng, 1080, 1920, keep=0.2, restricted=0.05)
    masks[2] = rng.integers(1, 255, masks[2].shape).astype(np.uint8)
    for i in (0, 2):
        frames[i].tile_mask.copy_(torch.from_numpy(masks[i]))
        Wf, Hf, pitch, seed = specs[i]
        img = frames[i].img.cpu().numpy()[:, :Wf].copy()
        wants[i] = oracle.pipeline(img, C, S, 8, tile_mask=masks[i])
    frames[1].acc.fill_(-7)
    frames[1].peaks.fill_(-5)
    b.select([1, 0, 1, 1, 1])
    b.launch()
    torch.cuda.synchronize()
    check([frames[i] for i in (0, 2, 3, 4)], [wants[i] for i in (0, 2, 3, 4)])
    assert (frames[1].acc == -7).all() and (frames[1].peaks == -5).all()
    b.close()


def small_table(n, q):
    """Rows of cos/sin rounded to q fractional bits (q = 0: C = S = 1)."""
    if q == 0:
        return np.ones(n, np.int16), np.ones(n, np.int16)
    a = np.arange(n) * np.pi / n
    return (np.round(np.cos(a) * 2 ** q).astype(np.int16),
            np.round(np.sin(a) * 2 ** q).astype(np.int16))


@pytest.mark.parametrize("rows", [32, 64])
@pytest.mark.parametrize("q", [8, 6, 0])
def test_vote_small_tables_many_rows(lane, synth, oracle, q, rows):
    """Tables with small entries (Q8, Q6, C = S = 1) put thousands of pixels
    in neighbouring r cells; at 32 and 64 rows per workgroup a slice must not
    take the paired counters then (their 14-bit pair sum would wrap).  A road
    frame at 640 x 480 and a dense 200 x 200 frame (every interior pixel an
    edge), bit-exact against the oracle."""
    say("small table q", q, "rows", rows)
    n = 360
    C, S = small_table(n, q)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    road = synth.road(640, 480, 7)
    dense = np.tile(np.array([0, 0, 255, 255], np.uint8), (200, 50)).copy()
    frames, wants = [], []
    for img in (road, dense):
        H, W = img.shape
        frames.append(lane.FrameBuffers(torch.from_numpy(img).cuda(), W, n, 8, Cd, Sd))
        wants.append(oracle.pipeline(img, C, S, 8))
    pair = max(int((w["acc"][:, :-1].astype(np.int64) + w["acc"][:, 1:]).max()) for w in wants)
    assert pair > 16383
    b = lane.Batch(frames, vote_rows=rows)
    for rep in range(2):
        scribble(frames)
        b.launch()
        check(frames, wants)
    b.close()


def test_mixed_batch_64_frames_tuned(lane, synth, oracle):
    """The mixed-resolution batch as specified: 64 frames, 16 each at 640x480,
    1280x720, 1920x1080 and 3840x2160 with 2..6 lanes, 360 angles, top-8, in
    one plan whose setting comes from the autotuner run on these frames
    (lane_tune_batch); every frame bit-exact against the oracle on two graph
    replays with the outputs scribbled between them."""
    from concurrent.futures import ThreadPoolExecutor

    say("mixed batch 64 frames: generate, oracle")
    imgs = [synth.mixed_batch(i) for i in range(64)]
    assert sorted({im.shape for im in imgs}) == [(480, 640), (720, 1280), (1080, 1920), (2160, 3840)]
    C, S = synth.trig_q14(360)
    with ThreadPoolExecutor(max_workers=16) as ex:
        wants = list(ex.map(lambda im: oracle.pipeline(im, C, S, 8), imgs))
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    frames = [lane.FrameBuffers(torch.from_numpy(im).cuda(), im.shape[1], 360, 8, Cd, Sd)
              for im in imgs]
    say("mixed batch 64 frames: tune")
    t, vote_ms, sobel_ms = lane.tune_batch(frames)
    assert t.vote_rows in (0, 1, 2, 4, 8, 16, 32, 64) and t.vote_queue in (0, 1, 2)
    assert t.sobel_strip_rows in (8, 16, 24, 32, 64, 128) and t.sobel_groups_per_cu in (0, 1, 2)
    assert vote_ms > 0 and sobel_ms > 0
    b = lane.Batch(frames, tune=t)
    for rep in range(2):
        say("mixed batch 64 frames: replay", rep, lane.tune_dict(t))
        scribble(frames)
        b.launch()
        check(frames, wants)
    b.close()


def test_sobel_list_stages_agree(lane, synth, oracle):
    """A frame whose tile rows hold up to 8192 edges (every pass count of
    both list stages) gives the oracle's edge map, count and accumulator in
    a plan of few frames (the large list stage) and in one of many (the
    small one)."""
    say("sobel list stages")
    C, S = synth.trig_q14(360)
    Cd, Sd = torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda()
    rng = np.random.default_rng(4242)
    W, H = 1100, 64
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    img[:, 512:600] = 0  # flat band: tile rows of every density
    want = oracle.pipeline(img, C, S, 8, threshold=40)
    assert want["n_edges"] > 0.6 * W * H
    road = synth.gen_frame(synth.scene_road(1920, 1080), 77)
    want_road = oracle.pipeline(road, C, S, 8)
    for n_road in (0, 8):  # 8 1080p frames: more items than one round of the large stage
        fb = lane.FrameBuffers(torch.from_numpy(img).cuda(), W, 360, 8, Cd, Sd, threshold=40)
        others = [lane.FrameBuffers(torch.from_numpy(road).cuda(), 1920, 360, 8, Cd, Sd)
                  for _ in range(n_road)]
        b = lane.Batch([fb] + others, vote_rows=16)
        for rep in range(2):
            scribble([fb] + others)
            b.launch()
            check([fb] + others, [want] + [want_road] * n_road)
        b.close()
