"""Serving host logic without a GPU: the arrival schedule, HBM-budget
admission, argument checks, and failure paths that return before (or
instead of) touching a device."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lane():
    import paper_2212_09460_amd.lane as m

    return m


@pytest.fixture(scope="module")
def serve():
    import paper_2212_09460_amd.serve as m

    return m


def test_schedule_deterministic_sorted_and_rate(serve):
    a = serve.poisson_schedule(16, 30.0, 20.0, seed=3)
    b = serve.poisson_schedule(16, 30.0, 20.0, seed=3)
    assert all((x == y).all() for x, y in zip(a, b))
    t, s, k = a
    assert (np.diff(t) >= 0).all() and t.min() > 0 and t.max() < 20.0
    # 16 streams x 30 Hz x 20 s = 9600 arrivals expected, sd ~ 98
    assert abs(len(t) - 9600) < 5 * 98
    for st in range(16):
        ks = k[s == st]
        assert (ks == np.arange(len(ks))).all()      # per-stream frame index counts up
        gaps = np.diff(np.concatenate([[0.0], t[s == st]]))
        assert abs(gaps.mean() - 1 / 30) < 0.2 / 30  # exponential gaps, mean 1/rate
    c = serve.poisson_schedule(16, 30.0, 20.0, seed=4)
    assert len(c[0]) != len(t) or not (c[0] == t).all()


def test_mix_matches_workload(serve):
    st = serve.mix_streams()
    sizes = [(s["W"], s["H"]) for s in st]
    assert sizes.count((1280, 720)) == 8 and sizes.count((1920, 1080)) == 6
    assert sizes.count((3840, 2160)) == 2
    px = sum(w * h for w, h in sizes) * 30
    assert abs(px / 1e9 - 1.09) < 0.01


def test_admission_in_order_within_budget(lane, serve):
    st = serve.mix_streams()
    adm, sb, tot = lane.server_plan(st, 8 << 30)
    assert all(adm) and tot == sum(sb)
    # a budget that holds exactly the first five streams admits those five;
    # later streams that would fit are still admitted (greedy, in order)
    b5 = sum(sb[:5])
    adm, sb2, tot = lane.server_plan(st, b5)
    assert adm[:5] == [True] * 5 and tot <= b5
    assert sb2[:5] == sb[:5]
    adm, _, tot = lane.server_plan(st, 0)
    assert not any(adm) and tot == 0
    # a small stream after a rejected large one is admitted
    mixed = [dict(W=3840, H=2160), dict(W=320, H=240)]
    _, alone, _ = lane.server_plan(mixed[1:], 1 << 40)
    adm, _, _ = lane.server_plan(mixed, alone[0])
    assert adm == [False, True]


def test_admission_pruned_counts_network_state(lane, serve):
    st = serve.mix_streams()
    p = np.zeros(lane.CNN_PARAMS, np.float32)
    _, plain, _ = lane.server_plan(st, 8 << 30)
    _, pruned, tot = lane.server_plan(st, 8 << 30, pruned=True, cnn_params=p)
    assert all(b > a for a, b in zip(plain, pruned))
    assert tot > sum(pruned) - 1  # shared weights on top of the streams
    # per stream, the pruned state adds the tile mask, the logits and (the
    # vote being split) the pruned copy of the edge list the plan allocates
    # (one per refill lane: two by default)
    al = lambda v: (v + 255) // 256 * 256
    _, pruned1, _ = lane.server_plan(st, 8 << 30, pruned=True, cnn_params=p, lanes=1)
    _, plain3, _ = lane.server_plan(st, 8 << 30, lanes=3)
    assert plain3 == plain  # the plain path's plans hold no per-stream state
    for s_, a, b, b1 in zip(st, plain, pruned, pruned1):
        th, tw = (s_["H"] + 7) // 8, (s_["W"] + 7) // 8
        lst = al(lane.edge_list_size(s_["W"], s_["H"]))
        extra = al(th * tw) + al(4 * 9 * th * tw)
        assert b - a == extra + 2 * lst and b1 - a == extra + lst


@pytest.mark.parametrize("kw,code", [
    (dict(vote_rows=3), -1), (dict(max_pending=0), -1), (dict(sobel_strip_rows=12), -1),
    (dict(pruned=True, conf=0.4), -1), (dict(pruned=True), -1),  # no weights
    (dict(lanes=-1), -1), (dict(lanes=5), -1), (dict(spin_us=-1), -1), (dict(spin_us=10 ** 7 + 1), -1),
])
def test_plan_rejects_bad_config(lane, kw, code):
    args = dict(hbm_budget=1 << 30)
    args.update(kw)
    if kw.get("pruned") and "conf" in kw:
        args["cnn_params"] = np.zeros(lane.CNN_PARAMS, np.float32)
    with pytest.raises(lane.LaneError) as e:
        lane.server_plan([dict(W=64, H=64)], **args)
    assert e.value.code == code


@pytest.mark.parametrize("st,code", [
    (dict(W=0, H=4), -1), (dict(W=9000, H=4), -2), (dict(W=64, H=64, k=65), -1),
    (dict(W=64, H=64, n_theta=9000), -2), (dict(W=64, H=64, border_mode=7), -6),
])
def test_plan_rejects_bad_stream(lane, st, code):
    with pytest.raises(lane.LaneError) as e:
        lane.server_plan([st], 1 << 30)
    assert e.value.code == code
    p = np.zeros(lane.CNN_PARAMS, np.float32)
    with pytest.raises(lane.LaneError) as e:  # pruned needs n_theta % 4 == 0
        lane.server_plan([dict(W=64, H=64, n_theta=90)], 1 << 30, pruned=True, cnn_params=p)
    assert e.value.code == -6


def test_null_handles_rejected(lane):
    lib = lane._lib
    out = (lane.Result * 2)()
    n = ctypes.c_int32(0)
    assert lib.lane_server_submit(None, 0, None, 0, ctypes.c_uint64(0)) == -1
    assert lib.lane_server_poll(None, out, 2, 0, ctypes.byref(n)) == -1
    assert lib.lane_server_replay(None, None, 1, out) == -1
    assert lib.lane_server_destroy(None) == -1
    assert lib.lane_batch_active_flags(None, None) == -1


def test_create_fails_cleanly_without_budget_or_device(lane):
    with pytest.raises(lane.LaneError) as e:  # nothing fits: refused before any device call
        lane.Server([dict(W=64, H=64)], hbm_budget=16)
    assert e.value.code == -4
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(lane.LaneError) as e:  # no device: an error, not a crash
        lane.Server([dict(W=64, H=64)], hbm_budget=1 << 30)
    assert e.value.code == -5


def test_host_frames_are_checked_before_submission(lane):
    """The binding refuses frames the server could not read as uint8 rows."""
    ok = np.zeros((4, 8), np.uint8)
    assert lane._host_frame(ok) is ok
    assert lane._host_frame(np.zeros((4, 16), np.uint8)[:, :8]) is not None  # pitch 16, W 8
    with pytest.raises(TypeError):
        lane._host_frame(np.zeros((4, 8), np.int16))
    with pytest.raises(TypeError):
        lane._host_frame(np.zeros((2, 4, 8), np.uint8))
    with pytest.raises(ValueError):
        lane._host_frame(np.zeros((8, 4), np.uint8).T)                     # columns not contiguous


def test_deadline_must_not_be_negative(lane, serve):
    st = serve.mix_streams()[:2]
    cfg, _ = lane._server_cfg(1 << 30, False, 0.9, None, 4, 0, 0, 0, deadline_ms=-1.0)
    arr = lane._stream_cfgs(st)
    rc = lane._srv_plan(arr, len(st), ctypes.byref(cfg), None, None, None)
    assert rc == -1  # LANE_E_ARG
