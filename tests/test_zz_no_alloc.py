"""lane_hough_peaks_noalloc (the peak search on the library's fixed device
scratch, for callers that cannot allocate) against lane_hough_peaks with a
caller workspace: bit-exact on two calls in a row, the second on a smaller
accumulator, and on a third that needs the whole scratch array; the plain
call's result is checked against the oracle as well."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _road_acc(synth, oracle, W, H, n_theta, seed):
    img = synth.plain_640(seed) if (W, H) == (640, 480) else synth.plain_1080(seed)
    C, S = synth.trig_q14(n_theta)
    edges = oracle.sobel_binarize(img, border_mode=1)[0]
    D = oracle.r_offset(W, H)
    acc = oracle.hough_vote(edges, C, S, D, 2 * D + 1)[0]
    return acc, D


def _check_pair(lane, acc_np, D, k, **kw):
    dev = torch.device("cuda:0")
    acc = torch.from_numpy(np.ascontiguousarray(acc_np)).to(dev)
    want = [t.cpu().numpy() for t in lane.hough_peaks(acc, D, k, **kw)]
    got = [t.cpu().numpy() for t in lane.hough_peaks_noalloc(acc, D, k, **kw)]
    torch.cuda.synchronize()
    for w, g, name in zip(want, got, ("theta_idx", "r_idx", "votes", "count")):
        assert np.array_equal(w, g), name
    return want


def test_noalloc_peaks_equal_workspace_peaks(synth, oracle):
    import paper_2212_09460_amd.lane as lane

    assert lane.peaks_noalloc_max_bytes() == 65536
    # first call: a 1920x1080 frame at 360 angles, top 8
    print("noalloc: 1920x1080, 360 theta, k=8", flush=True)
    acc1, D1 = _road_acc(synth, oracle, 1920, 1080, 360, 3)
    want = _check_pair(lane, acc1, D1, 8)
    o = oracle.hough_peaks(acc1, D1, 8)
    assert np.array_equal(want[0], o[0]) and np.array_equal(want[1], o[1])
    assert np.array_equal(want[2], o[2])
    # second call, smaller: 640x480 at 180 angles, top 2 (keys of the first
    # call are still in the scratch array beyond this one's blocks)
    print("noalloc: 640x480, 180 theta, k=2", flush=True)
    acc2, D2 = _road_acc(synth, oracle, 640, 480, 180, 0)
    want = _check_pair(lane, acc2, D2, 2)
    o = oracle.hough_peaks(acc2, D2, 2)
    assert np.array_equal(want[0], o[0]) and np.array_equal(want[1], o[1])
    # random accumulators with ties, down to one row, and one at the block
    # limit of the search (8192 key blocks, the whole scratch array)
    rng = np.random.default_rng(7)
    for n_theta, D, k in ((361, 4000, 16), (1, 3, 4), (7, 40, 3), (4096, 63, 5)):
        print("noalloc: random %d x %d, k=%d" % (n_theta, 2 * D + 1, k), flush=True)
        acc = rng.integers(0, 50, size=(n_theta, 2 * D + 1), dtype=np.int32)
        _check_pair(lane, acc, D, k)
        _check_pair(lane, acc, D, k, h_theta=0, h_r=0, min_votes=49)
