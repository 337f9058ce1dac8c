"""Host-side pieces of bench.py: the one-GPU guard and the all-cores oracle
leg (worker processes started together), run on the CPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_all_cores_oracle_leg():
    sys.path.insert(0, ROOT)
    import bench

    r = bench.cpu_all_cores(2, 0.2)
    assert r["cores"] == 2 and r["unit"] == "Mpix/s"
    # each worker finishes at least one frame after the go line
    assert r["frames_per_s"] > 0 and r["value"] > 0
    assert "2 single-threaded oracle processes" in r["sample"]


def test_mixed_oracle_worker_and_check():
    """The mixed-batch oracle worker reports per-frame results that the check
    accepts for identical GPU outputs and rejects for a changed peak or a
    changed accumulator."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench

    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--oracle-mixed-worker", "0,1"]
    res = bench.run_workers([cmd], dict(os.environ, OMP_NUM_THREADS="1"))
    frames = res[0]["frames"]
    assert [f["i"] for f in frames] == [0, 1] and res[0]["seconds"] > 0
    k = bench.TOPK
    gpu = {}
    for f in frames:
        pk = np.array(f["theta_idx"] + f["r_idx"] + f["votes"] + [f["count"]], np.int32)
        gpu[f["i"]] = {"acc_sha": f["acc_sha"], "peaks": pk,
                       "counters": np.array([f["n_edges"], f["dropped"]], np.int32)}
    assert bench.check_mixed(frames, gpu)["ok"]
    gpu[1]["peaks"] = gpu[1]["peaks"].copy()
    gpu[1]["peaks"][k] += 1
    r = bench.check_mixed(frames, gpu)
    assert not r["ok"] and r["mismatched_frames"] == [1]
    gpu[1]["peaks"][k] -= 1
    gpu[0]["acc_sha"] = "0" * 64
    assert bench.check_mixed(frames, gpu)["mismatched_frames"] == [0]


def test_plan_check_covers_every_frame():
    """check_plan_256 compares every plan frame with the oracle result of its
    pool frame and the first POOL accumulators in full."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench

    k, P = bench.TOPK, bench.POOL
    rng = np.random.default_rng(1)
    ref = {}
    for j in range(P):
        ref[j] = {"count": 3, "theta_idx": rng.integers(0, 360, k).astype(np.int32),
                  "r_idx": rng.integers(0, 999, k).astype(np.int32),
                  "votes": rng.integers(0, 99, k).astype(np.int32), "n_edges": int(j),
                  "dropped": 0, "acc": rng.integers(0, 9, (4, 5)).astype(np.int32)}
    n = 3 * P
    peaks = np.stack([np.concatenate([ref[i % P]["theta_idx"], ref[i % P]["r_idx"],
                                      ref[i % P]["votes"], [3]]) for i in range(n)])
    counters = np.array([[i % P, 0] for i in range(n)], np.int32)
    gpu = {"peaks": peaks, "counters": counters, "acc": [ref[j]["acc"].copy() for j in range(P)]}
    r = bench.check_plan_256(ref, gpu)
    assert r["ok"] and r["frames_peaks_checked"] == n and r["accumulators_checked"] == P
    gpu["peaks"][2 * P + 5, 2 * k] += 1          # a late frame's votes
    gpu["acc"][3][1, 2] += 1                     # an early frame's accumulator
    r = bench.check_plan_256(ref, gpu)
    assert not r["ok"] and r["mismatched_frames"] == [3, 2 * P + 5]


def test_openmp_oracle_leg_matches_single_thread():
    """The oracle's OpenMP build (the multi-core baseline) in two threads
    gives the single-threaded accumulator on the workload's first frame."""
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from paper_2212_09460_amd import synth

    img = synth.gen_frame(synth.scene_road(bench.W, bench.H),
                          synth.frame_seed(0, synth.CONFIG_PLAIN_1080, 0))
    C, S = synth.trig_q14(bench.N_THETA)
    ref = oracle.pipeline(img, C, S, bench.TOPK)
    r = bench.cpu_openmp(2, 0.1, ref)
    assert r["cores"] == 2 and r["value"] > 0 and r["same_result"] is True


def test_lds_probe_rejects_bad_arguments():
    """The probe's argument checks come before any HIP call (CPU only)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2212_09460_amd", "liblaneprobe.so"))
    f = lib.lane_probe_lds_add
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_uint64)]
    rate, chk = ctypes.c_double(0.0), ctypes.c_uint64(0)
    for args in ((0, 1, 0), (1, 0, 0), (1, 1, 3), (1, 1, -1), (70000, 1, 0)):
        assert f(*args, ctypes.byref(rate), ctypes.byref(chk)) == -1
    assert f(1, 1, 0, None, ctypes.byref(chk)) == -1


def test_cnn_flops_match_the_oracle_layer_shapes():
    """The proposal network's FLOP count used for its roofline equals
    2 x (output pixels x c_out x c_in x 9) summed over the oracle's layers,
    with the output shapes the oracle's forward pass produces."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    from oracle import cnn as ocnn
    rng = np.random.default_rng(3)
    params = ocnn.unflatten(rng.standard_normal(6105) * 0.1)
    for W, H in ((16, 16), (37, 21), (1920, 1080)):
        img = np.zeros((H, W), np.uint8) if W * H > 100000 else rng.integers(0, 256, (H, W)).astype(np.uint8)
        if W * H > 100000:
            # shapes only: the layers' outputs of a strided 3x3 with padding 1
            shapes, h, w = [], H, W
            for (_, _, s, _) in ocnn.LAYERS:
                h, w = (h + s - 1) // s, (w + s - 1) // s
                shapes.append((h, w))
        else:
            _, acts = ocnn.forward(img, params)
            shapes = [a.shape[1:] for a in acts[1:]]
        want = 0
        for (h, w), (wt, _) in zip(shapes, params):
            c_out, c_in = wt.shape[0], wt.shape[1]
            want += 2 * h * w * c_out * c_in * 9
        assert bench.cnn_flops(W, H) == want, (W, H)
