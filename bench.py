"""Benchmark of the lane-detection hot path on one MI355X.

A step is one pass of the whole path -- Sobel + binarize + compaction, Hough
vote, peaks -- over a batch of seeded synthetic 1920x1080 road frames (4
lanes with the inner two dashed, 200 clutter segments, 2 % salt, threshold
128, 360 theta bins, r step 1 px, top-8 peaks), launched as one HIP graph.
The frames are resident in HBM before the timed region starts.

Prints one JSON line with the throughput (Mpix/s; frames/s beside it), the
roofline of the dominant kernel (the vote, LDS-atomic bound) measured live
with HIP events on the launch stream beside the rate of a conflict-free LDS
increment probe, the Sobel pass's HBM roofline, single-frame latency, the
mixed-resolution batch (64 frames, 16 each at 640x480, 1280x720, 1920x1080
and 3840x2160, 2-6 lanes) in one autotuned graph launch, the serving latency
(p50/p99 over 16 camera streams with Poisson arrivals, continuous batching,
plain and pruned path, 60 s each), and the CPU oracle timed on a bounded
sample of the same workload, single-threaded and in one process per usable
core.  Beside it, on 64 other frames: Sobel against the Canny detector, the
coarse-to-fine Hough and the angle-paired vote against the plain vote, and
the oracle timed step by step on two of those frames.

What is timed is also checked: the oracle runs of the CPU-baseline leg are
compared with the GPU outputs of the timed plans (every peak of the 256-frame
plan, the accumulators of its 16 distinct frames, every accumulator and peak
of the 64-frame mixed plan), and every served result is compared with its
frame alone through the single-frame entry points.  Any mismatch sets
"parity": {"ok": false} and the exit status 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s & frames/s Sobel+Hough at 1080p; p99 frame latency, pruned vs plain"
W, H, N_THETA, TOPK = 1920, 1080, 360, 8
POOL = 16            # distinct generated frames; copied to distinct HBM buffers
HBM_PEAK_GBS = 8000.0
MFMA_FP16_PEAK_TFLOPS = 2500.0  # dense FP16 MFMA, published
CUS, CLOCK_GHZ = 256, 2.4
# LDS: 32 banks, one 4-byte access per bank per clock per CU
LDS_BANK_PEAK_GVOTES = CUS * 32 * CLOCK_GHZ


def note(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=256, help="frames per step")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU-oracle budget for the baseline sample (0 = skip)")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="processes of the all-cores oracle leg (capped at the usable cores; 0 = skip)")
    ap.add_argument("--latency-iters", type=int, default=1000)
    ap.add_argument("--vote-rows", type=int, default=0,
                    help="theta rows per vote workgroup (0 = tuned default)")
    ap.add_argument("--vote-queue", type=int, default=-1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-tune-cache", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of each serving run, plain and pruned (0 = skip)")
    ap.add_argument("--serve-pool", type=int, default=64, help="pre-generated frames per stream")
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="refills the server may run at once (1: one refill at a time)")
    ap.add_argument("--mixed", type=int, default=1,
                    help="run the 64-frame mixed-resolution batch leg (0 = skip)")
    ap.add_argument("--edge-frames", type=int, default=64,
                    help="frames of the Sobel vs Canny comparison (0 = skip)")
    return ap.parse_args()


def gen_pool(synth):
    seeds = [synth.frame_seed(0, synth.CONFIG_PLAIN_1080, i) for i in range(POOL)]
    sc = synth.scene_road(W, H)
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        return list(ex.map(lambda s: synth.gen_frame(sc, s), seeds))


def event_time(torch, fn, iters, stream):
    """Average ms of fn() over iters launches, HIP events on `stream`."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(iters):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / iters


def profiled_traffic(kernel: str, src: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "hbm_traffic_1080p_x256.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(kernel + r":.*?\n\s+traffic_bytes_per_launch (\S+)\s+\(source (\S+) sha256\[:16\] (\w+)\)",
                  text, re.S)
    if not m:
        return None
    cur = hashlib.sha256(open(os.path.join(ROOT, "paper_2212_09460_amd", "csrc", src), "rb")
                         .read()).hexdigest()[:16]
    return float(m.group(1)) if cur == m.group(3) else None


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def usable_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_worker(budget_s, first_seed):
    """One process of the all-cores oracle leg (no torch, no GPU): makes two
    frames of the workload, reports ready, waits for the go line on stdin,
    runs the single-threaded oracle over them for budget_s seconds and prints
    its frame count and time as JSON."""
    import oracle
    from paper_2212_09460_amd import synth

    sc = synth.scene_road(W, H)
    imgs = [synth.gen_frame(sc, synth.frame_seed(0, synth.CONFIG_PLAIN_1080, first_seed + i))
            for i in range(2)]
    C, S = synth.trig_q14(N_THETA)
    print("ready", flush=True)
    sys.stdin.readline()
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oracle.pipeline(imgs[n % 2], C, S, TOPK)
        n += 1
    print(json.dumps({"frames": n, "seconds": time.perf_counter() - t0}), flush=True)


def oracle_omp_worker(budget_s):
    """The OpenMP build of the oracle (Sobel rows and vote rows over the
    host's cores; LANE_ORACLE_LIB points to it) on frames of the 1080p
    workload, one frame at a time, for budget_s seconds after the go line;
    prints the frame count, the time and the SHA-256 of the first frame's
    accumulator."""
    import hashlib

    import oracle
    from paper_2212_09460_amd import synth

    sc = synth.scene_road(W, H)
    imgs = [synth.gen_frame(sc, synth.frame_seed(0, synth.CONFIG_PLAIN_1080, i)) for i in range(2)]
    C, S = synth.trig_q14(N_THETA)
    print("ready", flush=True)
    sys.stdin.readline()
    n, t0, sha = 0, time.perf_counter(), None
    while time.perf_counter() - t0 < budget_s or n == 0:
        r = oracle.pipeline(imgs[n % 2], C, S, TOPK)
        if n == 0:
            sha = hashlib.sha256(r["acc"].tobytes()).hexdigest()
        n += 1
    print(json.dumps({"frames": n, "seconds": time.perf_counter() - t0, "acc_sha": sha}), flush=True)


def oracle_mixed_worker(indices):
    """One process of the mixed-batch oracle leg (no torch, no GPU): makes
    frames `indices` of the 64-frame mixed batch, reports ready, waits for
    the go line, runs the oracle over them and prints, per frame, its edge
    count, dropped votes, peaks and the SHA-256 of its accumulator, with the
    time taken."""
    import hashlib

    import oracle
    from paper_2212_09460_amd import synth

    imgs = [synth.mixed_batch(i) for i in indices]
    C, S = synth.trig_q14(N_THETA)
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    res = [oracle.pipeline(im, C, S, TOPK) for im in imgs]
    dt = time.perf_counter() - t0
    out = [{"i": i, "px": int(im.shape[0] * im.shape[1]), "n_edges": r["n_edges"],
            "dropped": r["dropped"], "count": r["count"], "theta_idx": r["theta_idx"].tolist(),
            "r_idx": r["r_idx"].tolist(), "votes": r["votes"].tolist(),
            "acc_sha": hashlib.sha256(r["acc"].tobytes()).hexdigest()}
           for i, im, r in zip(indices, imgs, res)]
    print(json.dumps({"frames": out, "seconds": dt}), flush=True)


def run_workers(cmds, env):
    """Starts the worker processes, waits until all are ready, starts them
    together and returns their JSON results."""
    import subprocess

    ps = [subprocess.Popen(c, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
          for c in cmds]
    try:
        for p in ps:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker failed to start")
        for p in ps:
            p.stdin.write("go\n")
            p.stdin.flush()
        res = [json.loads(p.stdout.readline()) for p in ps]
        for p in ps:
            if p.wait(timeout=300) != 0:
                raise RuntimeError("oracle worker failed")
    finally:
        for p in ps:
            if p.poll() is None:
                p.kill()
    return res


def lds_probe():
    """Rate of LDS atomic increments (ds_add_u32) on this GPU from the probe
    library: conflict-free (the 64 lanes of an instruction on 64 consecutive
    words), hashed addresses over a 64 KB table, and the vote's own pattern
    and instruction mix (16 angle rows x 4 pixel slots, paired counters,
    four VALU instructions per increment); the best over 1, 2 and 4
    workgroups of 1024 threads per CU; in G increments per second."""
    import ctypes

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2212_09460_amd", "liblaneprobe.so"))
    f = lib.lane_probe_lds_add
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_uint64)]
    out = {}
    for random, name in ((0, "conflict_free"), (1, "hashed"), (2, "vote_pattern")):
        best = 0.0
        for groups in (CUS, 2 * CUS, 4 * CUS):
            steps = 1000
            rate, chk = ctypes.c_double(0.0), ctypes.c_uint64(0)
            if f(groups, steps, random, ctypes.byref(rate), ctypes.byref(chk)) != 0:
                raise RuntimeError("LDS probe failed")
            if chk.value != groups * 1024 * 16 * steps:
                raise RuntimeError("LDS probe lost increments")
            best = max(best, rate.value)
        out[name] = round(best / 1e9, 1)
    return out


def cnn_flops(W, H):
    """Useful FLOPs of the proposal network on one W x H frame (2 per
    multiply-add; zero padding and MFMA padding not counted): conv1 1->16,
    conv2 and conv3 16->16 at stride 2, head 16->9, all 3x3."""
    h1, w1 = (H + 1) // 2, (W + 1) // 2
    h2, w2 = (h1 + 1) // 2, (w1 + 1) // 2
    h3, w3 = (h2 + 1) // 2, (w2 + 1) // 2
    return 2 * 9 * (h1 * w1 * 16 * 1 + h2 * w2 * 16 * 16 + h3 * w3 * 16 * 16 + h3 * w3 * 9 * 16)


def cnn_roofline(torch, lane, pool_d, stream, iters=20):
    """The fused proposal network (lane_cnn_infer) on the 16 pool frames in
    one call, trained weights: us per frame and useful TFLOP/s against the
    dense FP16 MFMA peak."""
    from paper_2212_09460_amd.learned.model import ProposalNet, load_params
    net = ProposalNet(load_params())
    imgs = torch.stack(pool_d)
    n = imgs.shape[0]
    logits = torch.empty((n, 9, (H + 7) // 8, (W + 7) // 8), dtype=torch.float32, device=imgs.device)
    run = lambda: lane.cnn_infer(imgs, net.packed, logits, stream=stream)
    run()
    ms = event_time(torch, run, iters, stream)
    tflops = cnn_flops(W, H) * n / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "k_cnn_infer", "frames_per_call": n,
            "us_per_frame": round(ms * 1e3 / n, 2), "achieved": round(tflops, 1),
            "peak": MFMA_FP16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / MFMA_FP16_PEAK_TFLOPS, 4),
            "flops_per_frame": cnn_flops(W, H)}


def mixed_leg(args, torch, lane, synth, stream):
    """The mixed-resolution batch: 64 frames (16 each at 640x480, 1280x720,
    1920x1080 and 3840x2160, 2..6 lanes, 360 theta, top-8) resident in HBM,
    one graph launch per step, the plan's setting from the autotuner run on
    these frames.  Returns the figures and the GPU outputs of one clean
    launch (per frame: accumulator SHA-256, peaks, counters) for the check."""
    import hashlib

    dev = torch.device("cuda:0")
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        imgs = list(ex.map(synth.mixed_batch, range(64)))
    C, S = synth.trig_q14(N_THETA)
    Cd, Sd = torch.from_numpy(C).to(dev), torch.from_numpy(S).to(dev)
    frames = [lane.FrameBuffers(torch.from_numpy(im).to(dev), im.shape[1], N_THETA, TOPK, Cd, Sd)
              for im in imgs]
    tune, vote_ms, sobel_ms = lane.tune_batch(frames)
    b = lane.Batch(frames, tune=tune)
    b.launch(stream)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        b.launch(stream)
    torch.cuda.synchronize()
    ms = event_time(torch, lambda: b.launch(stream), args.steps, stream)
    for f in frames:  # the check reads one clean launch's outputs
        f.acc.fill_(-1)
        f.peaks.fill_(-2)
    b.launch(stream)
    torch.cuda.synchronize()
    gpu = [{"acc_sha": hashlib.sha256(f.acc.cpu().numpy().tobytes()).hexdigest(),
            "peaks": f.peaks.cpu().numpy(), "counters": f.counters.cpu().numpy()} for f in frames]
    px = sum(im.shape[0] * im.shape[1] for im in imgs)
    edges = sum(int(g["counters"][0]) for g in gpu)
    out = {"workload": "64 seeded road frames, 16 each at 640x480, 1280x720, 1920x1080 and "
                       "3840x2160 with 2-6 lanes, clutter and salt; threshold 128, ring masked; "
                       "360 theta, Q14 trig, int32 accumulators; top-8 peaks",
           "launch": "one HIP graph per step", "steps": args.steps,
           "value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "Mpix/s",
           "frames_per_s": round(64 / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
           "megapixels_per_step": round(px / 1e6, 3), "edge_fraction": round(edges / px, 4),
           "votes_per_step": edges * N_THETA,
           "tuned": dict(lane.tune_dict(tune), vote_ms=round(vote_ms, 4), sobel_ms=round(sobel_ms, 4))}
    b.close()
    del frames
    torch.cuda.empty_cache()
    return out, gpu


def check_plan_256(oracle_res, gpu256):
    """Every frame's peaks, edge count and dropped votes of the timed
    256-frame plan against the oracle's result for its pool frame, and the
    full accumulators of the first POOL frames."""
    bad = []
    k = TOPK
    for i in range(gpu256["peaks"].shape[0]):
        w = oracle_res[i % POOL]
        pk, cn = gpu256["peaks"][i], gpu256["counters"][i]
        ok = (int(pk[3 * k]) == w["count"] and (pk[0:k] == w["theta_idx"]).all()
              and (pk[k:2 * k] == w["r_idx"]).all() and (pk[2 * k:3 * k] == w["votes"]).all()
              and int(cn[0]) == w["n_edges"] and int(cn[1]) == w["dropped"])
        if ok and i < len(gpu256["acc"]):
            ok = bool((gpu256["acc"][i] == w["acc"]).all())
        if not ok:
            bad.append(i)
    return {"frames_peaks_checked": int(gpu256["peaks"].shape[0]),
            "accumulators_checked": len(gpu256["acc"]), "mismatched_frames": bad[:16],
            "ok": not bad}


def check_mixed(oracle_frames, gpu):
    bad = []
    k = TOPK
    for w in oracle_frames:
        g = gpu[w["i"]]
        pk, cn = g["peaks"], g["counters"]
        ok = (g["acc_sha"] == w["acc_sha"] and int(pk[3 * k]) == w["count"]
              and pk[0:k].tolist() == w["theta_idx"] and pk[k:2 * k].tolist() == w["r_idx"]
              and pk[2 * k:3 * k].tolist() == w["votes"] and int(cn[0]) == w["n_edges"]
              and int(cn[1]) == w["dropped"])
        if not ok:
            bad.append(w["i"])
    return {"frames_checked": len(oracle_frames), "mismatched_frames": bad[:16],
            "ok": not bad and len(oracle_frames) == len(gpu)}


def cpu_mixed(procs, gpu):
    """The oracle over the 64-frame mixed batch in `procs` processes (frame
    i in process i mod procs, so each holds sizes of every kind), started
    together: the host's time for the batch, and the check of the GPU plan."""
    procs = max(1, min(procs, 64))
    cmds = [[sys.executable, "-u", os.path.abspath(__file__), "--oracle-mixed-worker",
             ",".join(str(i) for i in range(p, 64, procs))] for p in range(procs)]
    res = run_workers(cmds, dict(os.environ, OMP_NUM_THREADS="1"))
    frames = [f for r in res for f in r["frames"]]
    span = max(r["seconds"] for r in res)
    px = sum(f["px"] for f in frames)
    return ({"value": round(px / span / 1e6, 3), "unit": "Mpix/s", "cores": procs,
             "frames_per_s": round(len(frames) / span, 3),
             "sample": f"the 64-frame mixed batch once, frame i in process i mod {procs} "
                       f"(single-threaded oracle processes started together), {span:.1f} s"},
            check_mixed(frames, gpu))


def cpu_all_cores(procs, budget_s):
    """The same untuned oracle, one frame per process at a time, in `procs`
    processes started together: the host's throughput over independent
    frames.  Frame generation happens before the start."""
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--oracle-worker", str(budget_s)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = run_workers([cmd + [str(1000 + 2 * i)] for i in range(procs)], env)
    frames = sum(r["frames"] for r in res)
    span = max(r["seconds"] for r in res)
    return {"value": round(frames * W * H / span / 1e6, 3), "unit": "Mpix/s", "cores": procs,
            "frames_per_s": round(frames / span, 3),
            "sample": f"{frames} frames of the same workload in {procs} single-threaded oracle "
                      f"processes started together, {span:.1f} s"}


def cpu_openmp(threads, budget_s, ref0):
    """The oracle's OpenMP build in one process with `threads` threads: the
    per-frame multi-core baseline (Sobel rows and vote rows split over the
    cores); its first accumulator must equal the single-threaded one."""
    import hashlib

    import oracle

    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--oracle-omp-worker", str(budget_s)]
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), LANE_ORACLE_LIB=oracle.OMP_LIB_PATH)
    r = run_workers([cmd], env)[0]
    out = {"value": round(r["frames"] * W * H / r["seconds"] / 1e6, 3), "unit": "Mpix/s",
           "cores": threads, "frames_per_s": round(r["frames"] / r["seconds"], 3),
           "sample": f"{r['frames']} frames of the same workload, one at a time, oracle built "
                     f"with OpenMP ({threads} threads: image rows of Sobel, theta rows of the "
                     f"vote), {r['seconds']:.1f} s"}
    if ref0 is not None:
        out["same_result"] = r["acc_sha"] == hashlib.sha256(ref0["acc"].tobytes()).hexdigest()
    return out


def cpu_baseline(pool, C, S, budget_s, procs, gpu256=None, mixed_gpu=None):
    """The oracle timed on the host (single-threaded on the 1080p workload;
    all cores on the same workload and on the mixed batch).  Its results are
    also the reference the timed GPU plans are checked against."""
    import oracle

    n, px, t0 = 0, 0, time.perf_counter()
    first = {}
    while time.perf_counter() - t0 < budget_s and n < 60:
        j = n % len(pool)
        r = oracle.pipeline(pool[j], C, S, TOPK)
        first.setdefault(j, r)
        n += 1
        px += W * H
    dt = time.perf_counter() - t0
    out = {"value": round(px / dt / 1e6, 3), "unit": "Mpix/s", "cores": 1, "kind": "oracle",
           "sample": f"{n} frames of the 1920x1080 workload (full path: Sobel, binarize, "
                     f"vote over 360 theta, top-8 peaks), single-threaded C oracle, "
                     f"{dt:.1f} s", "frames_per_s": round(n / dt, 4),
           "host_cpu": host_cpu_model(), "host_usable_cores": usable_cores()}
    checks = {}
    if gpu256 is not None:
        for j in range(len(pool)):  # untimed: pool frames the budget did not reach
            if j not in first:
                first[j] = oracle.pipeline(pool[j], C, S, TOPK)
        checks["plan_1080p_x256"] = check_plan_256(first, gpu256)
    procs = min(procs, usable_cores())
    if procs > 1:
        out["all_cores"] = cpu_all_cores(procs, budget_s)
        out["openmp"] = cpu_openmp(procs, budget_s, first.get(0))
    if mixed_gpu is not None:
        out["mixed_batch"], checks["mixed_64"] = cpu_mixed(max(procs, 1), mixed_gpu)
    return out, checks


def edge_detectors(n_frames):
    """Sobel + binarization (the paper's detector) against Canny (its
    proposed replacement) on the same seeded 1080p frames, each through the
    single-frame entry points (detector -> vote -> peaks): GPU time per frame,
    edge fraction, and the share of painted lanes found among the top-4
    peaks.  Frames come from seeds disjoint from the throughput pool."""
    import torch

    import paper_2212_09460_amd.lane as lane
    from paper_2212_09460_amd import synth
    from paper_2212_09460_amd.learned.evaluate import lanes_found

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sc = synth.scene_road(W, H)
    seeds = [synth.frame_seed(0, synth.CONFIG_PLAIN_1080, 100000 + i) for i in range(n_frames)]
    imgs = [torch.from_numpy(synth.gen_frame(sc, sd)).to(dev) for sd in seeds]
    C, S = synth.trig_q14(N_THETA)
    Cd, Sd = torch.from_numpy(C).to(dev), torch.from_numpy(S).to(dev)
    D = lane.r_offset(W, H)
    n_r = 2 * D + 1
    ws = torch.empty(lane.canny_workspace_size(W, H) // 8 + 2, dtype=torch.int64, device=dev)
    T_LOW, T_HIGH = 64, 128

    def detect(kind, img):
        if kind == "sobel":
            _, _, lst, cnt = lane.sobel_binarize(img, W, 128, 1, stream=stream)
        else:
            _, _, lst, cnt = lane.canny(img, W, T_LOW, T_HIGH, 1, ws=ws, stream=stream)
        return lst, cnt

    out = {"frames": n_frames, "canny_thresholds": [T_LOW, T_HIGH], "sobel_threshold": 128,
           "oracle_ms_per_frame": oracle_rows([synth.gen_frame(sc, sd) for sd in seeds[:2]], C, S, D,
                                              T_LOW, T_HIGH)}
    for kind in ("sobel", "canny"):
        # warm-up, then the detector alone and the whole path, back to back
        for img in imgs[:2]:
            detect(kind, img)
        torch.cuda.synchronize()
        t_det = event_time(torch, lambda: [detect(kind, im) for im in imgs], 1, stream) / n_frames
        results = []

        def path():
            results.clear()
            for im in imgs:
                lst, cnt = detect(kind, im)
                acc, _ = lane.hough_vote(lst, W, H, Cd, Sd, D, n_r, stream=stream)
                results.append((cnt, lane.hough_peaks(acc, D, TOPK, stream=stream)))

        t_path = event_time(torch, path, 1, stream) / n_frames
        found = total = 0
        edges = 0
        for sd, (cnt, (t, r, v, c)) in zip(seeds, results):
            n = int(c.cpu()[0])
            f = lanes_found(synth.lane_segments(sc, sd), t.cpu().numpy(), r.cpu().numpy(), n,
                            N_THETA, D, k=4)
            found += int(f.sum())
            total += len(f)
            edges += int(cnt.cpu()[0])
        out[kind] = {"detector_ms_per_frame": round(t_det, 4), "path_ms_per_frame": round(t_path, 4),
                     "edge_fraction": round(edges / (n_frames * W * H), 4),
                     "lanes_found_top4": round(found / max(total, 1), 4)}
        lists = [detect(kind, im)[0] for im in imgs]
        out[kind]["progressive"] = progressive_vs_plain(torch, lane, lists, seeds, sc, Cd, Sd, D, stream)
        out[kind]["angle_pairing"] = paired_vote(torch, lane, lists, Cd, Sd, D, stream)
    return out


def oracle_rows(imgs, C, S, D, t_low, t_high):
    """The CPU oracle (single-threaded C) on two of the same frames, step by
    step, for comparison with the GPU times of each row."""
    import oracle

    from paper_2212_09460_amd import lane

    n_r = 2 * D + 1
    steps = {}

    def timed(name, fn):
        t0 = time.perf_counter()
        res = [fn(im) for im in imgs]
        steps[name] = round((time.perf_counter() - t0) / len(imgs) * 1000, 1)
        return res

    sob = timed("sobel_binarize", lambda im: oracle.sobel_binarize(im, W, 128, 1)[0])
    can = timed("canny", lambda im: oracle.canny(im, W, t_low, t_high, 1)[0])
    it = iter(sob)
    accs = timed("vote", lambda im: oracle.hough_vote(next(it), C, S, D, n_r)[0])
    it = iter(accs)
    pk = timed("peaks", lambda im: oracle.hough_peaks(next(it), D, TOPK))
    it, ip = iter(sob), iter(pk)
    timed("line_segments", lambda im: oracle.hough_lines(next(it), C, S, D, *next(ip)[:2]))
    prm = lane.progressive_params(N_THETA, n_r)
    it = iter(sob)
    timed("coarse_to_fine_hough", lambda im: oracle.hough_progressive(next(it), C, S, D, **prm))
    it = iter(can)
    timed("vote_canny_edges", lambda im: oracle.hough_vote(next(it), C, S, D, n_r)[0])
    return steps


def paired_vote(torch, lane, lists, Cd, Sd, D, stream):
    """The angle pairing of the FPGA design (rows k and n - k from shared
    products) against the same kernel without it and against the library's
    single-frame vote, on the same edge lists: GPU time per frame of the
    vote alone."""
    n = len(lists)
    n_r = 2 * D + 1

    def run(fn):
        fn()
        torch.cuda.synchronize()
        return round(event_time(torch, fn, 1, stream) / n, 4)

    return {"vote_ms_per_frame": {
        "library_vote": run(lambda: [lane.hough_vote(l, W, H, Cd, Sd, D, n_r, stream=stream) for l in lists]),
        "pair_kernel_unpaired": run(lambda: [lane.hough_vote_paired(l, W, H, Cd, Sd, D, n_r, 0, stream=stream)
                                             for l in lists]),
        "pair_kernel_paired": run(lambda: [lane.hough_vote_paired(l, W, H, Cd, Sd, D, n_r, 1, stream=stream)
                                           for l in lists])}}


def progressive_vs_plain(torch, lane, lists, seeds, sc, Cd, Sd, D, stream):
    """The coarse-to-fine Hough against the plain vote + peaks on the same
    edge lists: GPU time per frame of each, agreement of the top-4 (same line
    within one theta bin and one r cell), exact cells, and painted lanes
    found among the progressive top-4."""
    from paper_2212_09460_amd import synth
    from paper_2212_09460_amd.learned.evaluate import agreement_counts, lanes_found

    n = len(lists)
    n_r = 2 * D + 1
    params = lane.progressive_params(N_THETA, n_r)
    pws = torch.empty(lane.progressive_layout(W, H, N_THETA, D, params)["bytes"] // 8 + 2,
                      dtype=torch.int64, device=lists[0].device)
    plain, prog = [], []

    def run_plain():
        plain.clear()
        for lst in lists:
            acc, _ = lane.hough_vote(lst, W, H, Cd, Sd, D, n_r, stream=stream)
            plain.append(lane.hough_peaks(acc, D, TOPK, stream=stream))

    def run_prog():
        prog.clear()
        for lst in lists:
            prog.append(lane.hough_progressive(lst, W, H, Cd, Sd, D, params, ws=pws, stream=stream)[:4])

    run_plain()
    run_prog()
    torch.cuda.synchronize()
    t_plain = event_time(torch, run_plain, 1, stream) / n
    t_prog = event_time(torch, run_prog, 1, stream) / n
    agree = tot = same = found = lanes = 0
    for sd, (pt, pr, pv, pc), (qt, qr, qv, qc) in zip(seeds, plain, prog):
        pt, pr, qt, qr = (x.cpu().numpy() for x in (pt, pr, qt, qr))
        pn, qn = int(pc.cpu()[0]), int(qc.cpu()[0])
        m, k = agreement_counts(pt, pr, pn, qt, qr, qn, 4, N_THETA, D)
        agree += m
        tot += k
        same += len({(int(a), int(b)) for a, b in zip(pt[:min(4, pn)], pr[:min(4, pn)])} &
                    {(int(a), int(b)) for a, b in zip(qt[:min(4, qn)], qr[:min(4, qn)])})
        f = lanes_found(synth.lane_segments(sc, sd), qt, qr, qn, N_THETA, D, k=4)
        found += int(f.sum())
        lanes += len(f)
    return {"params": params, "hough_ms_per_frame": {"plain": round(t_plain, 4),
                                                     "progressive": round(t_prog, 4)},
            "speedup": round(t_plain / t_prog, 3), "agreement_top4": round(agree / max(tot, 1), 4),
            "same_cell_top4": round(same / max(tot, 1), 4),
            "lanes_found_top4": round(found / max(lanes, 1), 4)}


def serving(args):
    """p50 / p99 latency (arrival to peaks in host memory) of the 16-stream
    mix through the continuous-batching server, plain then pruned."""
    from paper_2212_09460_amd import serve

    res = {"streams": "8x1280x720 + 6x1920x1080 + 2x3840x2160, Poisson arrivals 30 Hz each",
           "seconds": args.serve_seconds}
    pools = None
    res["pool_frames_per_stream"] = args.serve_pool
    res["refill_lanes"] = args.serve_lanes
    for pruned in (False, True):
        note(f"serving, {'pruned' if pruned else 'plain'}: {args.serve_seconds} s")
        r, pools = serve.run(args.serve_seconds, pruned=pruned, pool=args.serve_pool, pools=pools,
                             verbose=False, verify=True, lanes=args.serve_lanes)
        note(f"serving done: p50 {r['p50_ms']:.4f} ms, p99 {r['p99_ms']:.4f} ms, verified {r['verified']}")
        res["pruned" if pruned else "plain"] = {
            k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
            if k in ("p50_ms", "p99_ms", "max_ms", "frames_per_s", "gpx_per_s", "completed",
                     "dropped", "mean_batch_frames", "per_size", "verified")}
    res["p99_pruned_over_plain"] = round(res["pruned"]["p99_ms"] / res["plain"]["p99_ms"], 4)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; multi-GPU runs are not "
                                   "supported (frames would shard across GPUs with no "
                                   "exchange)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2212_09460_amd.lane as lane
    from paper_2212_09460_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    note("generating the 1080p pool")
    pool = gen_pool(synth)
    C, S = synth.trig_q14(N_THETA)
    Cd, Sd = torch.from_numpy(C).to(dev), torch.from_numpy(S).to(dev)
    pool_d = [torch.from_numpy(f).to(dev) for f in pool]
    B = args.frames
    # autotune (outside the timed region): theta-slice width, vote work
    # distribution, Sobel strip height and grid, for this batch size
    from paper_2212_09460_amd import tune as tuner
    if args.vote_rows > 0:
        tune = lane.LaneTune(args.vote_rows, args.vote_queue, 0, 0)
        tune_info = lane.tune_dict(tune)
    else:
        tune, tune_info = tuner.tuned(pool_d[0], N_THETA, B, W, use_cache=not args.no_tune_cache)
    note(f"tuned: {tune_info}")
    frames = []
    for i in range(B):
        img = torch.empty((H, W), dtype=torch.uint8, device=dev)
        img.copy_(pool_d[i % POOL])
        frames.append(lane.FrameBuffers(img, W, N_THETA, TOPK, Cd, Sd))
    batch = lane.Batch(frames, tune=tune)

    # first launch outside the timed region
    batch.launch(stream)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        batch.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_step = event_time(torch, lambda: batch.launch(stream), args.steps, stream)
    wall = time.perf_counter() - t0
    note(f"timed {args.steps} steps of {B} frames: {ms_step:.4f} ms per step")

    # per-stage times (same kernels, launched one stage at a time)
    stage_iters = max(3, args.steps // 2)
    batch.launch_stage(0, stream)
    t_sobel = event_time(torch, lambda: batch.launch_stage(1, stream), stage_iters, stream)
    t_vote = event_time(torch, lambda: batch.launch_stage(2, stream), stage_iters, stream)
    t_peaks = event_time(torch, lambda: batch.launch_stage(3, stream), stage_iters, stream)

    # one clean full pass so the per-frame counters hold one run's counts
    batch.launch(stream)
    torch.cuda.synchronize()
    counters = torch.stack([f.counters for f in frames]).cpu().numpy()
    gpu256 = {"peaks": torch.stack([f.peaks for f in frames]).cpu().numpy(), "counters": counters,
              "acc": [frames[i].acc.cpu().numpy() for i in range(min(POOL, B))]}
    n_edges = counters[:, 0].astype(np.int64)
    dropped = int(counters[:, 1].sum())
    votes = int(n_edges.sum()) * N_THETA
    px = B * W * H

    # algorithmic bytes of the Sobel pass: image in, edge map out, one 4-byte
    # list entry per edge, one 4-byte tile record per 8x8 tile, segment counts
    th, tw = (H + 7) // 8, (W + 7) // 8
    nseg = th * ((W + 1023) // 1024)
    sobel_bytes = B * (2 * W * H + 4 * th * tw + 4 * nseg) + 4 * int(n_edges.sum())
    sobel_gbs = sobel_bytes / (t_sobel * 1e-3) / 1e9
    vote_gvotes = votes / (t_vote * 1e-3) / 1e9

    # single-frame latency: a one-frame plan shaped for latency (4 theta rows
    # per vote workgroup, each slice split over 8 workgroups, 8-row Sobel
    # strips), each launch timed alone
    lat = []
    if args.latency_iters > 0:
        one = lane.Batch([frames[0]], vote_rows=4, vote_queue=1, sobel_strip_rows=8, vote_split=8)
        for i in range(args.latency_iters + 5):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            one.launch(stream)
            b.record(stream)
            b.synchronize()
            if i >= 5:
                lat.append(a.elapsed_time(b))
        one.close()
    lat = np.array(lat if lat else [float("nan")])

    # line segments along each frame's peaks (one launch per frame, one
    # workgroup per peak): average over 64 frames launched back to back
    lines_us = None
    if args.latency_iters > 0:
        nl = min(64, B)

        def lines_all():
            for f in frames[:nl]:
                lane.hough_lines(f.edges, Cd, Sd, f.D, f.theta_idx(), f.r_idx(), f.count(),
                                 stream=stream)

        lines_all()
        torch.cuda.synchronize()
        lines_us = event_time(torch, lines_all, 5, stream) / nl * 1000

    # practical reference for the Sobel pass: a plain device copy moving the
    # same number of bytes (half read, half written), timed the same way
    nb = sobel_bytes // 2
    csrc = torch.empty(nb, dtype=torch.uint8, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        cdst.copy_(csrc)
    c1.record(stream)
    c1.synchronize()
    copy_gbs = 2 * nb / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del csrc, cdst
    if args.copy_calibration:
        # counter calibration for the traffic figures: an ordinary elementwise
        # kernel reading 1 GiB and writing 1 GiB (a device copy_ goes to the
        # runtime's blit kernel, whose counters behave differently)
        src = torch.zeros(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    probe = lds_probe()
    note(f"LDS increment probe (G/s): {probe}")
    cnn = cnn_roofline(torch, lane, pool_d, stream)
    note(f"proposal network: {cnn}")
    value = px / (ms_step * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "1920x1080 seeded road frames: 4 lanes (inner 2 dashed), 200 "
                               "clutter segments, 2% salt; threshold 128, ring masked; 360 theta, "
                               "r step 1 px, Q14 trig, int32 accumulator; top-8 peaks",
                   "frames_per_step": B, "launch": "one HIP graph per step",
                   "tuned": tune_info},
        "frames_per_s": round(B / (ms_step * 1e-3), 1),
        "edge_fraction": round(float(n_edges.sum()) / px, 4),
        "dropped_votes": dropped,
        "stage_ms": {"sobel": round(t_sobel, 4), "vote": round(t_vote, 4),
                     "peaks": round(t_peaks, 4)},
        "roofline": {"bound": "lds", "kernel": "k_vote_batch", "achieved": round(vote_gvotes, 1),
                     "peak": round(LDS_BANK_PEAK_GVOTES, 1), "unit": "Gvote/s",
                     "frac": round(vote_gvotes / LDS_BANK_PEAK_GVOTES, 4),
                     "peak_measured": probe["conflict_free"],
                     "frac_of_measured": round(vote_gvotes / probe["conflict_free"], 4),
                     "frac_of_vote_pattern": round(vote_gvotes / probe["vote_pattern"], 4),
                     "probe_gadds_per_s": probe,
                     "traffic": profiled_traffic("k_vote_batch", "vote.hip") if B == 256 else None,
                     "votes_per_launch": votes},
        "roofline_sobel": {"bound": "hbm", "kernel": "k_sobel_batch",
                           "achieved": round(sobel_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(sobel_gbs / HBM_PEAK_GBS, 4),
                           "traffic": profiled_traffic("k_sobel_batch", "sobel.hip") if B == 256 else None,
                           "bytes_per_launch": sobel_bytes,
                           "device_copy_gbs": round(copy_gbs, 1),
                           "frac_of_device_copy": round(sobel_gbs / copy_gbs, 4)},
        "roofline_cnn": cnn,
        "latency_ms_single_frame_gpu": {"p50": round(float(np.percentile(lat, 50)), 4),
                                        "p99": round(float(np.percentile(lat, 99)), 4),
                                        "max": round(float(np.max(lat)), 4), "runs": int(lat.size)},
        "lines_us_per_frame": None if lines_us is None else round(lines_us, 2),
        "wall_s_timed": round(wall, 3),
    }
    batch.close()
    del frames, pool_d
    torch.cuda.empty_cache()
    mixed_gpu = None
    if args.mixed:
        note("mixed-resolution batch: generate, tune, time")
        out["mixed_batch"], mixed_gpu = mixed_leg(args, torch, lane, synth, stream)
        note(f"mixed batch: {out['mixed_batch']['ms_per_step']} ms per step")
    if args.edge_frames > 0:
        note("edge detectors, coarse-to-fine Hough, paired vote")
        out["edge_detectors"] = edge_detectors(args.edge_frames)
    if args.serve_seconds > 0:
        out["serving"] = serving(args)
    checks = {}
    if args.cpu_seconds > 0:
        note("CPU oracle: single thread, all cores, mixed batch (and the checks)")
        out["cpu_baseline"], checks = cpu_baseline(pool, C, S, args.cpu_seconds, args.cpu_procs,
                                                   gpu256, mixed_gpu)
    if args.serve_seconds > 0:
        for mode in ("plain", "pruned"):
            v = out["serving"][mode]["verified"]
            checks["serving_" + mode] = dict(v, ok=v["mismatches"] == 0 and v["checked"] > 0)
    out["parity"] = dict(checks, ok=all(c["ok"] for c in checks.values()) if checks else None)
    print(json.dumps(out), flush=True)
    if checks and not out["parity"]["ok"]:
        sys.exit(1)


if __name__ == "__main__":
    if len(sys.argv) == 4 and sys.argv[1] == "--oracle-worker":
        oracle_worker(float(sys.argv[2]), int(sys.argv[3]))
    elif len(sys.argv) == 3 and sys.argv[1] == "--oracle-omp-worker":
        oracle_omp_worker(float(sys.argv[2]))
    elif len(sys.argv) == 3 and sys.argv[1] == "--oracle-mixed-worker":
        oracle_mixed_worker([int(x) for x in sys.argv[2].split(",")])
    else:
        main()
