"""Serving workload: many camera streams, Poisson arrivals, continuous
batching through lane_server (native refill lanes, device-resident
per-stream state, HBM-budget admission).

The stream mix is 8 x 1280x720, 6 x 1920x1080 and 2 x 3840x2160 at 30
frames/s each (480 frames/s, 1.09 Gpx/s).  Host-side frame generation at that
rate is out of reach, so every stream replays a pool of pre-generated seeded
road frames of its size held in page-locked memory.  Latency of a frame =
its arrival (submission) to its peaks in host memory, H2D copy included.

  python -m paper_2212_09460_amd.serve --seconds 20 --pruned
"""
from __future__ import annotations

import argparse
import json
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import synth

MIX = ((1280, 720, 8), (1920, 1080, 6), (3840, 2160, 2))
CONFIG_ID = 4


def mix_streams(mix=MIX, n_theta: int = 360, k: int = 8):
    out = []
    for W, H, n in mix:
        out += [dict(W=W, H=H, n_theta=n_theta, k=k) for _ in range(n)]
    return out


def poisson_schedule(n_streams: int, rate_hz: float, seconds: float, seed: int = 0):
    """Arrival times of every stream (exponential gaps of mean 1/rate, each
    stream its own seeded generator), merged in time order.  Returns
    (t_seconds float64 [n], stream int32 [n], per-stream frame index [n])."""
    ts, ss, ks = [], [], []
    for s in range(n_streams):
        g = np.random.default_rng([seed, s])
        t, i = 0.0, 0
        while True:
            t += g.exponential(1.0 / rate_hz)
            if t >= seconds:
                break
            ts.append(t)
            ss.append(s)
            ks.append(i)
            i += 1
    order = np.argsort(np.asarray(ts), kind="stable")
    return (np.asarray(ts)[order], np.asarray(ss, np.int32)[order], np.asarray(ks, np.int64)[order])


def frame_pools(streams, pool: int = 64, base_seed: int = 0, workers: int = 16, pinned: bool = True):
    """Per stream, `pool` seeded road frames of its size ([pool][H][W] uint8,
    page-locked when torch is available and pinned=True)."""
    import torch

    out = []
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for si, st in enumerate(streams):
            W, H = st["W"], st["H"]
            sc = synth.scene_road(W, H)
            seeds = [synth.frame_seed(base_seed, CONFIG_ID, (si << 20) + i) for i in range(pool)]
            frames = list(ex.map(lambda s: synth.gen_frame(sc, s), seeds))
            t = torch.empty((pool, H, W), dtype=torch.uint8, pin_memory=pinned)
            t.numpy()[:] = np.stack(frames)
            out.append(t)
    return out


def reference_peaks(streams, pools, pruned: bool = False, conf: float = 0.9, cnn_params=None):
    """Per stream and pool frame, the peaks of that frame alone through the
    single-frame entry points -- plain: Sobel, vote, peaks; pruned: the
    proposal network, its tile mask, the masked vote, peaks -- i.e. what
    every served result of that frame must equal.  Returns
    refs[stream][frame] = (count, theta_idx[:k], r_idx[:k], votes[:k])."""
    import torch

    from . import lane

    net = None
    if pruned:
        from .learned.model import ProposalNet, load_params

        net = ProposalNet(load_params() if cnn_params is None else cnn_params)
    tables = {}
    out_dev = []
    for s, st in enumerate(streams):
        W, H, n_theta, k = st["W"], st["H"], st.get("n_theta", 360), st.get("k", 8)
        if n_theta not in tables:
            C, S = lane.make_trig_q14(n_theta)
            tables[n_theta] = (torch.from_numpy(C).cuda(), torch.from_numpy(S).cuda())
        Cd, Sd = tables[n_theta]
        rows = []
        for j in range(pools[s].shape[0]):
            img = pools[s][j].cuda(non_blocking=True)
            mask = None
            if net is not None:
                lg = net.forward(img[None])
                mask = torch.empty((1, (H + 7) // 8, (W + 7) // 8), dtype=torch.uint8, device="cuda")
                lane.mask_from_logits(lg, W, H, 1, conf, mask)
                mask = mask[0]
            r = lane.pipeline(img, Cd, Sd, k, threshold=st.get("threshold", 128),
                              border_mode=st.get("border_mode", 1), tile_mask=mask)
            rows.append(torch.cat([r["count"].view(1), r["theta_idx"], r["r_idx"], r["votes"]]))
        out_dev.append(torch.stack(rows))
    refs = []
    for s, st in enumerate(streams):
        k = st.get("k", 8)
        a = out_dev[s].cpu().numpy()
        refs.append([(int(row[0]), row[1:1 + k].tolist(), row[1 + k:1 + 2 * k].tolist(),
                      row[1 + 2 * k:1 + 3 * k].tolist()) for row in a])
    return refs


def check_results(results, reqs_meta, refs, streams):
    """Compares every completed result with the reference peaks of its frame;
    reqs_meta[i] = (stream, pool index) of request i.  Returns (checked,
    mismatches)."""
    checked = bad = 0
    for r in results:
        if r.status != 0:
            continue
        s, j = reqs_meta[int(r.frame_id)]
        k = streams[s].get("k", 8)
        c, t, rr, v = refs[s][j]
        ok = (r.stream == s and r.count == c and list(r.theta_idx[:k]) == t
              and list(r.r_idx[:k]) == rr and list(r.votes[:k]) == v)
        checked += 1
        bad += not ok
    return checked, bad


def requests(schedule, pools):
    ts, ss, ks = schedule
    reqs = []
    for i in range(len(ts)):
        s = int(ss[i])
        pool = pools[s].numpy()
        fr = pool[int(ks[i]) % pool.shape[0]]
        reqs.append((s, float(ts[i]), fr, i))
    return reqs


def summarize(results, streams, seconds: float):
    lat = {}
    ok = [r for r in results if r.status == 0]
    dropped = sum(1 for r in results if r.status != 0)
    allv = np.array([(r.t_done_ns - r.t_submit_ns) / 1e6 for r in ok]) if ok else np.zeros(0)
    for r in ok:
        st = streams[r.stream]
        lat.setdefault(f"{st['W']}x{st['H']}", []).append((r.t_done_ns - r.t_submit_ns) / 1e6)
    bf = np.array([r.batch_frames for r in ok]) if ok else np.zeros(0)
    px = sum(streams[r.stream]["W"] * streams[r.stream]["H"] for r in ok)
    out = dict(frames=len(results), completed=len(ok), dropped=dropped,
               frames_per_s=len(ok) / seconds, gpx_per_s=px / seconds / 1e9,
               p50_ms=float(np.percentile(allv, 50)) if ok else None,
               p99_ms=float(np.percentile(allv, 99)) if ok else None,
               max_ms=float(allv.max()) if ok else None,
               mean_batch_frames=float(bf.mean()) if ok else None,
               per_size={k: dict(n=len(v), p50_ms=float(np.percentile(v, 50)),
                                 p99_ms=float(np.percentile(v, 99))) for k, v in lat.items()})
    return out


def run(seconds: float = 20.0, pruned: bool = False, conf: float = 0.9, cnn_params=None,
        rate_hz: float = 30.0, seed: int = 0, pool: int = 64, hbm_budget: int = 8 << 30,
        max_pending: int = 8, vote_rows: int = 0, pools=None, mix=MIX, verbose: bool = True,
        vote_split: int = 0, verify: bool = False, lanes: int = 0, spin_us: int = 0):
    """One serving run; with verify, every completed result is compared with
    its frame alone (reference_peaks) and out["verified"] holds the counts."""
    from . import lane

    streams = mix_streams(mix)
    if pools is None:
        pools = frame_pools(streams, pool)
    if pruned and cnn_params is None:
        from .learned.model import load_params

        cnn_params = load_params()
    refs = reference_peaks(streams, pools, pruned, conf, cnn_params) if verify else None
    srv = lane.Server(streams, hbm_budget=hbm_budget, pruned=pruned, conf=conf,
                      cnn_params=cnn_params, max_pending=max_pending, vote_rows=vote_rows,
                      vote_split=vote_split, lanes=lanes, spin_us=spin_us)
    try:
        # warm-up: one frame per stream through the server
        warm = [(s, 0.0, pools[s].numpy()[0], s) for s in range(len(streams)) if srv.admitted[s]]
        srv.replay(warm)
        sched = poisson_schedule(len(streams), rate_hz, seconds, seed)
        keep = [i for i in range(len(sched[0])) if srv.admitted[int(sched[1][i])]]
        sched = tuple(a[keep] for a in sched)
        reqs = requests(sched, pools)
        if verbose:
            print(f"[serve] {'pruned' if pruned else 'plain'}: {len(reqs)} requests over {seconds} s",
                  flush=True)
        res = srv.replay(reqs)
        out = summarize(list(res), streams, seconds)
        if refs is not None:
            meta = [(int(sched[1][i]), int(sched[2][i]) % pools[int(sched[1][i])].shape[0])
                    for i in range(len(sched[0]))]
            checked, bad = check_results(list(res), meta, refs, streams)
            out["verified"] = dict(checked=checked, mismatches=bad)
        out["mode"] = "pruned" if pruned else "plain"
        out["streams_admitted"] = sum(srv.admitted)
        out["server"] = srv.stats()
    finally:
        srv.close()
    return out, pools


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=20.0)
    ap.add_argument("--pruned", action="store_true")
    ap.add_argument("--both", action="store_true")
    ap.add_argument("--conf", type=float, default=0.9)
    ap.add_argument("--vote-rows", type=int, default=0)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--spin-us", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    modes = [False, True] if a.both else [a.pruned]
    pools = None
    allres = []
    for m in modes:
        r, pools = run(a.seconds, m, a.conf, pool=a.pool, pools=pools, vote_rows=a.vote_rows,
                       lanes=a.lanes, spin_us=a.spin_us)
        print(json.dumps(r), flush=True)
        allres.append(r)
    if a.out:
        json.dump(allres, open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
