"""Evaluate the pruned vote against the plain one on held-out frames.

For every frame the plain batched path gives the reference top-k peaks; the
network's logits become a tile mask (lane_mask_from_logits, confidence
`conf`), and the same frame goes through the masked vote and the peak search.
Reported: top-4 and top-8 peak agreement within +-1 theta bin and +-1 r bin
(theta wrapping with r mirrored), missed-peak rate, tile fractions (pruned
to bands / skipped / fallback), votes cast as a fraction of plain, and GPU
times of the vote stage, plain vs pruned, with the network's own cost.

Baselines at the same vote budget: a random-initialised network, and a
heuristic that keeps a tile (every theta) iff it has at least tau edge
pixels, tau chosen so its votes match the trained network's.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .. import lane, synth
from .model import ProposalNet
from .train import N_THETA, TOPK, gen_batch


def same_line(t1, r1, t2, r2, n_theta, D, tol=1):
    for q in (-1, 0, 1):
        tt = t2 + q * n_theta
        rr = (2 * D - r2) if q % 2 else r2
        if abs(tt - t1) <= tol and abs(rr - r1) <= tol:
            return True
    return False


def agreement_counts(pt, pr, pn, qt, qr, qn, k, n_theta, D, only=None):
    """(matched, total) for the top-k plain peaks against the top-k pruned;
    `only` restricts the plain peaks counted (a boolean per peak)."""
    kk = min(k, pn)
    m = n = 0
    for i in range(kk):
        if only is not None and not only[i]:
            continue
        n += 1
        if any(same_line(pt[i], pr[i], qt[j], qr[j], n_theta, D) for j in range(min(k, qn))):
            m += 1
    return m, n


def lane_flags(segs, pt, pr, pn, n_theta, D, tol_px=8.0):
    """Which peaks lie on a painted lane: both ends of the lane's centre
    segment are within tol_px of the peak's line (the band is 6 px wide and
    its edge pixels lie up to about 4 px from the centre line)."""
    out = np.zeros(pn, bool)
    for i in range(pn):
        th = pt[i] * math.pi / n_theta
        c, s_ = math.cos(th), math.sin(th)
        r = pr[i] - D
        for x0, y0, x1, y1 in segs:
            if max(abs(x0 * c + y0 * s_ - r), abs(x1 * c + y1 * s_ - r)) <= tol_px:
                out[i] = True
    return out


def lanes_found(segs, pt, pr, pn, n_theta, D, k=4, tol_px=8.0):
    """Per painted lane, whether one of the top-k peaks lies on it (both ends
    of its centre segment within tol_px of the peak's line)."""
    found = np.zeros(len(segs), bool)
    for i in range(min(k, pn)):
        th = pt[i] * math.pi / n_theta
        c, s_ = math.cos(th), math.sin(th)
        r = pr[i] - D
        for j, (x0, y0, x1, y1) in enumerate(segs):
            if max(abs(x0 * c + y0 * s_ - r), abs(x1 * c + y1 * s_ - r)) <= tol_px:
                found[j] = True
    return found


class EvalPlans:
    def __init__(self, W, H, B, device="cuda"):
        self.W, self.H, self.B = W, H, B
        self.th, self.tw = (H + 7) // 8, (W + 7) // 8
        self.imgs = torch.empty((B, H, W), dtype=torch.uint8, device=device)
        C, S = synth.trig_q14(N_THETA)
        self.C, self.S = torch.from_numpy(C).to(device), torch.from_numpy(S).to(device)
        self.mask = torch.full((B, self.th, self.tw), 0xFF, dtype=torch.uint8, device=device)
        self.plain = [lane.FrameBuffers(self.imgs[b], W, N_THETA, TOPK, self.C, self.S)
                      for b in range(B)]
        self.pruned = [lane.FrameBuffers(self.imgs[b], W, N_THETA, TOPK, self.C, self.S,
                                         tile_mask=self.mask[b]) for b in range(B)]
        self.plain_plan = lane.Batch(self.plain)
        self.pruned_plan = lane.Batch(self.pruned)
        L = self.plain[0]
        nseg = self.th * ((W + 1023) // 1024)
        self.off_info = nseg
        self.D = L.D

    def tile_counts(self, b):
        info = self.plain[b].edge_list[self.off_info:self.off_info + self.th * self.tw]
        return (info >> 16).view(self.th, self.tw)


def evaluate(net, n_frames=1000, batch=16, seed_base=2_000_000, conf=0.9, W=1920, H=1080,
             baselines=True, workers=16, verbose=True):
    dev = torch.device("cuda")
    # batches of `batch` frames and a last, partial one for the remainder
    sizes = [batch] * (n_frames // batch) + ([n_frames % batch] if n_frames % batch else [])
    plans = {b: EvalPlans(W, H, b, dev) for b in sorted(set(sizes))}
    rand_net = ProposalNet(seed=12345) if baselines else None
    gpool = ThreadPoolExecutor(max_workers=workers)
    stream = torch.cuda.current_stream()
    agg = dict(m4=0, n4=0, m8=0, n8=0, l4=0, ln4=0, l8=0, ln8=0, lanes=0, lanes_solid=0,
               found_plain=0, found_pruned=0, found_plain_solid=0, found_pruned_solid=0,
               votes_plain=0, votes_pruned=0, tiles=0, t_skip=0,
               t_fall=0, t_band=0, ms_plain=0.0, ms_pruned=0.0, ms_cnn=0.0, frames=0)
    rnd = dict(m4=0, n4=0, m8=0, n8=0, votes=0)
    heur_stats = []  # per frame: (tile counts, plain peaks) for the budget-matched heuristic
    nb = len(sizes)
    scene = synth.scene_road(W, H)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    first = 0

    def run_pruned(P, mask_src):
        P.mask.copy_(mask_src)
        P.pruned_plan.launch(stream)
        torch.cuda.synchronize()
        out = []
        for fb in P.pruned:
            pk = fb.peaks.cpu().numpy()
            out.append((pk[:TOPK], pk[TOPK:2 * TOPK], int(pk[3 * TOPK]),
                        int(fb.acc.sum().item())))
        return out

    for bi in range(nb):
        batch = sizes[bi]
        P = plans[batch]
        seeds = [seed_base + first + i for i in range(batch)]
        first += batch
        frames = gen_batch(gpool, W, H, seeds)
        P.imgs.copy_(torch.from_numpy(frames))
        # plain
        P.plain_plan.launch(stream)
        # timing of the vote stages (after a full launch so the lists exist)
        ev[0].record(stream)
        P.plain_plan.launch_stage(2, stream)
        ev[1].record(stream)
        logits = net.forward(P.imgs, stream=stream)
        mask = torch.empty_like(P.mask)
        lane.mask_from_logits(logits, W, H, batch, conf, mask, stream)
        ev[2].record(stream)
        P.mask.copy_(mask)
        P.pruned_plan.launch(stream)
        ev[3].record(stream)
        P.pruned_plan.launch_stage(2, stream)
        ev[4].record(stream)
        torch.cuda.synchronize()
        agg["ms_plain"] += ev[0].elapsed_time(ev[1])
        agg["ms_cnn"] += ev[1].elapsed_time(ev[2])
        agg["ms_pruned"] += ev[3].elapsed_time(ev[4])
        m = mask.cpu().numpy()
        agg["tiles"] += m.size
        agg["t_skip"] += int((m == 0).sum())
        agg["t_fall"] += int((m == 0xFF).sum())
        agg["t_band"] += int(((m != 0) & (m != 0xFF)).sum())
        for b in range(batch):
            pp = P.plain[b].peaks.cpu().numpy()
            qq = P.pruned[b].peaks.cpu().numpy()
            pt, pr, pn = pp[:TOPK], pp[TOPK:2 * TOPK], int(pp[3 * TOPK])
            qt, qr, qn = qq[:TOPK], qq[TOPK:2 * TOPK], int(qq[3 * TOPK])
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 4, N_THETA, P.D)
            agg["m4"] += a
            agg["n4"] += n
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 8, N_THETA, P.D)
            agg["m8"] += a
            agg["n8"] += n
            segs = synth.lane_segments(scene, seeds[b])
            lf = lane_flags(segs, pt, pr, pn, N_THETA, P.D)
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 4, N_THETA, P.D, only=lf)
            agg["l4"] += a
            agg["ln4"] += n
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 8, N_THETA, P.D, only=lf)
            agg["l8"] += a
            agg["ln8"] += n
            fp = lanes_found(segs, pt, pr, pn, N_THETA, P.D)
            fq = lanes_found(segs, qt, qr, qn, N_THETA, P.D)
            solid = np.zeros(len(segs), bool)
            solid[[0, len(segs) - 1]] = True
            agg["lanes"] += len(segs)
            agg["lanes_solid"] += int(solid.sum())
            agg["found_plain"] += int(fp.sum())
            agg["found_pruned"] += int(fq.sum())
            agg["found_plain_solid"] += int((fp & solid).sum())
            agg["found_pruned_solid"] += int((fq & solid).sum())
            agg["votes_plain"] += int(P.plain[b].counters[0].item()) * N_THETA
            agg["votes_pruned"] += int(P.pruned[b].acc.sum().item())
            agg["frames"] += 1
            if baselines and bi < max(1, nb // 4):
                heur_stats.append((P.tile_counts(b).cpu().numpy(), (pt, pr, pn), frames[b],
                                   synth.lane_segments(scene, seeds[b])))
        if baselines:
            rl = rand_net.forward(P.imgs, stream=stream)
            rm = torch.empty_like(P.mask)
            lane.mask_from_logits(rl, W, H, batch, conf, rm, stream)
            res = run_pruned(P, rm)
            for b in range(batch):
                pp = P.plain[b].peaks.cpu().numpy()
                pt, pr, pn = pp[:TOPK], pp[TOPK:2 * TOPK], int(pp[3 * TOPK])
                qt, qr, qn, votes = res[b]
                a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 4, N_THETA, P.D)
                rnd["m4"] += a
                rnd["n4"] += n
                a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 8, N_THETA, P.D)
                rnd["m8"] += a
                rnd["n8"] += n
                rnd["votes"] += votes
        if verbose and (bi + 1) % 10 == 0:
            print(f"[eval] {agg['frames']} frames: agree@4 {agg['m4'] / max(1, agg['n4']):.4f} "
                  f"agree@8 {agg['m8'] / max(1, agg['n8']):.4f} votes "
                  f"{agg['votes_pruned'] / max(1, agg['votes_plain']):.3f}", flush=True)
    frac = agg["votes_pruned"] / max(1, agg["votes_plain"])
    res = dict(
        frames=agg["frames"], conf=conf, size=[W, H],
        agreement_top4=agg["m4"] / max(1, agg["n4"]),
        agreement_top8=agg["m8"] / max(1, agg["n8"]),
        lane_share_top4=agg["ln4"] / max(1, agg["n4"]),
        lane_share_top8=agg["ln8"] / max(1, agg["n8"]),
        agreement_top4_lane_peaks=agg["l4"] / max(1, agg["ln4"]),
        agreement_top8_lane_peaks=agg["l8"] / max(1, agg["ln8"]),
        lanes_found_top4_plain=agg["found_plain"] / max(1, agg["lanes"]),
        lanes_found_top4_pruned=agg["found_pruned"] / max(1, agg["lanes"]),
        solid_lanes_found_top4_plain=agg["found_plain_solid"] / max(1, agg["lanes_solid"]),
        solid_lanes_found_top4_pruned=agg["found_pruned_solid"] / max(1, agg["lanes_solid"]),
        missed_top4=1 - agg["m4"] / max(1, agg["n4"]),
        missed_top8=1 - agg["m8"] / max(1, agg["n8"]),
        votes_fraction=frac,
        tiles_band=agg["t_band"] / agg["tiles"], tiles_skip=agg["t_skip"] / agg["tiles"],
        tiles_fallback=agg["t_fall"] / agg["tiles"],
        vote_ms_per_frame_plain=agg["ms_plain"] / agg["frames"],
        vote_ms_per_frame_pruned=agg["ms_pruned"] / agg["frames"],
        cnn_mask_ms_per_frame=agg["ms_cnn"] / agg["frames"])
    if baselines:
        res["random_init"] = dict(
            agreement_top4=rnd["m4"] / max(1, rnd["n4"]), agreement_top8=rnd["m8"] / max(1, rnd["n8"]),
            votes_fraction=rnd["votes"] / max(1, agg["votes_plain"]))
        res["heuristic"] = heuristic_at_budget(plans[sizes[0]], heur_stats, frac)
    gpool.shutdown()
    for P in plans.values():
        P.plain_plan.close()
        P.pruned_plan.close()
    return res


def frontier(net, confs=(0.9, 0.99, 0.999, 0.9999), n_frames=1000, batch=20, verbose=True):
    """Agreement with the plain top-4 / top-8 against the votes kept, over
    mask confidences: a higher confidence sends more tiles to the full vote
    (fallback), trading vote savings for agreement."""
    rows = []
    for c in confs:
        r = evaluate(net, n_frames, batch, conf=c, baselines=False, verbose=verbose)
        rows.append({k: r[k] for k in ("conf", "frames", "agreement_top4", "agreement_top8",
                                       "missed_top4", "votes_fraction", "tiles_skip",
                                       "tiles_band", "tiles_fallback", "lanes_found_top4_pruned",
                                       "vote_ms_per_frame_plain", "vote_ms_per_frame_pruned")})
        if verbose:
            print("[frontier]", json.dumps(rows[-1]), flush=True)
    return rows


def heuristic_at_budget(P, stats, frac):
    """Keep tiles with >= tau edge pixels (every theta), tau the smallest
    whose votes do not exceed `frac` of plain; agreement on the same frames."""
    counts = np.stack([s[0] for s in stats]).astype(np.int64)
    total = counts.sum()
    tau = 0
    for t in range(0, 66):
        if counts[counts >= t].sum() <= frac * total:
            tau = t
            break
    else:
        tau = 65
    m4 = n4 = m8 = n8 = 0
    votes = 0
    found = lanes = 0
    B = P.B
    for i0 in range(0, len(stats), B):
        chunk = stats[i0:i0 + B]
        if len(chunk) < B:
            break
        P.imgs.copy_(torch.from_numpy(np.stack([c[2] for c in chunk])))
        hm = torch.from_numpy(np.where(np.stack([c[0] for c in chunk]) >= tau, 255, 0)
                              .astype(np.uint8)).cuda()
        P.mask.copy_(hm)
        P.pruned_plan.launch()
        torch.cuda.synchronize()
        for b, c in enumerate(chunk):
            pt, pr, pn = c[1]
            qq = P.pruned[b].peaks.cpu().numpy()
            qt, qr, qn = qq[:TOPK], qq[TOPK:2 * TOPK], int(qq[3 * TOPK])
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 4, N_THETA, P.D)
            m4 += a
            n4 += n
            a, n = agreement_counts(pt, pr, pn, qt, qr, qn, 8, N_THETA, P.D)
            m8 += a
            n8 += n
            votes += int(P.pruned[b].acc.sum().item())
            f = lanes_found(c[3], qt, qr, qn, N_THETA, P.D)
            found += int(f.sum())
            lanes += len(f)
    plain_votes = int(counts.sum()) * N_THETA
    return dict(tau=tau, agreement_top4=m4 / max(1, n4), agreement_top8=m8 / max(1, n8),
                votes_fraction=votes / max(1, plain_votes), frames=len(stats),
                lanes_found_top4=found / max(1, lanes))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", required=True)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--conf", type=float, nargs="+", default=[0.9])
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--frontier", action="store_true",
                    help="agreement against votes kept for every --conf (no baselines)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    net, _ = ProposalNet.load(a.weights)
    if a.frontier:
        rows = frontier(net, a.conf, a.frames, a.batch)
        if a.out:
            json.dump(rows, open(a.out, "w"), indent=1)
        return
    allres = []
    for c in a.conf:
        res = evaluate(net, a.frames, a.batch, conf=c, baselines=not a.no_baselines)
        print(json.dumps(res), flush=True)
        allres.append(res)
    if a.out:
        json.dump(allres if len(allres) > 1 else allres[0], open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
