"""Train the proposal network on frames labelled by the plain pipeline.

Frames: seeded synthetic road frames (the same recipe as the 1080p workload:
4 lanes, clutter, salt) at 1280x720 and 1920x1080, alternating per batch,
seeds [seed_base, seed_base + n_frames).  For every batch the plain batched
path (Sobel -> vote -> top-8 peaks) runs on the GPU, the labels kernel marks
the tiles whose edge pixels vote for those peaks, and one Adam step of the
CNN follows -- forward, loss, backward and update all in liblane.so.
Frame generation runs on CPU threads one batch ahead of the GPU.

  python -m paper_2212_09460_amd.learned.train --frames 20000 --out ckpt.npz
"""
from __future__ import annotations

import argparse
import math
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .. import lane, synth
from .model import ProposalNet

SIZES = ((1280, 720), (1920, 1080))
N_THETA, TOPK = 360, 8


class LabelPlan:
    """Plain batched path over a reusable [B][H][W] image tensor, plus the
    per-frame label buffers."""

    def __init__(self, W: int, H: int, B: int, device="cuda", k: int = TOPK):
        self.W, self.H, self.B = W, H, B
        self.imgs = torch.empty((B, H, W), dtype=torch.uint8, device=device)
        C, S = synth.trig_q14(N_THETA)
        self.C, self.S = torch.from_numpy(C).to(device), torch.from_numpy(S).to(device)
        # the labels mark the tiles that vote for the top-k plain peaks
        self.fbs = [lane.FrameBuffers(self.imgs[b], W, N_THETA, k, self.C, self.S)
                    for b in range(B)]
        self.plan = lane.Batch(self.fbs)
        th, tw = (H + 7) // 8, (W + 7) // 8
        self.keep = torch.empty((B, th, tw), dtype=torch.uint8, device=device)
        self.bands = torch.empty_like(self.keep)

    def label(self, stream=None):
        self.plan.launch(stream)
        for b, fb in enumerate(self.fbs):
            lane.tile_labels(fb, self.keep[b], self.bands[b], stream)


def gen_batch(pool, W, H, seeds):
    sc = synth.scene_road(W, H)
    return np.stack(list(pool.map(lambda s: synth.gen_frame(sc, s), seeds)))


def lr_at(step, total, lr0, lr_min):
    return lr_min + 0.5 * (lr0 - lr_min) * (1 + math.cos(math.pi * min(1.0, step / max(1, total))))


def train(n_frames=20000, batch=16, lr=2e-3, lr_min=1e-4, seed_base=1_000_000, out=None,
          resume=None, log_every=50, ckpt_every=250, workers=16, init_seed=0, max_seconds=None,
          verbose=True, epochs=1, label_k=TOPK):
    """Adam over `epochs` passes of the n_frames training frames (the same
    seeds each pass, each seed always at the same size), cosine LR decay over
    all steps.  label_k: the labels come from the top-label_k plain peaks."""
    dev = torch.device("cuda")
    if resume and os.path.exists(resume):
        net, meta = ProposalNet.load(resume)
        start = int(meta.get("cursor", net.step))
    else:
        net, start = ProposalNet(seed=init_seed), 0
    plans = {sz: LabelPlan(sz[0], sz[1], batch, dev, label_k) for sz in SIZES}
    per_epoch = n_frames // batch
    total = per_epoch * epochs
    pool = ThreadPoolExecutor(max_workers=workers)
    nxt = None
    t0 = time.time()
    losses = []
    hist = []

    def submit(step):
        W, H = SIZES[(step % per_epoch) % 2]
        seeds = [seed_base + (step % per_epoch) * batch + i for i in range(batch)]
        return pool.submit(gen_batch, pool_gen, W, H, seeds)

    pool_gen = ThreadPoolExecutor(max_workers=workers)
    if start < total:
        nxt = submit(start)
    for step in range(start, total):
        W, H = SIZES[(step % per_epoch) % 2]
        frames = nxt.result()
        nxt = submit(step + 1) if step + 1 < total else None
        p = plans[(W, H)]
        p.imgs.copy_(torch.from_numpy(frames), non_blocking=False)
        p.label()
        loss = net.train_step(p.imgs, p.keep, p.bands, lr_at(step, total, lr, lr_min))
        losses.append(loss)
        if (step + 1) % log_every == 0 or step + 1 == total:
            l = torch.stack(losses).mean().item()
            losses = []
            hist.append((step + 1, l))
            if verbose:
                print(f"[train] step {step + 1}/{total} frames {(step + 1) * batch} loss {l:.4f} "
                      f"lr {lr_at(step, total, lr, lr_min):.2e} {time.time() - t0:.1f}s", flush=True)
        if out and ((step + 1) % ckpt_every == 0 or step + 1 == total):
            net.save(out, cursor=np.array(step + 1, np.int64), seed_base=np.array(seed_base),
                     batch=np.array(batch), n_frames=np.array(n_frames), label_k=np.array(label_k))
        if max_seconds and time.time() - t0 > max_seconds:
            if verbose:
                print(f"[train] stopping at step {step + 1} (time limit)", flush=True)
            if out:
                net.save(out, cursor=np.array(step + 1, np.int64), seed_base=np.array(seed_base),
                         batch=np.array(batch), n_frames=np.array(n_frames),
                         label_k=np.array(label_k))
            break
    pool.shutdown()
    pool_gen.shutdown()
    torch.cuda.synchronize()
    return net, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default="proposal_ckpt.npz")
    ap.add_argument("--resume", default=None)
    ap.add_argument("--max-seconds", type=float, default=None)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--label-k", type=int, default=TOPK,
                    help="labels from the top-k plain peaks (default 8)")
    a = ap.parse_args()
    train(a.frames, a.batch, a.lr, out=a.out, resume=a.resume, max_seconds=a.max_seconds,
          workers=a.workers, epochs=a.epochs, label_k=a.label_k)


if __name__ == "__main__":
    main()
