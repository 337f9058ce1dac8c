"""Autotuner front end with a JSON cache.

The tuning itself is native (lane_tune_run in the C ABI): it times every
theta-slice width and work distribution of the vote and every Sobel strip
height / persistent grid size on a batch of copies of a sample frame and
keeps the fastest.  Results are cached per (device, frame size, theta bins,
batch size) in a JSON file (LANE_TUNE_CACHE, default
~/.cache/lane_tune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import lane


def cache_path() -> str:
    return os.environ.get("LANE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lane_tune.json"))


def _key(W: int, H: int, n_theta: int, n_frames: int) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    return f"{arch.split(':')[0]}/{W}x{H}/theta{n_theta}/batch{n_frames}"


def tuned(sample: torch.Tensor, n_theta: int, n_frames: int, W: int | None = None,
          use_cache: bool = True) -> tuple[lane.LaneTune, dict]:
    """Tuned setting for frames like `sample` in batches of n_frames."""
    H, pitch = sample.shape
    W = pitch if W is None else W
    key = _key(W, H, n_theta, n_frames)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        d = cache[key]
        return lane.LaneTune(d["vote_rows"], d["vote_queue"], d["sobel_groups_per_cu"],
                             d["sobel_strip_rows"]), d
    t, vote_ms, sobel_ms = lane.tune_run(sample, n_theta, n_frames, W)
    d = lane.tune_dict(t)
    d.update({"vote_ms": round(vote_ms, 4), "sobel_ms": round(sobel_ms, 4)})
    if use_cache:
        cache[key] = d
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return t, d
