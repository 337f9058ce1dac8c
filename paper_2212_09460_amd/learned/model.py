"""ProposalNet: host-side handle of the CNN whose kernels live in liblane.so.

Keeps the FP32 master parameters, Adam moments and the packed FP16 kernel
weights on the device, plus per-(size, batch) workspaces.  Checkpoints are
plain .npz files (arrays only; loaded with allow_pickle=False).
"""
from __future__ import annotations

import math
import os

import numpy as np
import torch

from .. import lane

# (c_in, c_out) per layer, master layout: weights [c_out][c_in][3][3], biases [c_out]
LAYERS = ((1, 16), (16, 16), (16, 16), (16, 9))


WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def default_weights() -> str:
    """The trained proposal weights shipped with the package."""
    return os.path.join(WEIGHTS_DIR, "proposal.npz")


def load_params(path: str | None = None) -> np.ndarray:
    """FP32 master parameters from a checkpoint (host array)."""
    z = np.load(default_weights() if path is None else path, allow_pickle=False)
    return np.asarray(z["params"], np.float32)


def he_uniform(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in LAYERS:
        lim = math.sqrt(6.0 / (ci * 9))
        parts.append(rng.uniform(-lim, lim, size=co * ci * 9))
        parts.append(np.zeros(co))
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == lane.CNN_PARAMS
    return v


class ProposalNet:
    def __init__(self, params: np.ndarray | None = None, seed: int = 0, device="cuda"):
        self.device = torch.device(device)
        p = he_uniform(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p.copy()).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0
        pk_bytes, _, _ = lane.cnn_sizes(8, 8, 1)
        self.packed = lane._bytes_tensor(pk_bytes, self.device)
        self._ws = {}
        self.pack()

    def pack(self, stream=None):
        lane.cnn_pack(self.params, self.packed, stream)

    def workspace(self, W: int, H: int, batch: int):
        key = (W, H, batch)
        if key not in self._ws:
            _, act_b, part_b = lane.cnn_sizes(W, H, batch)
            th, tw = (H + 7) // 8, (W + 7) // 8
            self._ws[key] = dict(
                act=lane._bytes_tensor(act_b, self.device),
                partial=lane._bytes_tensor(part_b, self.device),
                logits=torch.empty((batch, 9, th, tw), dtype=torch.float32, device=self.device),
                loss=torch.empty(batch, dtype=torch.float32, device=self.device))
        return self._ws[key]

    def forward(self, imgs: torch.Tensor, W: int | None = None, stream=None) -> torch.Tensor:
        """imgs uint8 [B][H][pitch] -> logits float32 [B][9][th][tw] (a reused
        buffer), by the fused inference kernel."""
        B, H, pitch = imgs.shape
        W = pitch if W is None else W
        key = ("infer", W, H, B)
        if key not in self._ws:
            th, tw = (H + 7) // 8, (W + 7) // 8
            self._ws[key] = torch.empty((B, 9, th, tw), dtype=torch.float32, device=self.device)
        lane.cnn_infer(imgs, self.packed, self._ws[key], W, stream)
        return self._ws[key]

    def forward_layers(self, imgs: torch.Tensor, W: int | None = None, stream=None) -> torch.Tensor:
        """The same logits through the layer-by-layer kernels the training
        uses (activations kept in the workspace for a backward pass)."""
        B, H, pitch = imgs.shape
        W = pitch if W is None else W
        ws = self.workspace(W, H, B)
        lane.cnn_forward(imgs, self.packed, ws["act"], ws["logits"], W, stream)
        return ws["logits"]

    def train_step(self, imgs: torch.Tensor, keep: torch.Tensor, bands: torch.Tensor, lr: float,
                   W: int | None = None, stream=None) -> torch.Tensor:
        """One Adam step on a batch; returns the per-frame losses (device)."""
        B, H, pitch = imgs.shape
        W = pitch if W is None else W
        ws = self.workspace(W, H, B)
        th, tw = (H + 7) // 8, (W + 7) // 8
        scale = float(th * tw)  # loss scale: keeps the FP16 logit gradients O(1)
        lane.cnn_forward(imgs, self.packed, ws["act"], ws["logits"], W, stream)
        lane.cnn_loss(ws["logits"], keep, bands, W, H, B, scale, ws["act"], ws["loss"], stream)
        lane.cnn_backward(imgs, self.packed, ws["act"], ws["partial"], self.grads, W, stream)
        self.step += 1
        lane.adam_step(self.params, self.grads, self.m, self.v, lr, self.step, 1.0 / (scale * B),
                       stream=stream)
        self.pack(stream)
        return ws["loss"]

    def state(self) -> dict:
        return dict(params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                    v=self.v.cpu().numpy(), step=np.array(self.step, np.int64))

    def save(self, path: str, **extra):
        np.savez(path, **self.state(), **{k: np.asarray(v) for k, v in extra.items()})

    @classmethod
    def load(cls, path: str, device="cuda"):
        z = np.load(path, allow_pickle=False)
        net = cls(z["params"], device=device)
        if "m" in z:
            net.m.copy_(torch.from_numpy(z["m"]))
            net.v.copy_(torch.from_numpy(z["v"]))
            net.step = int(z["step"])
        return net, {k: z[k] for k in z.files}
