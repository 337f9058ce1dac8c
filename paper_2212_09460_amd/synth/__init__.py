"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module draws frames and tabulates the Q14 cos/sin table; it holds none
of the lane-detection arithmetic (no gradient, threshold, vote or peak).  The
C source ``lanesynth.c`` documents the random-number recipe.

The frames stand in for the paper's single 512x512 road image (Sec. 5,
Fig. 9), which is not available: Gaussian gray background, bright straight
lane bands toward a vanishing point, optional clutter segments and salt noise.

Workload recipes (one function per named workload):
  * ``plain_640``  : 640x480, 2 solid lanes, no clutter, no salt, 180 theta.
  * ``plain_1080`` : 1920x1080, 4 lanes (inner two dashed), 200 clutter
    segments, 2 % salt, 360 theta.
  * ``mixed_batch``: 64 frames, 16 each at 640x480, 1280x720, 1920x1080 and
    3840x2160, 2..6 lanes, clutter and salt as in ``plain_1080``.
  * ``road``       : any size, lanes/clutter/salt as in ``plain_1080`` (used
    for training/eval sets and serving streams).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblanesynth.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile lanesynth.c with gcc into liblanesynth.so (always recompiles)."""
    import subprocess

    src = os.path.join(_HERE, "lanesynth.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Scene(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int), ("H", ctypes.c_int), ("n_lanes", ctypes.c_int),
                ("dashed_mask", ctypes.c_uint32), ("n_clutter", ctypes.c_int),
                ("salt_p", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.ls_frame_seed.restype = ctypes.c_uint64
        lib.ls_frame_seed.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
        lib.ls_gen_frame.restype = ctypes.c_int
        lib.ls_gen_frame.argtypes = [ctypes.POINTER(_Scene), ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_int]
        lib.ls_lane_segments.restype = ctypes.c_int
        lib.ls_lane_segments.argtypes = [ctypes.POINTER(_Scene), ctypes.c_uint64,
                                         ctypes.c_void_p]
        lib.ls_seed_uint.restype = ctypes.c_int64
        lib.ls_seed_uint.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        lib.ls_seed_u01.restype = None
        lib.ls_seed_u01.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        lib.ls_trig_q14.restype = ctypes.c_int
        lib.ls_trig_q14.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib.ls_crc32.restype = ctypes.c_uint32
        lib.ls_crc32.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Scene:
    W: int
    H: int
    n_lanes: int = 4
    dashed_mask: int = 0
    n_clutter: int = 0
    salt_p: float = 0.0

    def _c(self) -> _Scene:
        return _Scene(self.W, self.H, self.n_lanes, self.dashed_mask, self.n_clutter,
                      self.salt_p)


def inner_dashed(n_lanes: int) -> int:
    """Bit mask marking every lane except the two outermost as dashed."""
    m = 0
    for i in range(1, n_lanes - 1):
        m |= 1 << i
    return m


def frame_seed(base_seed: int, config_id: int, index: int) -> int:
    return int(_load().ls_frame_seed(base_seed & (2**64 - 1), config_id, index & (2**64 - 1)))


def gen_frame(scene: Scene, seed: int, pitch: int | None = None) -> np.ndarray:
    """Return a uint8 array [H][pitch] (columns >= W are zero)."""
    pitch = scene.W if pitch is None else pitch
    out = np.zeros((scene.H, pitch), dtype=np.uint8)
    sc = scene._c()
    rc = _load().ls_gen_frame(ctypes.byref(sc), seed & (2**64 - 1),
                              out.ctypes.data, pitch)
    if rc != 0:
        raise ValueError(f"bad scene {scene}")
    return out


def lane_segments(scene: Scene, seed: int) -> np.ndarray:
    out = np.zeros((max(scene.n_lanes, 1), 4), dtype=np.float64)
    sc = scene._c()
    _load().ls_lane_segments(ctypes.byref(sc), seed & (2**64 - 1), out.ctypes.data)
    return out[: scene.n_lanes]


def seed_uint(seed: int, a: int, b: int) -> int:
    return int(_load().ls_seed_uint(seed & (2**64 - 1), a, b))


def seed_u01(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _load().ls_seed_u01(seed & (2**64 - 1), n, out.ctypes.data)
    return out


def trig_q14(n_theta: int) -> tuple[np.ndarray, np.ndarray]:
    """Q14 cos/sin table for theta_k = k*180/n_theta degrees, k in [0, n_theta)."""
    c = np.zeros(n_theta, dtype=np.int16)
    s = np.zeros(n_theta, dtype=np.int16)
    if _load().ls_trig_q14(n_theta, c.ctypes.data, s.ctypes.data) != 0:
        raise ValueError("n_theta must be positive")
    return c, s


def crc32(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a)
    return int(_load().ls_crc32(a.ctypes.data, a.nbytes))


# ----------------------------------------------------------- workloads --

CONFIG_PLAIN_640 = 0
CONFIG_PLAIN_1080 = 1
CONFIG_MIXED_BATCH = 2
CONFIG_TRAIN = 3
CONFIG_SERVE = 4

MIXED_SIZES = ((640, 480), (1280, 720), (1920, 1080), (3840, 2160))


def scene_plain_640() -> Scene:
    return Scene(640, 480, n_lanes=2, dashed_mask=0, n_clutter=0, salt_p=0.0)


def scene_road(W: int, H: int, n_lanes: int = 4) -> Scene:
    return Scene(W, H, n_lanes=n_lanes, dashed_mask=inner_dashed(n_lanes),
                 n_clutter=200, salt_p=0.02)


def plain_640(index: int = 0, base_seed: int = 0) -> np.ndarray:
    return gen_frame(scene_plain_640(), frame_seed(base_seed, CONFIG_PLAIN_640, index))


def plain_1080(index: int = 0, base_seed: int = 0) -> np.ndarray:
    return gen_frame(scene_road(1920, 1080), frame_seed(base_seed, CONFIG_PLAIN_1080, index))


def mixed_batch_scene(index: int, base_seed: int = 0) -> tuple[Scene, int]:
    """Scene and seed of frame ``index`` (0..63) of the mixed-resolution batch."""
    W, H = MIXED_SIZES[(index // 16) % 4]
    seed = frame_seed(base_seed, CONFIG_MIXED_BATCH, index)
    n_lanes = seed_uint(seed, 2, 6)
    return scene_road(W, H, n_lanes), seed


def mixed_batch(index: int, base_seed: int = 0) -> np.ndarray:
    sc, seed = mixed_batch_scene(index, base_seed)
    return gen_frame(sc, seed)


def road(W: int, H: int, seed: int, n_lanes: int = 4) -> np.ndarray:
    return gen_frame(scene_road(W, H, n_lanes), seed)


def theta_bins(config_id: int) -> int:
    return 180 if config_id == CONFIG_PLAIN_640 else 360


def r_offset(W: int, H: int) -> int:
    """D = ceil(sqrt((W-1)^2 + (H-1)^2)), by exact integer square root."""
    import math

    q = (W - 1) ** 2 + (H - 1) ** 2
    d = math.isqrt(q)
    return d if d * d == q else d + 1
