"""Thin Python binding of liblane.so (the C ABI in include/lane.h).

Argument marshalling only: every step of the path runs in the HIP kernels.
torch tensors provide device memory and the current HIP stream.  If the
library is missing this module raises at import time; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblane.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2212_09460_amd.build.build()")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t


def _sig(name, args):
    f = getattr(_lib, name)
    f.restype = ctypes.c_int
    f.argtypes = args
    return f


_lib.lane_strerror.restype = ctypes.c_char_p
_lib.lane_strerror.argtypes = [ctypes.c_int]
_abi_version = _sig("lane_abi_version", [])
_make_trig = _sig("lane_make_trig_q14", [_i32, _vp, _vp])
_r_offset = _sig("lane_r_offset", [_i32, _i32, ctypes.POINTER(_i32)])
_list_size = _sig("lane_edge_list_size", [_i32, _i32, ctypes.POINTER(_sz)])
_sobel = _sig("lane_sobel_binarize", [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp])
_edges_to_list = _sig("lane_edges_to_list", [_vp, _i32, _i32, _i32, _vp, _vp, _vp])
_vote = _sig("lane_hough_vote", [_vp, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp])
_peaks_ws = _sig("lane_hough_peaks_workspace_size", [_i32, _i32, ctypes.POINTER(_sz)])
_peaks = _sig("lane_hough_peaks", [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp,
                                    _vp, _vp, _sz, _vp])

LANE_OK = 0
LANE_BORDER_ZERO = 0
LANE_BORDER_ZERO_MASKRING = 1

# Exported entry points of the C ABI (also checked by the CPU tests).
EXPORTS = ("lane_abi_version", "lane_strerror", "lane_make_trig_q14", "lane_r_offset",
           "lane_edge_list_size", "lane_sobel_binarize", "lane_edges_to_list", "lane_hough_vote",
           "lane_hough_peaks_workspace_size", "lane_hough_peaks")


class LaneError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_lib.lane_strerror(code).decode()} ({code})")
        self.code = code


def _check(code: int, what: str):
    if code != LANE_OK:
        raise LaneError(code, what)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def abi_version() -> int:
    return int(_abi_version())


def make_trig_q14(n_theta: int):
    import numpy as np

    c = np.zeros(n_theta, np.int16)
    s = np.zeros(n_theta, np.int16)
    _check(_make_trig(n_theta, c.ctypes.data, s.ctypes.data), "lane_make_trig_q14")
    return c, s


def r_offset(W: int, H: int) -> int:
    d = _i32(0)
    _check(_r_offset(W, H, ctypes.byref(d)), "lane_r_offset")
    return int(d.value)


def edge_list_size(W: int, H: int) -> int:
    n = _sz(0)
    _check(_list_size(W, H, ctypes.byref(n)), "lane_edge_list_size")
    return int(n.value)


def peaks_workspace_size(n_theta: int, n_r: int) -> int:
    n = _sz(0)
    _check(_peaks_ws(n_theta, n_r, ctypes.byref(n)), "lane_hough_peaks_workspace_size")
    return int(n.value)


def new_edge_list(W: int, H: int, device="cuda") -> torch.Tensor:
    return torch.empty(edge_list_size(W, H) // 4, dtype=torch.int32, device=device)


def sobel_binarize(img: torch.Tensor, W: int | None = None, threshold: int = 128,
                   border_mode: int = LANE_BORDER_ZERO_MASKRING, edges=None, mag=None,
                   edge_list=None, edge_count=None, want_mag: bool = False,
                   want_list: bool = True, stream=None):
    """img: uint8 [H][pitch] on the GPU.  Returns (edges, mag, list, count)."""
    H, pitch = img.shape
    W = pitch if W is None else W
    dev = img.device
    if edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=dev)
    if mag is None and want_mag:
        mag = torch.empty((H, W), dtype=torch.uint8, device=dev)
    if edge_list is None and want_list:
        edge_list = new_edge_list(W, H, dev)
    if edge_count is None:
        edge_count = torch.empty(1, dtype=torch.int32, device=dev)
    _check(_sobel(_p(img), W, H, pitch, int(threshold), int(border_mode), _p(edges), _p(mag),
                  _p(edge_list), _p(edge_count), _stream(stream)), "lane_sobel_binarize")
    return edges, mag, edge_list, edge_count


def edges_to_list(edges: torch.Tensor, W: int | None = None, edge_list=None, edge_count=None,
                  stream=None):
    H, pitch = edges.shape
    W = pitch if W is None else W
    if edge_list is None:
        edge_list = new_edge_list(W, H, edges.device)
    if edge_count is None:
        edge_count = torch.empty(1, dtype=torch.int32, device=edges.device)
    _check(_edges_to_list(_p(edges), W, H, pitch, _p(edge_list), _p(edge_count), _stream(stream)),
           "lane_edges_to_list")
    return edge_list, edge_count


def hough_vote(edge_list: torch.Tensor, W: int, H: int, cos_q14: torch.Tensor,
               sin_q14: torch.Tensor, r_offset: int, n_r: int, tile_mask=None, acc=None,
               dropped=None, stream=None):
    n_theta = cos_q14.shape[0]
    if acc is None:
        acc = torch.empty((n_theta, n_r), dtype=torch.int32, device=edge_list.device)
    if dropped is None:
        dropped = torch.empty(1, dtype=torch.int32, device=edge_list.device)
    _check(_vote(_p(edge_list), W, H, _p(cos_q14), _p(sin_q14), n_theta, int(r_offset), int(n_r),
                 _p(tile_mask), _p(acc), _p(dropped), _stream(stream)), "lane_hough_vote")
    return acc, dropped


def hough_peaks(acc: torch.Tensor, r_offset: int, k: int, h_theta: int | None = None,
                h_r: int | None = None, min_votes: int = 1, out=None, ws=None, stream=None):
    """Returns (theta_idx, r_idx, votes, count) int32 device tensors."""
    n_theta, n_r = acc.shape
    if h_theta is None:
        h_theta = max(1, -(-n_theta // 100))
    if h_r is None:
        h_r = max(1, -(-n_r // 100))
    dev = acc.device
    if out is None:
        out = torch.empty((3 * k + 1,), dtype=torch.int32, device=dev)
    t, r, v, c = out[0:k], out[k:2 * k], out[2 * k:3 * k], out[3 * k:3 * k + 1]
    if ws is None:
        ws = torch.empty(peaks_workspace_size(n_theta, n_r) // 8 + 2, dtype=torch.int64, device=dev)
    _check(_peaks(_p(acc), n_theta, n_r, int(r_offset), int(k), int(h_theta), int(h_r),
                  int(min_votes), _p(t), _p(r), _p(v), _p(c), _p(ws), ws.numel() * 8,
                  _stream(stream)), "lane_hough_peaks")
    return t, r, v, c


def pipeline(img: torch.Tensor, cos_q14: torch.Tensor, sin_q14: torch.Tensor, k: int,
             threshold: int = 128, border_mode: int = LANE_BORDER_ZERO_MASKRING, tile_mask=None,
             want_mag: bool = False, stream=None):
    """Sobel -> binarize -> compaction -> vote -> peaks for one frame."""
    H, W = img.shape
    D = r_offset(W, H)
    n_r = 2 * D + 1
    edges, mag, lst, cnt = sobel_binarize(img, W, threshold, border_mode, want_mag=want_mag,
                                          stream=stream)
    acc, dropped = hough_vote(lst, W, H, cos_q14, sin_q14, D, n_r, tile_mask, stream=stream)
    t, r, v, c = hough_peaks(acc, D, k, stream=stream)
    return dict(edges=edges, mag=mag, edge_list=lst, n_edges=cnt, acc=acc, dropped=dropped,
                theta_idx=t, r_idx=r, votes=v, count=c, D=D, n_r=n_r)
