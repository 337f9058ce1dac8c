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
# LANE_LIB_PATH: another build of the same sources (the host-sanitizer test)
LIB_PATH = os.environ.get("LANE_LIB_PATH") or os.path.join(_HERE, "liblane.so")

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
_vote_paired = _sig("lane_hough_vote_paired", [_vp, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _i32, _vp,
                                                _vp, _vp])
_peaks_ws = _sig("lane_hough_peaks_workspace_size", [_i32, _i32, ctypes.POINTER(_sz)])
_peaks = _sig("lane_hough_peaks", [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp,
                                    _vp, _vp, _sz, _vp])
_peaks_noalloc = _sig("lane_hough_peaks_noalloc", [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32,
                                                  _vp, _vp, _vp, _vp, _vp])
_lib.lane_hough_peaks_noalloc_max_bytes.restype = _sz
_lib.lane_hough_peaks_noalloc_max_bytes.argtypes = []
_canny_ws = _sig("lane_canny_workspace_size", [_i32, _i32, ctypes.POINTER(_sz)])
_canny = _sig("lane_canny", [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz,
                              _vp])
_lines = _sig("lane_hough_lines", [_vp, _i32, _i32, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _i32, _i32,
                                    _i32, _i32, _vp, _vp, _vp, _vp])

PROGRESSIVE_FIELDS = ("theta_step", "r_width", "k_coarse", "h_theta_coarse", "h_r_coarse",
                      "min_votes_coarse", "margin_theta", "margin_r", "k", "h_theta", "h_r",
                      "min_votes")


class LaneProgressive(ctypes.Structure):
    _fields_ = [(n, _i32) for n in PROGRESSIVE_FIELDS]


class LaneProgressiveLayout(ctypes.Structure):
    _fields_ = [("n_coarse_theta", _i32), ("n_coarse_r", _i32), ("coarse_r_offset", _i32),
                ("win_rows", _i32), ("win_cols", _i32), ("coarse_acc", _sz), ("coarse_peaks", _sz),
                ("windows", _sz), ("candidates", _sz), ("bytes", _sz)]


_prog_layout = _sig("lane_hough_progressive_layout", [_i32, _i32, _i32, _i32,
                                                       ctypes.POINTER(LaneProgressive),
                                                       ctypes.POINTER(LaneProgressiveLayout)])
_prog = _sig("lane_hough_progressive", [_vp, _i32, _i32, _vp, _vp, _i32, _i32,
                                         ctypes.POINTER(LaneProgressive), _vp, _vp, _vp, _vp, _vp,
                                         _sz, _vp])

LANE_OK = 0
LANE_BORDER_ZERO = 0
LANE_BORDER_ZERO_MASKRING = 1

# Exported entry points of the C ABI (also checked by the CPU tests).
EXPORTS = ("lane_abi_version", "lane_strerror", "lane_make_trig_q14", "lane_r_offset",
           "lane_edge_list_size", "lane_sobel_binarize", "lane_edges_to_list", "lane_hough_vote",
           "lane_hough_vote_paired",
           "lane_hough_peaks_workspace_size", "lane_hough_peaks", "lane_hough_peaks_noalloc",
           "lane_hough_peaks_noalloc_max_bytes", "lane_hough_lines",
           "lane_canny_workspace_size", "lane_canny", "lane_hough_progressive_layout",
           "lane_hough_progressive", "lane_batch_create",
           "lane_batch_launch", "lane_batch_launch_stage", "lane_batch_destroy", "lane_tune_run",
           "lane_tune_batch",
           "lane_cnn_param_count", "lane_cnn_sizes", "lane_cnn_pack", "lane_cnn_forward",
           "lane_cnn_loss", "lane_cnn_backward", "lane_adam_step", "lane_tile_labels",
           "lane_mask_from_logits", "lane_cnn_infer", "lane_batch_active_flags", "lane_batch_select", "lane_server_plan",
           "lane_server_create", "lane_server_submit", "lane_server_poll", "lane_server_replay",
           "lane_server_stats_get", "lane_server_destroy", "lane_server_pause")


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


def hough_vote_paired(edge_list: torch.Tensor, W: int, H: int, cos_q14: torch.Tensor,
                      sin_q14: torch.Tensor, r_offset: int, n_r: int, pairing: int = 1, acc=None,
                      dropped=None, stream=None):
    """Vote with rows k and n - k sharing their products (pairing=1) or not
    (pairing=0).  Returns (acc, dropped) device tensors."""
    n_theta = cos_q14.shape[0]
    dev = edge_list.device
    if acc is None:
        acc = torch.empty((n_theta, n_r), dtype=torch.int32, device=dev)
    if dropped is None:
        dropped = torch.empty((1,), dtype=torch.int32, device=dev)
    _check(_vote_paired(_p(edge_list), W, H, _p(cos_q14), _p(sin_q14), n_theta, int(r_offset),
                        int(n_r), int(pairing), _p(acc), _p(dropped), _stream(stream)),
           "lane_hough_vote_paired")
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


def hough_peaks_noalloc(acc: torch.Tensor, r_offset: int, k: int, h_theta: int | None = None,
                        h_r: int | None = None, min_votes: int = 1, out=None, stream=None):
    """lane_hough_peaks_noalloc: the peak search with the library's own fixed
    device scratch (no workspace).  Returns (theta_idx, r_idx, votes, count)."""
    n_theta, n_r = acc.shape
    if h_theta is None:
        h_theta = max(1, -(-n_theta // 100))
    if h_r is None:
        h_r = max(1, -(-n_r // 100))
    if out is None:
        out = torch.empty((3 * k + 1,), dtype=torch.int32, device=acc.device)
    t, r, v, c = out[0:k], out[k:2 * k], out[2 * k:3 * k], out[3 * k:3 * k + 1]
    _check(_peaks_noalloc(_p(acc), n_theta, n_r, int(r_offset), int(k), int(h_theta), int(h_r),
                          int(min_votes), _p(t), _p(r), _p(v), _p(c), _stream(stream)),
           "lane_hough_peaks_noalloc")
    return t, r, v, c


def peaks_noalloc_max_bytes() -> int:
    return int(_lib.lane_hough_peaks_noalloc_max_bytes())


def progressive_params(n_theta: int, n_r: int, **over) -> dict:
    """Parameters of the coarse-to-fine Hough: 4-row coarse steps, 9-cell r
    bins, 16 coarse peaks, windows widened by 2 rows and 6 cells, 8 final
    peaks with the default windows of hough_peaks; keywords override."""
    p = dict(theta_step=4, r_width=9, k_coarse=16, h_theta_coarse=1, h_r_coarse=2,
             min_votes_coarse=1, margin_theta=2, margin_r=6, k=8,
             h_theta=max(1, -(-n_theta // 100)), h_r=max(1, -(-n_r // 100)), min_votes=1)
    unknown = set(over) - set(p)
    if unknown:
        raise TypeError(f"unknown progressive parameters {sorted(unknown)}")
    p.update(over)
    return p


def _prog_struct(params: dict) -> LaneProgressive:
    if set(params) != set(PROGRESSIVE_FIELDS):
        raise TypeError(f"progressive parameters must be exactly {PROGRESSIVE_FIELDS}")
    return LaneProgressive(*[int(params[n]) for n in PROGRESSIVE_FIELDS])


def progressive_layout(W: int, H: int, n_theta: int, r_offset: int, params: dict) -> dict:
    lay = LaneProgressiveLayout()
    p = _prog_struct(params)
    _check(_prog_layout(W, H, n_theta, int(r_offset), ctypes.byref(p), ctypes.byref(lay)),
           "lane_hough_progressive_layout")
    return {n: getattr(lay, n) for n, _ in LaneProgressiveLayout._fields_}


def hough_progressive(lst: torch.Tensor, W: int, H: int, C: torch.Tensor, S: torch.Tensor,
                      r_offset: int, params: dict, ws=None, out=None, stream=None):
    """Coarse-to-fine Hough (see lane_hough_progressive).  Returns
    (theta_idx, r_idx, votes, count, detail); detail holds device views of the
    intermediate results in the workspace (coarse_acc, coarse_peaks, windows,
    candidates)."""
    n_theta = C.shape[0]
    lay = progressive_layout(W, H, n_theta, r_offset, params)
    k, kc = int(params["k"]), int(params["k_coarse"])
    dev = lst.device
    if out is None:
        out = torch.empty((3 * k + 1,), dtype=torch.int32, device=dev)
    t, r, v, c = out[0:k], out[k:2 * k], out[2 * k:3 * k], out[3 * k:3 * k + 1]
    if ws is None:
        ws = torch.empty(lay["bytes"] // 8 + 2, dtype=torch.int64, device=dev)
    if ws.numel() * ws.element_size() < lay["bytes"]:
        raise ValueError("progressive workspace too small")
    p = _prog_struct(params)
    _check(_prog(_p(lst), W, H, _p(C), _p(S), n_theta, int(r_offset), ctypes.byref(p), _p(t),
                 _p(r), _p(v), _p(c), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "lane_hough_progressive")
    b = ws.view(torch.uint8)

    def i32(off, n):
        return b[off:off + 4 * n].view(torch.int32)

    n_c, n_rc, R, Wc = lay["n_coarse_theta"], lay["n_coarse_r"], lay["win_rows"], lay["win_cols"]
    detail = dict(layout=lay, coarse_acc=i32(lay["coarse_acc"], n_c * n_rc).view(n_c, n_rc),
                  coarse_peaks=i32(lay["coarse_peaks"], 3 * kc + 1),
                  windows=i32(lay["windows"], kc * R * Wc).view(kc, R, Wc),
                  candidates=i32(lay["candidates"], 3 * kc).view(kc, 3))
    return t, r, v, c, detail


def canny_workspace_size(W: int, H: int) -> int:
    n = _sz(0)
    _check(_canny_ws(W, H, ctypes.byref(n)), "lane_canny_workspace_size")
    return int(n.value)


def canny(img: torch.Tensor, W: int | None = None, t_low: int = 64, t_high: int = 128,
          border_mode: int = LANE_BORDER_ZERO_MASKRING, want_mag: bool = False,
          want_list: bool = True, ws=None, stream=None):
    """Canny edges (see lane_canny).  Returns (edges, mag or None, edge list or
    None, edge count) as device tensors."""
    H, pitch = img.shape
    W = pitch if W is None else W
    dev = img.device
    edges = torch.empty((H, W), dtype=torch.uint8, device=dev)
    mag = torch.empty((H, W), dtype=torch.uint8, device=dev) if want_mag else None
    lst = new_edge_list(W, H, dev) if want_list else None
    cnt = torch.empty((1,), dtype=torch.int32, device=dev)
    if ws is None:
        ws = torch.empty(canny_workspace_size(W, H) // 8 + 2, dtype=torch.int64, device=dev)
    _check(_canny(_p(img), W, H, pitch, int(t_low), int(t_high), int(border_mode), _p(edges),
                  _p(mag), _p(lst), _p(cnt), _p(ws), ws.numel() * 8, _stream(stream)), "lane_canny")
    return edges, mag, lst, cnt


def hough_lines(edges: torch.Tensor, cos_q14: torch.Tensor, sin_q14: torch.Tensor, r_offset: int,
                theta_idx: torch.Tensor, r_idx: torch.Tensor, count: torch.Tensor | None = None,
                fill_gap: int = 20, min_length: int = 40, max_segments: int = 16, W: int | None = None,
                stream=None, segments=None, seg_count=None, npts=None):
    """Line segments along peaks.  edges: device uint8 [H][W].  Returns
    (segments [k][max_segments][4], seg_count [k], npts [k]) int32 device tensors
    (the given output tensors, if any)."""
    H, pitch = edges.shape
    W = pitch if W is None else W
    assert W == pitch, "the edge map must be [H][W]"
    k = int(theta_idx.numel())
    dev = edges.device
    segs = torch.empty((k, max_segments, 4), dtype=torch.int32, device=dev) if segments is None else segments
    cnt = torch.empty((k,), dtype=torch.int32, device=dev) if seg_count is None else seg_count
    npts = torch.empty((k,), dtype=torch.int32, device=dev) if npts is None else npts
    _check(_lines(_p(edges), W, H, _p(cos_q14), _p(sin_q14), int(cos_q14.numel()), int(r_offset),
                  _p(theta_idx), _p(r_idx), None if count is None else _p(count), k, int(fill_gap),
                  int(min_length), int(max_segments), _p(segs), _p(cnt), _p(npts), _stream(stream)),
           "lane_hough_lines")
    return segs, cnt, npts


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


# ------------------------------------------------------------------ batch --

class LaneFrame(ctypes.Structure):
    _fields_ = [("img", _vp), ("W", _i32), ("H", _i32), ("pitch", _i32),
                ("threshold", _i32), ("border_mode", _i32),
                ("edges", _vp), ("mag_opt", _vp), ("list", _vp),
                ("cos_q14", _vp), ("sin_q14", _vp),
                ("n_theta", _i32), ("r_offset", _i32), ("n_r", _i32),
                ("tile_mask_opt", _vp), ("acc", _vp),
                ("k", _i32), ("h_theta", _i32), ("h_r", _i32), ("min_votes", _i32),
                ("peaks", _vp), ("peaks_ws", _vp), ("peaks_ws_bytes", _sz),
                ("counters_opt", _vp), ("lines_max_seg", _i32), ("lines_fill_gap", _i32),
                ("lines_min_length", _i32), ("lines_opt", _vp)]


class LaneTune(ctypes.Structure):
    _fields_ = [("vote_rows", _i32), ("vote_queue", _i32), ("sobel_groups_per_cu", _i32),
                ("sobel_strip_rows", _i32), ("vote_split", _i32)]


_batch_create = _sig("lane_batch_create", [ctypes.POINTER(LaneFrame), _i32,
                                           ctypes.POINTER(LaneTune), ctypes.POINTER(_vp)])
_batch_launch = _sig("lane_batch_launch", [_vp, _vp])
_batch_stage = _sig("lane_batch_launch_stage", [_vp, _i32, _vp])
_batch_destroy = _sig("lane_batch_destroy", [_vp])
_batch_flags = _sig("lane_batch_active_flags", [_vp, ctypes.POINTER(_vp)])
_batch_select = _sig("lane_batch_select", [_vp, _vp, _vp])
_tune_run = _sig("lane_tune_run", [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32,
                                   ctypes.POINTER(LaneTune), ctypes.POINTER(ctypes.c_float)])


def tune_run(sample: torch.Tensor, n_theta: int, n_frames: int, W: int | None = None,
             threshold: int = 128, border_mode: int = LANE_BORDER_ZERO_MASKRING):
    """Run the native autotuner on a device frame; returns (LaneTune, vote_ms, sobel_ms)."""
    H, pitch = sample.shape
    W = pitch if W is None else W
    t = LaneTune()
    ms = (ctypes.c_float * 2)()
    _check(_tune_run(_p(sample), W, H, pitch, threshold, border_mode, n_theta, n_frames,
                     ctypes.byref(t), ms), "lane_tune_run")
    return t, float(ms[0]), float(ms[1])


_tune_batch = _sig("lane_tune_batch", [ctypes.POINTER(LaneFrame), _i32, ctypes.POINTER(LaneTune),
                                       ctypes.POINTER(ctypes.c_float)])


def tune_batch(frames):
    """Run the native autotuner on the plan's own frames (FrameBuffers, any
    mix of sizes); returns (LaneTune, vote_ms, sobel_ms).  The plans it times
    write the frames' outputs."""
    arr = (LaneFrame * len(frames))(*[f.desc() for f in frames])
    t = LaneTune()
    ms = (ctypes.c_float * 2)()
    _check(_tune_batch(arr, len(frames), ctypes.byref(t), ms), "lane_tune_batch")
    return t, float(ms[0]), float(ms[1])


def tune_dict(t: LaneTune) -> dict:
    return {"vote_rows": t.vote_rows, "vote_queue": t.vote_queue,
            "sobel_groups_per_cu": t.sobel_groups_per_cu, "sobel_strip_rows": t.sobel_strip_rows,
            "vote_split": t.vote_split}


class FrameBuffers:
    """Device buffers of one frame for the batched path (allocated with torch)."""

    def __init__(self, img: torch.Tensor, W: int | None = None, n_theta: int = 360, k: int = 8,
                 cos_q14=None, sin_q14=None, threshold: int = 128,
                 border_mode: int = LANE_BORDER_ZERO_MASKRING, tile_mask=None,
                 want_mag: bool = False, h_theta=None, h_r=None, min_votes: int = 1,
                 lines_max_seg: int = 0, lines_fill_gap: int = 20, lines_min_length: int = 40):
        H, pitch = img.shape
        W = pitch if W is None else W
        dev = img.device
        self.img, self.W, self.H, self.pitch = img, W, H, pitch
        self.threshold, self.border_mode = threshold, border_mode
        self.D = r_offset(W, H)
        self.n_r = 2 * self.D + 1
        self.n_theta = n_theta if cos_q14 is None else cos_q14.shape[0]
        if cos_q14 is None:
            c, s = make_trig_q14(n_theta)
            cos_q14, sin_q14 = torch.from_numpy(c).to(dev), torch.from_numpy(s).to(dev)
        self.cos_q14, self.sin_q14 = cos_q14, sin_q14
        self.tile_mask = tile_mask
        self.edges = torch.empty((H, W), dtype=torch.uint8, device=dev)
        self.mag = torch.empty((H, W), dtype=torch.uint8, device=dev) if want_mag else None
        self.edge_list = new_edge_list(W, H, dev)
        self.acc = torch.empty((self.n_theta, self.n_r), dtype=torch.int32, device=dev)
        self.k = k
        self.h_theta = max(1, -(-self.n_theta // 100)) if h_theta is None else h_theta
        self.h_r = max(1, -(-self.n_r // 100)) if h_r is None else h_r
        self.min_votes = min_votes
        self.peaks = torch.empty(3 * k + 1, dtype=torch.int32, device=dev)
        nws = peaks_workspace_size(self.n_theta, self.n_r)
        self.peaks_ws = torch.empty(nws // 8 + 2, dtype=torch.int64, device=dev)
        self.counters = torch.empty(2, dtype=torch.int32, device=dev)
        # line segments along the peaks (the batch runs them after the peaks)
        self.lines_max_seg = lines_max_seg if k > 0 else 0
        self.lines_fill_gap, self.lines_min_length = lines_fill_gap, lines_min_length
        self.lines = (torch.empty(k * self.lines_max_seg * 4 + 2 * k, dtype=torch.int32, device=dev)
                      if self.lines_max_seg > 0 else None)

    def desc(self) -> LaneFrame:
        f = LaneFrame()
        f.img = self.img.data_ptr()
        f.W, f.H, f.pitch = self.W, self.H, self.pitch
        f.threshold, f.border_mode = self.threshold, self.border_mode
        f.edges = self.edges.data_ptr()
        f.mag_opt = None if self.mag is None else self.mag.data_ptr()
        f.list = self.edge_list.data_ptr()
        f.cos_q14, f.sin_q14 = self.cos_q14.data_ptr(), self.sin_q14.data_ptr()
        f.n_theta, f.r_offset, f.n_r = self.n_theta, self.D, self.n_r
        f.tile_mask_opt = None if self.tile_mask is None else self.tile_mask.data_ptr()
        f.acc = self.acc.data_ptr()
        f.k, f.h_theta, f.h_r, f.min_votes = self.k, self.h_theta, self.h_r, self.min_votes
        f.peaks = self.peaks.data_ptr() if self.k > 0 else None
        f.peaks_ws = self.peaks_ws.data_ptr()
        f.peaks_ws_bytes = self.peaks_ws.numel() * 8
        f.counters_opt = self.counters.data_ptr()
        if self.lines is not None:
            f.lines_max_seg = self.lines_max_seg
            f.lines_fill_gap, f.lines_min_length = self.lines_fill_gap, self.lines_min_length
            f.lines_opt = self.lines.data_ptr()
        return f

    def theta_idx(self):
        return self.peaks[0:self.k]

    def r_idx(self):
        return self.peaks[self.k:2 * self.k]

    def votes(self):
        return self.peaks[2 * self.k:3 * self.k]

    def count(self):
        return self.peaks[3 * self.k]

    def segments(self):
        """[k][lines_max_seg][4] int32 view (x1, y1, x2, y2)."""
        n = self.k * self.lines_max_seg * 4
        return self.lines[:n].view(self.k, self.lines_max_seg, 4)

    def seg_count(self):
        n = self.k * self.lines_max_seg * 4
        return self.lines[n:n + self.k]

    def line_npts(self):
        n = self.k * self.lines_max_seg * 4
        return self.lines[n + self.k:n + 2 * self.k]


class Batch:
    """A plan over a list of FrameBuffers: launch() runs the whole path for
    every frame as one graph launch."""

    def __init__(self, frames, vote_rows: int = 0, vote_queue: int = -1,
                 sobel_groups_per_cu: int = 0, sobel_strip_rows: int = 0, tune=None,
                 vote_split: int = 0):
        self.frames = list(frames)
        arr = (LaneFrame * len(self.frames))(*[f.desc() for f in self.frames])
        if tune is None:
            tune = LaneTune(vote_rows, vote_queue, sobel_groups_per_cu, sobel_strip_rows, vote_split)
        self.tune = tune
        h = _vp()
        _check(_batch_create(arr, len(self.frames), ctypes.byref(tune), ctypes.byref(h)),
               "lane_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(_batch_launch(self._h, _stream(stream)), "lane_batch_launch")

    def launch_stage(self, stage: int, stream=None):
        _check(_batch_stage(self._h, stage, _stream(stream)), "lane_batch_launch_stage")

    def select(self, active, stream=None):
        """Run only the frames whose entry of `active` is true in the next
        launches (their work lists are rebuilt on the host and copied in on
        `stream`).  Call again only after those launches have completed."""
        import numpy as np

        a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8))
        assert a.size == len(self.frames)
        _check(_batch_select(self._h, a.ctypes.data, _stream(stream)), "lane_batch_select")

    def active_flags_ptr(self) -> int:
        """Device address of the plan's per-frame switches (uint8 [n])."""
        p = _vp()
        _check(_batch_flags(self._h, ctypes.byref(p)), "lane_batch_active_flags")
        return int(p.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize()
            _batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- learned proposal --

_i64, _f32 = ctypes.c_int64, ctypes.c_float
_cnn_count = _sig("lane_cnn_param_count", [])
_cnn_sizes = _sig("lane_cnn_sizes", [_i32, _i32, _i32, ctypes.POINTER(_sz), ctypes.POINTER(_sz),
                                     ctypes.POINTER(_sz)])
_cnn_pack = _sig("lane_cnn_pack", [_vp, _vp, _vp])
_cnn_fwd = _sig("lane_cnn_forward", [_vp, _i32, _i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp])
_cnn_infer = _sig("lane_cnn_infer", [_vp, _i32, _i32, _i32, _i64, _i32, _vp, _vp, _vp])
_cnn_loss = _sig("lane_cnn_loss", [_vp, _vp, _vp, _i32, _i32, _i32, _f32, _vp, _vp, _vp])
_cnn_bwd = _sig("lane_cnn_backward", [_vp, _i32, _i32, _i32, _i64, _i32, _vp, _vp, _vp, _sz, _vp,
                                      _vp])
_adam = _sig("lane_adam_step", [_vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _i32, _f32, _vp])
_labels = _sig("lane_tile_labels", [_vp, _i32, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp,
                                    _vp])
_mask = _sig("lane_mask_from_logits", [_vp, _i32, _i32, _i32, _f32, _vp, _vp])

CNN_PARAMS = 6105


def cnn_param_count() -> int:
    return int(_cnn_count())


def cnn_sizes(W: int, H: int, batch: int):
    a, b, c = _sz(0), _sz(0), _sz(0)
    _check(_cnn_sizes(W, H, batch, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "lane_cnn_sizes")
    return int(a.value), int(b.value), int(c.value)


def _bytes_tensor(n: int, device):
    return torch.empty((n + 255) // 256 * 256, dtype=torch.uint8, device=device)


def cnn_pack(params: torch.Tensor, packed: torch.Tensor, stream=None):
    _check(_cnn_pack(_p(params), _p(packed), _stream(stream)), "lane_cnn_pack")


def cnn_forward(imgs: torch.Tensor, packed, act, logits, W: int | None = None, stream=None):
    """imgs: uint8 [B][H][pitch] (contiguous frames)."""
    B, H, pitch = imgs.shape
    W = pitch if W is None else W
    _check(_cnn_fwd(_p(imgs), W, H, pitch, H * pitch, B, _p(packed), _p(act), _p(logits),
                    _stream(stream)), "lane_cnn_forward")


def cnn_infer(imgs: torch.Tensor, packed, logits, W: int | None = None, stream=None):
    """Forward only (fused, no activation workspace); imgs uint8 [B][H][pitch]."""
    B, H, pitch = imgs.shape
    W = pitch if W is None else W
    _check(_cnn_infer(_p(imgs), W, H, pitch, H * pitch, B, _p(packed), _p(logits),
                      _stream(stream)), "lane_cnn_infer")


def cnn_loss(logits, keep, bands, W: int, H: int, batch: int, scale: float, act, loss,
             stream=None):
    _check(_cnn_loss(_p(logits), _p(keep), _p(bands), W, H, batch, float(scale), _p(act), _p(loss),
                     _stream(stream)), "lane_cnn_loss")


def cnn_backward(imgs: torch.Tensor, packed, act, partial, grads, W: int | None = None,
                 stream=None):
    B, H, pitch = imgs.shape
    W = pitch if W is None else W
    _check(_cnn_bwd(_p(imgs), W, H, pitch, H * pitch, B, _p(packed), _p(act), _p(partial),
                    partial.numel() * partial.element_size(), _p(grads), _stream(stream)),
           "lane_cnn_backward")


def adam_step(params, grads, m, v, lr: float, step: int, grad_scale: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, stream=None):
    _check(_adam(_p(params), _p(grads), _p(m), _p(v), params.numel(), float(lr), float(beta1),
                 float(beta2), float(eps), int(step), float(grad_scale), _stream(stream)),
           "lane_adam_step")


def tile_labels(fb: "FrameBuffers", keep, bands, stream=None):
    """Labels of one frame from its plain-pipeline results in a batch plan."""
    _check(_labels(_p(fb.edge_list), fb.W, fb.H, _p(fb.cos_q14), _p(fb.sin_q14), fb.n_theta, fb.D,
                   _p(fb.peaks), fb.k, _p(keep), _p(bands), _stream(stream)), "lane_tile_labels")


def mask_from_logits(logits, W: int, H: int, batch: int, conf: float, mask, stream=None):
    _check(_mask(_p(logits), W, H, batch, float(conf), _p(mask), _stream(stream)),
           "lane_mask_from_logits")


# ---------------------------------------------------------------- serving --

LANE_E_BUSY = -7
LANE_E_TIMEOUT = -8
SERVE_MAX_K = 64


class StreamCfg(ctypes.Structure):
    _fields_ = [("W", _i32), ("H", _i32), ("n_theta", _i32), ("k", _i32), ("threshold", _i32),
                ("border_mode", _i32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", _sz), ("pruned", _i32), ("conf", ctypes.c_float),
                ("cnn_params", _vp), ("max_pending", _i32), ("vote_rows", _i32),
                ("sobel_strip_rows", _i32), ("vote_split", _i32), ("deadline_ns", ctypes.c_int64),
                ("lanes", _i32), ("spin_us", _i32)]


class Result(ctypes.Structure):
    _fields_ = [("stream", _i32), ("status", _i32), ("frame_id", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("batch_frames", _i32), ("count", _i32),
                ("theta_idx", _i32 * SERVE_MAX_K), ("r_idx", _i32 * SERVE_MAX_K),
                ("votes", _i32 * SERVE_MAX_K)]


class Request(ctypes.Structure):
    _fields_ = [("stream", _i32), ("pitch", _i32), ("t_offset_ns", ctypes.c_int64),
                ("frame", _vp), ("frame_id", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("dropped", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("frames_in_batches", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("streams_admitted", _i32), ("error", _i32), ("timed_out", ctypes.c_int64)]


_srv_plan = _sig("lane_server_plan", [ctypes.POINTER(StreamCfg), _i32, ctypes.POINTER(ServerCfg),
                                      _vp, _vp, ctypes.POINTER(_sz)])
_srv_create = _sig("lane_server_create", [ctypes.POINTER(StreamCfg), _i32,
                                          ctypes.POINTER(ServerCfg), ctypes.POINTER(_vp), _vp])
_srv_submit = _sig("lane_server_submit", [_vp, _i32, _vp, _i32, ctypes.c_uint64])
_srv_poll = _sig("lane_server_poll", [_vp, ctypes.POINTER(Result), _i32, _i32,
                                      ctypes.POINTER(_i32)])
_srv_replay = _sig("lane_server_replay", [_vp, ctypes.POINTER(Request), _i32,
                                          ctypes.POINTER(Result)])
_srv_stats = _sig("lane_server_stats_get", [_vp, ctypes.POINTER(ServerStats)])
_srv_destroy = _sig("lane_server_destroy", [_vp])
_srv_pause = _sig("lane_server_pause", [_vp, _i32])


def _server_cfg(hbm_budget, pruned, conf, cnn_params, max_pending, vote_rows, sobel_strip_rows,
                vote_split=0, deadline_ms=0.0, lanes=0, spin_us=0):
    import numpy as np

    keep = None
    if cnn_params is not None:
        keep = np.ascontiguousarray(np.asarray(cnn_params, dtype=np.float32))
    cfg = ServerCfg(int(hbm_budget), int(pruned), float(conf),
                    None if keep is None else keep.ctypes.data, int(max_pending), int(vote_rows),
                    int(sobel_strip_rows), int(vote_split), int(round(deadline_ms * 1e6)), int(lanes),
                    int(spin_us))
    return cfg, keep


def _host_frame(frame):
    """A frame the server may read later: host uint8 [H][pitch] with rows of
    contiguous bytes."""
    import numpy as np

    if not isinstance(frame, np.ndarray) or frame.dtype != np.uint8 or frame.ndim != 2:
        raise TypeError("a frame is a host numpy uint8 array [H][pitch]")
    if frame.strides[1] != 1 or frame.strides[0] < frame.shape[1]:
        raise ValueError("frame rows must be contiguous bytes (strides[1] == 1, pitch >= W)")
    return frame


def _stream_cfgs(streams):
    arr = (StreamCfg * len(streams))()
    for i, st in enumerate(streams):
        d = dict(n_theta=360, k=8, threshold=128, border_mode=LANE_BORDER_ZERO_MASKRING)
        d.update(st)
        arr[i] = StreamCfg(d["W"], d["H"], d["n_theta"], d["k"], d["threshold"], d["border_mode"])
    return arr


def server_plan(streams, hbm_budget: int, pruned: bool = False, conf: float = 0.9,
                cnn_params=None, max_pending: int = 4, vote_rows: int = 0, sobel_strip_rows: int = 0,
                vote_split: int = 0, lanes: int = 0, spin_us: int = 0):
    """Host-only admission plan: (admitted list of bool, per-stream bytes, total bytes)."""
    import numpy as np

    arr = _stream_cfgs(streams)
    cfg, keep = _server_cfg(hbm_budget, pruned, conf, cnn_params, max_pending, vote_rows,
                            sobel_strip_rows, vote_split, lanes=lanes, spin_us=spin_us)
    adm = np.zeros(len(streams), np.uint8)
    sb = np.zeros(len(streams), np.uint64)
    tot = _sz(0)
    _check(_srv_plan(arr, len(streams), ctypes.byref(cfg), adm.ctypes.data, sb.ctypes.data,
                     ctypes.byref(tot)), "lane_server_plan")
    return [bool(a) for a in adm], [int(b) for b in sb], int(tot.value)


class Server:
    """Continuous-batching server over camera streams (lane_server_*).

    streams: list of dicts with W, H and optionally n_theta, k, threshold,
    border_mode; lanes: refills that may run at once (0: the library's 2);
    spin_us: how long an idle lane polls for work before it sleeps."""

    def __init__(self, streams, hbm_budget: int = 8 << 30, pruned: bool = False,
                 conf: float = 0.9, cnn_params=None, max_pending: int = 4, vote_rows: int = 0,
                 sobel_strip_rows: int = 0, vote_split: int = 0, deadline_ms: float = 0.0,
                 lanes: int = 0, spin_us: int = 0):
        import collections

        import numpy as np

        self.streams = [dict(s) for s in streams]
        arr = _stream_cfgs(streams)
        cfg, keep = _server_cfg(hbm_budget, pruned, conf, cnn_params, max_pending, vote_rows,
                                sobel_strip_rows, vote_split, deadline_ms, lanes, spin_us)
        adm = np.zeros(len(streams), np.uint8)
        h = _vp()
        _check(_srv_create(arr, len(streams), ctypes.byref(cfg), ctypes.byref(h), adm.ctypes.data),
               "lane_server_create")
        self._h = h
        self.admitted = [bool(a) for a in adm]
        # frames submitted and not yet polled, per stream in submission order:
        # a stream's requests complete in that order, so each polled result
        # releases the oldest held frame of its stream
        self._hold = collections.defaultdict(collections.deque)

    def submit(self, stream: int, frame, frame_id: int = 0) -> int:
        """frame: host numpy uint8 [H][pitch]; kept alive until its result is
        polled.  Returns LANE_OK or LANE_E_BUSY (dropped: its result is
        already complete and holds no frame)."""
        frame = _host_frame(frame)
        rc = _srv_submit(self._h, stream, frame.ctypes.data, frame.strides[0], frame_id)
        if rc == LANE_OK:
            self._hold[stream].append(frame)
        elif rc != LANE_E_BUSY:
            _check(rc, "lane_server_submit")
        return rc

    def poll(self, max_n: int = 64, wait_ms: int = 0):
        out = (Result * max_n)()
        n = _i32(0)
        _check(_srv_poll(self._h, out, max_n, wait_ms, ctypes.byref(n)), "lane_server_poll")
        res = [out[i] for i in range(n.value)]
        for r in res:
            if r.status != LANE_E_BUSY and self._hold[r.stream]:
                self._hold[r.stream].popleft()
        return res

    def pause(self, paused: bool = True):
        """Hold (True) or resume (False) the refill lanes; requests keep queueing."""
        _check(_srv_pause(self._h, 1 if paused else 0), "lane_server_pause")

    def replay(self, reqs):
        """reqs: list of (stream, t_offset_s, frame ndarray, frame_id); returns results in order."""
        arr = (Request * len(reqs))()
        for i, (st, t, fr, fid) in enumerate(reqs):
            fr = _host_frame(fr)
            arr[i] = Request(st, fr.strides[0], int(round(t * 1e9)), fr.ctypes.data, fid)
        out = (Result * len(reqs))()
        _check(_srv_replay(self._h, arr, len(reqs), out), "lane_server_replay")
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(_srv_stats(self._h, ctypes.byref(st)), "lane_server_stats_get")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _srv_destroy(self._h)
            self._h = None
            self._hold.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
