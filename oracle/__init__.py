"""CPU oracle for the lane-detection hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library never imports, links
or calls it; the oracle imports nothing from the product.

``lane_oracle.c`` holds the integer path (Sobel + binarize, Q14 vote, greedy
NMS peaks, line segments along the peaks, the Canny detector and the
coarse-to-fine Hough transform) as plain nested loops; ``cnn.py``
the FP64 proposal network and its analytic backward, tile labels, masks and
peak agreement.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblane_oracle.so")
# the same source built with OpenMP: Sobel rows and vote rows split over the
# host's cores (the multi-core CPU baseline; results identical)
OMP_LIB_PATH = os.path.join(_HERE, "liblane_oracle_omp.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile lane_oracle.c with gcc (plain -O2, no vector intrinsics), once
    single-threaded and once with OpenMP."""
    src = os.path.join(_HERE, "lane_oracle.c")
    for path, extra in ((LIB_PATH, []), (OMP_LIB_PATH, ["-fopenmp"])):
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra, src, "-o", tmp]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        # LANE_ORACLE_LIB: another build of the same source (the sanitizer test)
        path = os.environ.get("LANE_ORACLE_LIB")
        if not path:
            path = LIB_PATH
            if not os.path.exists(path):
                build()
        lib = ctypes.CDLL(path)
        vp, i32 = ctypes.c_void_p, ctypes.c_int
        lib.oracle_sobel_binarize.restype = ctypes.c_int64
        lib.oracle_sobel_binarize.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
        lib.oracle_hough_vote.restype = ctypes.c_int64
        lib.oracle_hough_vote.argtypes = [vp, i32, i32, i32, vp, vp, i32, i32, i32, vp, vp,
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_hough_peaks.restype = i32
        lib.oracle_hough_peaks.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp]
        lib.oracle_band_bits.restype = i32
        lib.oracle_band_bits.argtypes = [i32, i32]
        lib.oracle_hough_lines.restype = i32
        lib.oracle_hough_lines.argtypes = [vp, i32, i32, i32, vp, vp, i32, i32, vp, vp, i32, i32,
                                           i32, i32, vp, vp, vp]
        lib.oracle_canny.restype = ctypes.c_int64
        lib.oracle_canny.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp]
        lib.oracle_hough_progressive.restype = i32
        lib.oracle_hough_progressive.argtypes = [vp, i32, i32, i32, vp, vp, i32, i32, vp] + [vp] * 9
        lib.oracle_r_offset.restype = i32
        lib.oracle_r_offset.argtypes = [i32, i32]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def sobel_binarize(img: np.ndarray, W: int | None = None, threshold: int = 128,
                   border_mode: int = 1):
    """Return (edges[H][W] uint8 0/255, mag[H][W] uint8, n_edges).

    ``img`` is uint8 [H][pitch]; ``W`` defaults to the pitch."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, pitch = img.shape
    W = pitch if W is None else W
    edges = np.zeros((H, W), np.uint8)
    mag = np.zeros((H, W), np.uint8)
    n = _load().oracle_sobel_binarize(_ptr(img), W, H, pitch, int(threshold), int(border_mode),
                                      _ptr(edges), _ptr(mag))
    return edges, mag, int(n)


def canny(img: np.ndarray, W: int | None = None, t_low: int = 64, t_high: int = 128,
          border_mode: int = 1):
    """Canny edges (see oracle_canny).  Returns (edges[H][W] 0/255,
    mag[H][W] = min(|gx|+|gy|, 255) of the blurred image, n_edges)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, pitch = img.shape
    W = pitch if W is None else W
    edges = np.zeros((H, W), np.uint8)
    mag = np.zeros((H, W), np.uint8)
    n = _load().oracle_canny(_ptr(img), W, H, pitch, int(t_low), int(t_high), int(border_mode),
                             _ptr(edges), _ptr(mag))
    if n < 0:
        raise ValueError("bad Canny arguments")
    return edges, mag, int(n)


def hough_vote(edges: np.ndarray, cos_q14: np.ndarray, sin_q14: np.ndarray, r_offset: int,
               n_r: int, tile_mask: np.ndarray | None = None, W: int | None = None):
    """Return (acc[n_theta][n_r] int32, votes cast, dropped)."""
    edges = np.ascontiguousarray(edges, dtype=np.uint8)
    H, epitch = edges.shape
    W = epitch if W is None else W
    C = np.ascontiguousarray(cos_q14, dtype=np.int16)
    S = np.ascontiguousarray(sin_q14, dtype=np.int16)
    n_theta = C.shape[0]
    acc = np.zeros((n_theta, n_r), np.int32)
    if tile_mask is not None:
        tile_mask = np.ascontiguousarray(tile_mask, dtype=np.uint8)
        assert tile_mask.shape == ((H + 7) // 8, (W + 7) // 8)
    dropped = ctypes.c_int64(0)
    cast = _load().oracle_hough_vote(_ptr(edges), W, H, epitch, _ptr(C), _ptr(S), n_theta,
                                     int(r_offset), int(n_r), _ptr(tile_mask), _ptr(acc),
                                     ctypes.byref(dropped))
    return acc, int(cast), int(dropped.value)


def default_nms(n_theta: int, n_r: int) -> tuple[int, int]:
    """Default half-window: max(1, ceil(n/100)) on each axis."""
    return max(1, -(-n_theta // 100)), max(1, -(-n_r // 100))


def hough_peaks(acc: np.ndarray, r_offset: int, k: int, h_theta: int | None = None,
                h_r: int | None = None, min_votes: int = 1):
    """Return (theta_idx[k], r_idx[k], votes[k]) int32, -1 padded, and count."""
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    n_theta, n_r = acc.shape
    dt, dr = default_nms(n_theta, n_r)
    h_theta = dt if h_theta is None else h_theta
    h_r = dr if h_r is None else h_r
    t = np.zeros(k, np.int32)
    r = np.zeros(k, np.int32)
    v = np.zeros(k, np.int32)
    n = _load().oracle_hough_peaks(_ptr(acc), n_theta, n_r, int(r_offset), int(k), int(h_theta),
                                   int(h_r), int(min_votes), _ptr(t), _ptr(r), _ptr(v))
    if n < 0:
        raise ValueError("bad peak arguments")
    return t, r, v, n


def hough_lines(edges: np.ndarray, cos_q14, sin_q14, r_offset: int, theta_idx, r_idx,
                fill_gap: int = 20, min_length: int = 40, max_seg: int = 16, W: int | None = None):
    """Line segments along peaks (see oracle_hough_lines).  Returns
    (segs[k][max_seg][4] int32 -1 padded, counts[k], npts[k])."""
    edges = np.ascontiguousarray(edges, dtype=np.uint8)
    H, epitch = edges.shape
    W = epitch if W is None else W
    C = np.ascontiguousarray(cos_q14, dtype=np.int16)
    S = np.ascontiguousarray(sin_q14, dtype=np.int16)
    t = np.ascontiguousarray(theta_idx, dtype=np.int32)
    r = np.ascontiguousarray(r_idx, dtype=np.int32)
    k = t.shape[0]
    segs = np.zeros((k, max_seg, 4), np.int32)
    counts = np.zeros(k, np.int32)
    npts = np.zeros(k, np.int32)
    st = _load().oracle_hough_lines(_ptr(edges), W, H, epitch, _ptr(C), _ptr(S), C.shape[0],
                                    int(r_offset), _ptr(t), _ptr(r), k, int(fill_gap),
                                    int(min_length), int(max_seg), _ptr(segs), _ptr(counts),
                                    _ptr(npts))
    if st != 0:
        raise ValueError("bad line arguments")
    return segs, counts, npts


PROGRESSIVE_FIELDS = ("theta_step", "r_width", "k_coarse", "h_theta_coarse", "h_r_coarse",
                      "min_votes_coarse", "margin_theta", "margin_r", "k", "h_theta", "h_r",
                      "min_votes")


def hough_progressive(edges: np.ndarray, cos_q14, sin_q14, r_offset: int, W: int | None = None,
                      **params):
    """Coarse-to-fine Hough (see oracle_hough_progressive).  ``params`` holds
    every name of PROGRESSIVE_FIELDS.  Returns a dict with the geometry
    (n_c, n_rc, Dc, R, Wc), the coarse accumulator, the coarse peaks, the
    windows, the candidates and the final peaks (theta_idx, r_idx, votes,
    count)."""
    edges = np.ascontiguousarray(edges, dtype=np.uint8)
    H, epitch = edges.shape
    W = epitch if W is None else W
    C = np.ascontiguousarray(cos_q14, dtype=np.int16)
    S = np.ascontiguousarray(sin_q14, dtype=np.int16)
    n_theta = C.shape[0]
    missing = [f for f in PROGRESSIVE_FIELDS if f not in params]
    if missing or len(params) != len(PROGRESSIVE_FIELDS):
        raise ValueError(f"progressive parameters: missing {missing}, got {sorted(params)}")
    p = np.array([int(params[f]) for f in PROGRESSIVE_FIELDS], np.int32)
    f, w, kc, m_t, m_r, k = (int(p[0]), int(p[1]), int(p[2]), int(p[6]), int(p[7]), int(p[8]))
    if f < 1 or n_theta % f or w < 1 or w % 2 == 0 or kc < 1 or not 1 <= k <= kc:
        raise ValueError("bad progressive arguments")
    q = (w - 1) // 2
    D = int(r_offset)
    n_c, Dc = n_theta // f, (D + q) // w
    n_rc, R, Wc = 2 * Dc + 1, f + 2 * m_t, w + 2 * m_r
    coarse = np.zeros((n_c, n_rc), np.int32)
    ct, cr, cv = (np.zeros(kc, np.int32) for _ in range(3))
    win = np.zeros((kc, R, Wc), np.int32)
    cand = np.zeros((kc, 3), np.int32)
    t, r, v = (np.zeros(k, np.int32) for _ in range(3))
    n = _load().oracle_hough_progressive(_ptr(edges), W, H, epitch, _ptr(C), _ptr(S), n_theta, D,
                                         _ptr(p), _ptr(coarse), _ptr(ct), _ptr(cr), _ptr(cv),
                                         _ptr(win), _ptr(cand), _ptr(t), _ptr(r), _ptr(v))
    if n < 0:
        raise ValueError("bad progressive arguments")
    n_coarse = int((ct >= 0).sum())
    return dict(n_c=n_c, n_rc=n_rc, Dc=Dc, R=R, Wc=Wc, coarse_acc=coarse, coarse_theta=ct,
                coarse_r=cr, coarse_votes=cv, coarse_count=n_coarse, windows=win, cand=cand,
                theta_idx=t, r_idx=r, votes=v, count=n)


def band_bits(n_theta: int) -> np.ndarray:
    lib = _load()
    return np.array([lib.oracle_band_bits(n_theta, k) for k in range(n_theta)], np.uint8)


def r_offset(W: int, H: int) -> int:
    return int(_load().oracle_r_offset(W, H))


def pipeline(img: np.ndarray, cos_q14, sin_q14, k: int, threshold: int = 128,
             border_mode: int = 1, tile_mask=None):
    """Sobel -> binarize -> vote -> peaks on one frame; returns a dict."""
    H, W = img.shape
    D = r_offset(W, H)
    n_r = 2 * D + 1
    edges, mag, n_e = sobel_binarize(img, W, threshold, border_mode)
    acc, cast, dropped = hough_vote(edges, cos_q14, sin_q14, D, n_r, tile_mask)
    t, r, v, n = hough_peaks(acc, D, k)
    return dict(edges=edges, mag=mag, n_edges=n_e, acc=acc, cast=cast, dropped=dropped,
                theta_idx=t, r_idx=r, votes=v, count=n, D=D, n_r=n_r)
