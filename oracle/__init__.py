"""CPU oracle for the ImprovedGS+ densification hot path (arXiv 2603.08661).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py``; never by the product path. It shares no
code with the GPU library. The arithmetic lives in ``igsp_oracle.c`` (plain
C, int64-exact through the gradient and orientation bins, FP64 after);
this module only marshals numpy arrays.

Edge map: Sec. 2.1 (grayscale, 5x5 Gaussian blur, Sobel magnitude and
orientation, non-maximum suppression, median normalisation).
Long-Axis-Split: Sec. 2.2, Algorithms 1 and 2, constants alpha = 0.5,
gamma = 0.85, beta = 0.6.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# The split constants printed in Sec. 2.2 (paragraph after Algorithm 1).
ALPHA, GAMMA, BETA = 0.5, 0.85, 0.6


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP across views)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             os.path.join(_HERE, "igsp_oracle.c"), "-o", _LIB_PATH + ".tmp", "-lm"])
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_blur_taps.argtypes = [vp]
        L.orc_blur_taps.restype = None
        L.orc_bin.argtypes = [i64, i64]
        L.orc_bin.restype = i32
        L.orc_nms.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
        L.orc_nms.restype = None
        L.orc_edge_view.argtypes = [vp, i32, i32] + [vp] * 12
        L.orc_edge_view.restype = i64
        L.orc_edge_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        L.orc_edge_batch.restype = None
        L.orc_quat_to_R.argtypes = [vp, vp]
        L.orc_quat_to_R.restype = None
        L.orc_opacity.argtypes = [dbl, dbl]
        L.orc_opacity.restype = dbl
        L.orc_las.argtypes = [i64, i64, vp, vp, vp, vp, vp, i32, vp, dbl, dbl, dbl,
                              vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_las.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def blur_taps() -> np.ndarray:
    out = np.zeros(5, np.int64)
    lib().orc_blur_taps(_p(out))
    return out


def bin_of(gx: int, gy: int) -> int:
    """Orientation bin: 0 horizontal, 1 vertical, 2 diagonal gx*gy>0, 3 otherwise."""
    return int(lib().orc_bin(int(gx), int(gy)))


def nms(gx: np.ndarray, gy: np.ndarray) -> dict:
    """Suppression step alone (Sec. 2.1 step 3) on a given integer gradient
    field (H, W): squared magnitude M, orientation bin, keep, and the
    decision margin c(p)."""
    gx = np.ascontiguousarray(gx, np.int64)
    gy = np.ascontiguousarray(gy, np.int64)
    if gx.shape != gy.shape or gx.ndim != 2:
        raise ValueError("gx and gy must be 2-D arrays of one shape")
    H, W = gx.shape
    if W < 3 or H < 3:
        raise ValueError("fields must be at least 3x3")
    o = {"M": np.zeros((H, W), np.int64), "bin": np.zeros((H, W), np.uint8),
         "keep": np.zeros((H, W), np.uint8), "margin": np.zeros((H, W), np.float64)}
    lib().orc_nms(_p(gx), _p(gy), W, H, _p(o["M"]), _p(o["bin"]), _p(o["keep"]), _p(o["margin"]))
    return o


def edge_view(rgb: np.ndarray) -> dict:
    """Every stage of the edge pipeline for one (H, W, 3) uint8 view."""
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W = rgb.shape[:2]
    o = {k: np.zeros((H, W), np.int64) for k in ("gray", "b", "gx", "gy", "M")}
    o["bin"] = np.zeros((H, W), np.uint8)
    o["keep"] = np.zeros((H, W), np.uint8)
    for k in ("m", "E", "margin"):
        o[k] = np.zeros((H, W), np.float64)
    med = np.zeros(1, np.float64)
    Mmed = np.zeros(1, np.int64)
    n = lib().orc_edge_view(_p(rgb), W, H, _p(o["gray"]), _p(o["b"]), _p(o["gx"]), _p(o["gy"]),
                            _p(o["M"]), _p(o["bin"]), _p(o["keep"]), _p(o["m"]), _p(o["E"]),
                            _p(o["margin"]), _p(med), _p(Mmed))
    if n < 0:
        raise ValueError("views must be at least 3x3")
    o["n"], o["med"], o["Mmed"] = int(n), float(med[0]), int(Mmed[0])
    return o


def edge_batch(rgb: np.ndarray, widths, heights, in_offset, out_offset, out_floats: int,
               threads: int = 0, want_keep: bool = False) -> dict:
    """Normalised maps (FP64) for packed views; layout as in the GPU call."""
    W = np.ascontiguousarray(widths, np.int32)
    H = np.ascontiguousarray(heights, np.int32)
    if (W < 3).any() or (H < 3).any():
        raise ValueError("views must be at least 3x3")
    io = np.ascontiguousarray(in_offset, np.int64)
    oo = np.ascontiguousarray(out_offset, np.int64)
    n = W.shape[0]
    E = np.zeros(out_floats, np.float64)
    keep = np.zeros(out_floats, np.uint8) if want_keep else None
    med = np.zeros(n, np.float64)
    ns = np.zeros(n, np.int64)
    lib().orc_edge_batch(_p(np.ascontiguousarray(rgb, np.uint8)), n, _p(W), _p(H), _p(io), _p(oo),
                         _p(E), _p(keep), _p(med), _p(ns), int(threads))
    out = {"E": E, "med": med, "n": ns}
    if want_keep:
        out["keep"] = keep
    return out


def quat_to_R(q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9, np.float64)
    lib().orc_quat_to_R(_p(q), _p(R))
    return R.reshape(3, 3)


def opacity_update(o: float, beta: float = BETA) -> float:
    return float(lib().orc_opacity(float(o), float(beta)))


def split_scores(maps, widths, heights, out_offset, gauss, view, pixel, weight, N: int) -> np.ndarray:
    """Edge scores of Gaussians [0, N) (int64, units of 2^-32).

    The paper moves its edge maps onto the Gaussians without a formula; the
    reading taken: a Gaussian's score is the sum over its pixel contributions
    of E_view[pixel] * weight, each product rounded to float32, then floor of
    the product times 2^32 (exact), summed exactly as integers. Entries naming
    a Gaussian >= N, an unknown view or a pixel outside its view add nothing,
    nor do non-positive products.
    """
    maps = np.asarray(maps, np.float32)
    W = np.asarray(widths, np.int64)
    H = np.asarray(heights, np.int64)
    off = np.asarray(out_offset, np.int64)
    g = np.asarray(gauss, np.int64)
    v = np.asarray(view, np.int64)
    p = np.asarray(pixel, np.int64)
    w = np.asarray(weight, np.float32)
    ok = (g >= 0) & (g < N) & (v >= 0) & (v < W.size)
    vv = np.where(ok, v, 0)
    ok &= (p >= 0) & (p < W[vv] * H[vv])
    e = np.zeros(g.size, np.float32)
    e[ok] = maps[off[vv[ok]] + p[ok]] * w[ok]              # float32 products
    ok &= e > 0
    q = np.floor(e[ok].astype(np.float64) * 2.0 ** 32).astype(np.int64)
    gs = g[ok]
    scores = np.zeros(N, np.int64)
    if gs.size:
        order = np.argsort(gs, kind="stable")
        gs, q = gs[order], q[order]
        starts = np.flatnonzero(np.r_[True, gs[1:] != gs[:-1]])
        scores[gs[starts]] = np.add.reduceat(q, starts)      # exact int64 sums
    return scores


def split_select(scores, grad, N: int, grad_threshold: float, warmup: bool, budget: int):
    """Split mask over [0, N): candidates are Gaussians with grad >= threshold
    (float32 compare), or all of them during warm-up; the K = min(candidates,
    max(0, budget - N)) candidates of largest score are selected, ties by
    lower index. Returns (mask uint8 [N], K)."""
    grad = np.asarray(grad, np.float32)[:N]
    cand = np.ones(N, bool) if warmup else grad >= np.float32(grad_threshold)
    K = int(min(int(cand.sum()), max(0, int(budget) - N)))
    idx = np.flatnonzero(cand)
    sc = np.asarray(scores, np.int64)[idx]
    order = np.lexsort((idx, -sc))                           # score descending, index ascending
    mask = np.zeros(N, np.uint8)
    mask[idx[order[:K]]] = 1
    return mask, K


def las_moments(N: int, split_idx, moments: dict) -> dict:
    """Optimiser state after the full-record split (FP64 copies).

    The paper does not say what happens to optimiser state; the reading taken
    (and stated with the GPU entry point) is the usual one for a split that
    replaces a parent by two new Gaussians: the moment rows of both children
    -- row i of every split Gaussian and rows N .. N + K - 1 -- become 0,
    every other row keeps its value.
    """
    idx = np.asarray(split_idx, np.int64)
    out = {}
    for k, a in moments.items():
        b = np.array(a, dtype=np.float64, copy=True)
        b[idx] = 0.0
        b[N:N + idx.size] = 0.0
        out[k] = b
    return out


def las(N: int, means, log_scales, quats, opacity_logits, mask, feats=None,
        alpha: float = ALPHA, gamma: float = GAMMA, beta: float = BETA) -> dict:
    """Long-Axis-Split in place over arrays of `capacity` rows (FP64 results).

    means (cap,3), log_scales (cap,3), quats (cap,4), opacity_logits (cap,),
    feats (cap,F) or None, all float32; mask (>= N,) uint8.
    """
    means = np.ascontiguousarray(means, np.float32)
    ls = np.ascontiguousarray(log_scales, np.float32)
    q = np.ascontiguousarray(quats, np.float32)
    op = np.ascontiguousarray(opacity_logits, np.float32)
    cap = means.shape[0]
    F = 0 if feats is None else int(feats.shape[1])
    f = np.zeros((cap, max(F, 1)), np.float32) if feats is None else np.ascontiguousarray(feats, np.float32)
    mk = np.zeros(cap, np.uint8)
    mk[:min(cap, mask.shape[0])] = np.asarray(mask, np.uint8)[:cap]
    out = {
        "means": np.zeros((cap, 3)), "log_scales": np.zeros((cap, 3)), "quats": np.zeros((cap, 4)),
        "opacity_logits": np.zeros(cap), "feats": np.zeros((cap, max(F, 1))),
        "split_idx": np.zeros(cap, np.int32), "axis": np.zeros(cap, np.int32),
    }
    K = np.zeros(1, np.int64)
    cnt = np.zeros(1, np.int64)
    st = lib().orc_las(int(N), cap, _p(means), _p(ls), _p(q), _p(op), _p(f), F, _p(mk),
                       alpha, gamma, beta, _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
                       _p(out["opacity_logits"]), _p(out["feats"]), _p(out["split_idx"]),
                       _p(out["axis"]), _p(K), _p(cnt))
    out["status"], out["K"], out["count"] = int(st), int(K[0]), int(cnt[0])
    out["split_idx"] = out["split_idx"][:out["K"]] if st == 0 else out["split_idx"][:0]
    out["axis"] = out["axis"][:out["K"]] if st == 0 else out["axis"][:0]
    if F == 0:
        out["feats"] = out["feats"][:, :0]
    return out


def lr_exponential(t: int, lr_init: float, lr_final: float, t_max: int) -> float:
    """Exponential learning-rate schedule (Sec. 3): log-linear interpolation
    from lr_init at t = 0 to lr_final at t = t_max, constant outside."""
    if not (lr_init > 0 and lr_final > 0 and t_max >= 1):
        return math.nan
    s = min(max(t, 0), t_max) / t_max
    return lr_init * (lr_final / lr_init) ** s
