"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Holds no arithmetic of the method itself: only scene-like RGB views (smooth
gradient background, random filled polygons, optional band-limited texture,
Gaussian sensor noise) and random 3D Gaussian sets with a split mask. The
bytes come from ``libsynth.so`` (``synth.c``); this module only marshals
arrays and states the named workloads.

The workloads mirror the view sizes of the Mip-NeRF360 captures the paper
evaluates on (Sec. 3.1): about 1297x840 (4x downsample) and 2473x1643
(2x downsample), 150-300 views per scene. The dataset itself is not used;
these seeded images stand in for it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (OpenMP); returns its path."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             os.path.join(_HERE, "synth.c"), "-o", _LIB_PATH + ".tmp", "-lm"])
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, i32, i64, dbl, vp = (ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_void_p)
        L.syn_image.argtypes = [u64, i32, i32, i32, i32, dbl, dbl, vp]
        L.syn_image_down2.argtypes = [u64, i32, i32, i32, i32, dbl, dbl, vp]
        L.syn_image_batch.argtypes = [i32, vp, vp, vp, vp, i32, i32, dbl, dbl, vp, vp]
        L.syn_view_sizes.argtypes = [u64, i32, i32, i32, dbl, dbl, vp, vp]
        L.syn_gaussians.argtypes = [u64, i64, dbl, dbl, vp, vp, vp, vp]
        L.syn_mask.argtypes = [u64, i64, i64, vp]
        L.syn_contrib_count.argtypes = [u64, i64, i32, vp, vp, i32, vp]
        L.syn_contrib_count.restype = i64
        L.syn_contrib_fill.argtypes = [u64, i64, i32, vp, vp, i32, vp, i32, vp, vp, vp, vp]
        for f in ("syn_image", "syn_image_down2", "syn_image_batch", "syn_view_sizes",
                  "syn_gaussians", "syn_mask", "syn_contrib_fill"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def image(seed: int, W: int, H: int, n_poly: int = 12, texture: bool = False,
          noise_sigma: float = 5.0, tex_amp: float = 20.0, down2: bool = False) -> np.ndarray:
    """One uint8 RGB view, shape (H, W, 3) (or (H//2, W//2, 3) with down2)."""
    h, w = (H // 2, W // 2) if down2 else (H, W)
    out = np.empty((h, w, 3), np.uint8)
    f = lib().syn_image_down2 if down2 else lib().syn_image
    f(seed, W, H, n_poly, int(texture), tex_amp, noise_sigma, _p(out))
    return out


@dataclass
class ViewBatch:
    """Views packed into one byte buffer with per-view offsets.

    ``rgb`` holds every view back to back (each starting at ``in_offset``,
    rows packed with pitch 3*W); ``out_offset`` is where each view's float32
    map starts in an output buffer of ``out_floats`` elements (pitch W).
    """
    widths: np.ndarray
    heights: np.ndarray
    in_offset: np.ndarray
    out_offset: np.ndarray
    rgb: np.ndarray
    out_floats: int

    @property
    def n(self) -> int:
        return int(self.widths.shape[0])

    @property
    def pixels(self) -> int:
        return int((self.widths.astype(np.int64) * self.heights).sum())

    def view(self, v: int) -> np.ndarray:
        W, H, o = int(self.widths[v]), int(self.heights[v]), int(self.in_offset[v])
        return self.rgb[o:o + 3 * W * H].reshape(H, W, 3)


def pack_views(imgs: list[np.ndarray], in_align: int = 1, out_align: int = 1) -> ViewBatch:
    """Pack explicit (H, W, 3) uint8 images into a ViewBatch."""
    n = len(imgs)
    W = np.array([im.shape[1] for im in imgs], np.int32)
    H = np.array([im.shape[0] for im in imgs], np.int32)
    ino, outo = _offsets(W, H, in_align, out_align)
    total = int(ino[-1] + 3 * int(W[-1]) * int(H[-1])) if n else 0
    rgb = np.zeros(max(total, 1), np.uint8)
    for v, im in enumerate(imgs):
        rgb[int(ino[v]):int(ino[v]) + im.size] = np.ascontiguousarray(im).reshape(-1)
    outf = int(outo[-1] + int(W[-1]) * int(H[-1])) if n else 0
    return ViewBatch(W, H, ino, outo, rgb, outf)


def _offsets(W, H, in_align, out_align):
    n = W.shape[0]
    ino = np.zeros(n, np.int64)
    outo = np.zeros(n, np.int64)
    a = b = 0
    for v in range(n):
        a = -(-a // in_align) * in_align
        b = -(-b // out_align) * out_align
        ino[v], outo[v] = a, b
        a += 3 * int(W[v]) * int(H[v])
        b += int(W[v]) * int(H[v])
    return ino, outo


def batch(seeds, full_w, full_h, down2=None, n_poly: int = 60, texture: bool = True,
          noise_sigma: float = 5.0, tex_amp: float = 20.0, in_align: int = 256,
          out_align: int = 64) -> ViewBatch:
    """Render many views in parallel into one packed buffer."""
    seeds = np.ascontiguousarray(seeds, np.uint64)
    fw = np.ascontiguousarray(full_w, np.int32)
    fh = np.ascontiguousarray(full_h, np.int32)
    n = seeds.shape[0]
    d2 = np.zeros(n, np.int32) if down2 is None else np.ascontiguousarray(down2, np.int32)
    W = np.where(d2 != 0, fw // 2, fw).astype(np.int32)
    H = np.where(d2 != 0, fh // 2, fh).astype(np.int32)
    ino, outo = _offsets(W, H, in_align, out_align)
    total = int(ino[-1] + 3 * int(W[-1]) * int(H[-1]))
    rgb = np.empty(total, np.uint8)
    lib().syn_image_batch(n, _p(seeds), _p(fw), _p(fh), _p(d2), n_poly, int(texture), tex_amp,
                          noise_sigma, _p(ino), _p(rgb))
    outf = int(outo[-1] + int(W[-1]) * int(H[-1]))
    return ViewBatch(W, H, ino, outo, rgb, outf)


def view_sizes(seed: int, n: int, wlo: int, whi: int, alo: float, ahi: float):
    W = np.empty(n, np.int32)
    H = np.empty(n, np.int32)
    lib().syn_view_sizes(seed, n, wlo, whi, alo, ahi, _p(W), _p(H))
    return W, H


@dataclass
class GaussianSet:
    """Structure-of-arrays float32 Gaussian parameters for N rows."""
    means: np.ndarray        # (N, 3)
    log_scales: np.ndarray   # (N, 3)
    quats: np.ndarray        # (N, 4), (w, x, y, z)
    opacity_logits: np.ndarray  # (N,)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


def gaussians(seed: int, N: int, ls_mu: float = -4.0, ls_sd: float = 0.5) -> GaussianSet:
    m = np.empty((N, 3), np.float32)
    s = np.empty((N, 3), np.float32)
    q = np.empty((N, 4), np.float32)
    o = np.empty((N,), np.float32)
    lib().syn_gaussians(seed, N, ls_mu, ls_sd, _p(m), _p(s), _p(q), _p(o))
    return GaussianSet(m, s, q, o)


def mask(seed: int, N: int, K: int) -> np.ndarray:
    out = np.empty(N, np.uint8)
    lib().syn_mask(seed, N, K, _p(out))
    return out


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

ASPECT_LO, ASPECT_HI = 1.5, 16.0 / 9.0


@dataclass
class Contributions:
    """Pixel contributions (Gaussian, view, pixel = y * width + x, weight)."""
    gauss: np.ndarray
    view: np.ndarray
    pixel: np.ndarray
    weight: np.ndarray

    @property
    def n(self) -> int:
        return int(self.gauss.shape[0])


def contributions(seed: int, n_gauss: int, widths, heights, mean_radius: int = 3, order: str = "rows") -> Contributions:
    """Synthetic contributions of n_gauss Gaussians over views of the given
    sizes (each Gaussian a clipped disc in one view; see synth.c). order
    "rows": grouped by view and image row, as a rasteriser meets them;
    "spread": neighbouring entries belong to different Gaussians."""
    W = np.ascontiguousarray(widths, np.int32)
    H = np.ascontiguousarray(heights, np.int32)
    off = np.zeros(n_gauss + 1, np.int64)
    n = lib().syn_contrib_count(seed, n_gauss, int(W.size), _p(W), _p(H), int(mean_radius), _p(off))
    c = Contributions(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.float32))
    lib().syn_contrib_fill(seed, n_gauss, int(W.size), _p(W), _p(H), int(mean_radius), _p(off),
                           {"spread": 0, "rows": 1}[order], _p(c.gauss), _p(c.view), _p(c.pixel), _p(c.weight))
    return c


def grad_accum(seed: int, n: int) -> np.ndarray:
    """Synthetic accumulated view-space gradient norms (log-normal, float32)."""
    return np.random.default_rng(seed).lognormal(-9.0, 1.0, n).astype(np.float32)


@dataclass
class Workload:
    """One of the named workloads: views to render plus a Gaussian set."""
    stream: int               # seed stream of the workload's inputs
    name: str
    seeds: np.ndarray
    full_w: np.ndarray
    full_h: np.ndarray
    down2: np.ndarray
    n_poly: int
    texture: bool
    precision: str            # intermediate storage of the batched/plain form
    batched: bool
    n_gauss: int
    ls_mu: float
    ls_sd: float
    split_frac: float
    graph: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def n_views(self) -> int:
        return int(self.seeds.shape[0])

    def sizes(self):
        W = np.where(self.down2 != 0, self.full_w // 2, self.full_w)
        H = np.where(self.down2 != 0, self.full_h // 2, self.full_h)
        return W.astype(np.int64), H.astype(np.int64)

    @property
    def pixels(self) -> int:
        W, H = self.sizes()
        return int((W * H).sum())

    @property
    def n_split(self) -> int:
        return int(round(self.split_frac * self.n_gauss))

    def render(self, views=None, **kw) -> ViewBatch:
        sel = np.arange(self.n_views) if views is None else np.asarray(views)
        return batch(self.seeds[sel], self.full_w[sel], self.full_h[sel], self.down2[sel],
                     n_poly=self.n_poly, texture=self.texture, **kw)

    def gaussian_set(self) -> GaussianSet:
        return gaussians(7000001 * self.stream, self.n_gauss, self.ls_mu, self.ls_sd)

    def split_mask(self) -> np.ndarray:
        return mask(7000001 * self.stream + 1, self.n_gauss, self.n_split)


# The workloads by name; the value is each one's seed stream.
WORKLOADS = {
    "view_256x192": 1,
    "view_1297x840": 2,
    "views200_w1000_1560": 3,
    "views150_2473x1643_mixed": 4,
    "step_views300_las3m": 5,
}


def workload(key: str) -> Workload:
    """The named workload `key` (one of WORKLOADS)."""
    if key not in WORKLOADS:
        raise ValueError(f"unknown workload {key!r}; one of {sorted(WORKLOADS)}")
    c = WORKLOADS[key]

    def seeds(n):
        return np.array([1000003 * c + v for v in range(n)], np.uint64)

    if c == 1:
        return Workload(1, "single 256x192 view, 12 polygons; LAS 10k Gaussians, 10% split",
                        seeds(1), np.array([256]), np.array([192]), np.zeros(1, np.int32),
                        12, False, "fp32", False, 10_000, -4.0, 0.5, 0.10)
    if c == 2:
        return Workload(2, "single 1297x840 view, 60 textured polygons; LAS 1M Gaussians, 5% split",
                        seeds(1), np.array([1297]), np.array([840]), np.zeros(1, np.int32),
                        60, True, "fp32", False, 1_000_000, -4.0, 0.5, 0.05)
    if c == 3:
        W, H = view_sizes(1000003 * c, 200, 1000, 1560, ASPECT_LO, ASPECT_HI)
        return Workload(3, "200 views, W in [1000,1560], aspect 3:2-16:9, batched fp16",
                        seeds(200), W, H, np.zeros(200, np.int32), 60, True, "fp16", True,
                        0, -4.0, 0.5, 0.0)
    if c == 4:
        W = np.full(150, 2473, np.int32)
        H = np.full(150, 1643, np.int32)
        d2 = (np.arange(150) % 2).astype(np.int32)
        return Workload(4, "150 views, 2473x1643 and 2x downsamples 50/50, batched fp16/bf16",
                        seeds(150), W, H, d2, 60, True, "fp16", True, 0, -4.0, 0.5, 0.0,
                        extra={"precisions": ["fp16", "bf16"]})
    if c == 5:
        W, H = view_sizes(1000003 * c, 300, 1000, 2473, ASPECT_LO, ASPECT_HI)
        return Workload(5, "densification step: 300 views W in [1000,2473] bf16 + LAS 3M Gaussians, 20% split",
                        seeds(300), W, H, np.zeros(300, np.int32), 60, True, "bf16", True,
                        3_000_000, -4.5, 0.7, 0.20, graph=True)
    raise AssertionError(c)
