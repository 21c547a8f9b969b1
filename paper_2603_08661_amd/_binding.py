"""ctypes binding of libigsp.so (the C ABI declared in include/igsp.h).

Argument marshalling only: tensors become device pointers, the view table a
C array, the current torch stream a hipStream_t. Every step of the path runs
in the library's HIP kernels; there is no fallback of any kind, so a missing
library or a non-gfx950 device raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigsp.so")

FP32, FP16, BF16 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "fp16": FP16, "bf16": BF16}

STATUS = {
    0: "IGSP_OK", -1: "IGSP_ERR_NULL", -2: "IGSP_ERR_DIMS", -3: "IGSP_ERR_ALIGN",
    -4: "IGSP_ERR_OVERLAP", -5: "IGSP_ERR_PARAM", -6: "IGSP_ERR_CAPACITY",
    -7: "IGSP_ERR_HIP", -8: "IGSP_ERR_UNSUPPORTED", -9: "IGSP_ERR_TIMEOUT", -10: "IGSP_ERR_TOO_LARGE",
}

# Every symbol include/igsp.h declares.
EXPORTS = ("edge_importance", "long_axis_split", "long_axis_split_noalloc", "long_axis_split_full", "split_mask",
           "igsp_edge_autotune",
           "igsp_edge_resolve", "igsp_step_create",
           "igsp_step_launch", "igsp_step_destroy", "igsp_status_string", "igsp_release_plans", "igsp_version",
           "igsp_lr_exponential")

# Tile shapes and launch forms the autotuner picked on MI355X for the
# benchmark geometries; the library reads this table unless the caller's
# environment names another.
TUNED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "gfx950.jsonl")


class IgspError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({status_string(code)})")


class View(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("in_offset", ctypes.c_int64), ("out_offset", ctypes.c_int64)]


class EdgeOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("seg_rows", ctypes.c_int32), ("wg_waves", ctypes.c_int32),
                ("medians", ctypes.c_void_p), ("survivors", ctypes.c_void_p),
                ("stage_events", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class Gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("features", ctypes.c_void_p), ("feat_dim", ctypes.c_int32),
                ("count", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class LasParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("gamma", ctypes.c_float), ("beta", ctypes.c_float)]


class Contributions(ctypes.Structure):
    _fields_ = [("gauss", ctypes.c_void_p), ("view", ctypes.c_void_p), ("pixel", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("n", ctypes.c_int64)]


class SelectParams(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("warmup", ctypes.c_int32), ("budget", ctypes.c_int64)]


class AdamMoments(ctypes.Structure):
    _fields_ = [(g, ctypes.c_void_p * 2) for g in ("means", "log_scales", "quats", "opacity_logits", "features")]


class LasOut(ctypes.Structure):
    _fields_ = [("split_idx", ctypes.c_void_p), ("status", ctypes.c_void_p), ("n_split", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libigsp.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname; load it first so
        # that this library binds to the runtime torch's tensors and streams use.
        import torch  # noqa: F401

        os.environ.setdefault("IGSP_TUNE_DEFAULTS", TUNED_TABLE)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.edge_importance.argtypes = [vp, ctypes.POINTER(View), i32, vp, ctypes.POINTER(EdgeOpts), vp]
        L.edge_importance.restype = i32
        L.long_axis_split.argtypes = [ctypes.POINTER(Gaussians), vp, ctypes.POINTER(LasOut),
                                      ctypes.POINTER(LasParams), vp]
        L.long_axis_split.restype = i32
        L.long_axis_split_noalloc.argtypes = L.long_axis_split.argtypes
        L.long_axis_split_noalloc.restype = i32
        L.long_axis_split_full.argtypes = [ctypes.POINTER(Gaussians), ctypes.POINTER(AdamMoments), vp,
                                           ctypes.POINTER(LasOut), ctypes.POINTER(LasParams), vp]
        L.long_axis_split_full.restype = i32
        L.split_mask.argtypes = [vp, ctypes.POINTER(View), i32, ctypes.POINTER(Contributions), vp, vp,
                                 ctypes.c_int64, ctypes.POINTER(SelectParams), vp, vp, vp, vp]
        L.split_mask.restype = i32
        L.igsp_edge_autotune.argtypes = [vp, ctypes.POINTER(View), i32, vp, i32, i32, ctypes.POINTER(EdgeOpts), vp]
        L.igsp_edge_autotune.restype = i32
        L.igsp_edge_resolve.argtypes = [ctypes.POINTER(View), i32, ctypes.POINTER(EdgeOpts)]
        L.igsp_edge_resolve.restype = i32
        L.igsp_step_create.argtypes = [vp, ctypes.POINTER(View), i32, vp, ctypes.POINTER(EdgeOpts),
                                       ctypes.POINTER(Gaussians), vp, ctypes.POINTER(LasOut),
                                       ctypes.POINTER(LasParams), vp, ctypes.POINTER(vp)]
        L.igsp_step_create.restype = i32
        L.igsp_step_launch.argtypes = [vp, vp]
        L.igsp_step_launch.restype = i32
        L.igsp_step_destroy.argtypes = [vp]
        L.igsp_step_destroy.restype = None
        L.igsp_status_string.argtypes = [i32]
        L.igsp_status_string.restype = ctypes.c_char_p
        L.igsp_lr_exponential.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int64]
        L.igsp_lr_exponential.restype = ctypes.c_double
        L.igsp_release_plans.argtypes = []
        L.igsp_release_plans.restype = None
        L.igsp_version.argtypes = []
        L.igsp_version.restype = i32
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().igsp_status_string(int(code)).decode()


def _check(code: int, where: str):
    if code != 0:
        raise IgspError(code, where)


def view_table(widths, heights, in_offset, out_offset):
    n = len(widths)
    arr = (View * max(n, 1))()
    for v in range(n):
        arr[v] = View(int(widths[v]), int(heights[v]), int(in_offset[v]), int(out_offset[v]))
    return arr, n


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _need(t, dtype, name):
    import torch

    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    _ = torch


PLAIN, BATCHED, BATCHED_STAGED, BATCHED_PERSISTENT, UNFUSED = 0, 1, 2, 3, 4
FORMS = {"plain": PLAIN, "batched": BATCHED, "staged": BATCHED_STAGED, "persistent": BATCHED_PERSISTENT,
         "unfused": UNFUSED}
FORM_NAMES = {v: k for k, v in FORMS.items()}


def form_code(batched) -> int:
    """Launch form: True / "batched" (library's choice), False / "plain",
    "staged", "persistent", "unfused", or the integer code."""
    if isinstance(batched, str):
        return FORMS[batched]
    if isinstance(batched, bool):
        return BATCHED if batched else PLAIN
    return int(batched)


def edge_opts(precision="fp32", batched=True, seg_rows=0, wg_waves=0, medians=None, survivors=None,
              stage_events=None, status=None):
    import torch

    _need(medians, torch.float32, "medians")
    _need(survivors, torch.int32, "survivors")
    _need(status, torch.int32, "status")
    if status is not None and status.numel() < 1:
        raise ValueError("status needs one entry")
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ev = None
    if stage_events is not None:   # 4 torch.cuda.Event, each recorded once already
        handles = [int(e.cuda_event) for e in stage_events]
        if len(handles) != 4 or not all(handles):
            raise ValueError("stage_events: four torch.cuda.Event that have been recorded at least once")
        arr = (ctypes.c_void_p * 4)(*handles)
        ev = ctypes.cast(arr, ctypes.c_void_p)
        _EVENT_KEEPALIVE.append(arr)
        del _EVENT_KEEPALIVE[:-8]
    return EdgeOpts(p, form_code(batched), int(seg_rows), int(wg_waves), _ptr(medians), _ptr(survivors), ev,
                    _ptr(status))


_EVENT_KEEPALIVE: list = []


def edge_importance(images, views, out_maps, precision="fp32", batched=True, seg_rows=0, wg_waves=0,
                    medians=None, survivors=None, stage_events=None, stream=None, status=None):
    """Edge-score maps of every view into ``out_maps`` (float32, device).

    images: uint8 device tensor holding the packed views; views: (widths,
    heights, in_offset, out_offset) sequences or a prebuilt view table.
    status: optional int32 device tensor, set to 0 (IGSP_OK) or, by the
    persistent form, -9 (IGSP_ERR_TIMEOUT: the maps are not valid).
    """
    import torch

    _need(images, torch.uint8, "images")
    _need(out_maps, torch.float32, "out_maps")
    tab, n = views if isinstance(views, tuple) and isinstance(views[0], ctypes.Array) else view_table(*views)
    _check_extents(tab, n, images, out_maps, medians, survivors)
    opts = edge_opts(precision, batched, seg_rows, wg_waves, medians, survivors, stage_events, status)
    _check(lib().edge_importance(_ptr(images), tab, n, _ptr(out_maps), ctypes.byref(opts), _stream(stream)),
           "edge_importance")


def _check_extents(tab, n, images, out_maps, medians=None, survivors=None):
    """The C ABI trusts the caller that every view lies inside both buffers;
    check it here, where the tensor sizes are known."""
    if n == 0:
        return
    in_end = max(tab[v].in_offset + 3 * tab[v].width * tab[v].height for v in range(n))
    out_end = max(tab[v].out_offset + tab[v].width * tab[v].height for v in range(n))
    if in_end > images.numel():
        raise ValueError(f"views need {in_end} image bytes, the tensor has {images.numel()}")
    if out_end > out_maps.numel():
        raise ValueError(f"views need {out_end} output floats, the tensor has {out_maps.numel()}")
    for t, nm in ((medians, "medians"), (survivors, "survivors")):
        if t is not None and t.numel() < n:
            raise ValueError(f"{nm} needs {n} entries")


def edge_autotune(images, views, out_maps, precision="fp32", batched=True, stream=None):
    """Tune the tile shape (and, for batched=True, the launch form) on these
    views; returns (seg_rows, wg_waves, form name).

    Later calls with the same ``batched`` and default tile options use the
    result for geometries of the same size class (and IGSP_TUNE_CACHE, if set,
    keeps it across runs).
    """
    import torch

    _need(images, torch.uint8, "images")
    _need(out_maps, torch.float32, "out_maps")
    tab, n = view_table(*views)
    _check_extents(tab, n, images, out_maps)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    best = EdgeOpts()
    _check(lib().igsp_edge_autotune(_ptr(images), tab, n, _ptr(out_maps), p, form_code(batched),
                                    ctypes.byref(best), _stream(stream)), "igsp_edge_autotune")
    return int(best.seg_rows), int(best.wg_waves), FORM_NAMES[int(best.batched)]


def edge_resolve(views, precision="fp32", batched=True, seg_rows=0, wg_waves=0):
    """(form name, seg_rows, wg_waves) that edge_importance would use."""
    tab, n = view_table(*views)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o = EdgeOpts(p, form_code(batched), int(seg_rows), int(wg_waves), None, None, None)
    _check(lib().igsp_edge_resolve(tab, n, ctypes.byref(o)), "igsp_edge_resolve")
    return FORM_NAMES[int(o.batched)], int(o.seg_rows), int(o.wg_waves)


def gaussians_struct(means, log_scales, quats, opacity_logits, count, features=None):
    import torch

    for t, nm in ((means, "means"), (log_scales, "log_scales"), (quats, "quats"),
                  (opacity_logits, "opacity_logits"), (features, "features")):
        _need(t, torch.float32, nm)
    _need(count, torch.int64, "count")
    cap = int(means.shape[0])
    if log_scales.shape[0] != cap or quats.shape[0] != cap or opacity_logits.shape[0] != cap:
        raise ValueError("all Gaussian arrays need the same number of rows (capacity)")
    if count.numel() < 1:
        raise ValueError("count needs one entry")
    for t, w, nm in ((means, 3, "means"), (log_scales, 3, "log_scales"), (quats, 4, "quats")):
        if t.dim() != 2 or t.shape[1] != w:
            raise ValueError(f"{nm} must have shape (capacity, {w})")
    if features is not None and (features.dim() != 2 or features.shape[0] != cap):
        raise ValueError("features must have shape (capacity, F)")
    F = 0 if features is None else int(features.shape[1])
    return Gaussians(_ptr(means), _ptr(log_scales), _ptr(quats), _ptr(opacity_logits), _ptr(features), F,
                     _ptr(count), cap)


def las_params(alpha=0.5, gamma=0.85, beta=0.6):
    return LasParams(alpha, gamma, beta)


def long_axis_split(means, log_scales, quats, opacity_logits, count, mask, split_idx, status,
                    n_split=None, features=None, alpha=0.5, gamma=0.85, beta=0.6, stream=None):
    """Long-Axis-Split in place; N = count[0] on the device becomes N + K."""
    _las("long_axis_split", means, log_scales, quats, opacity_logits, count, mask, split_idx, status, n_split,
         features, alpha, gamma, beta, stream)


def long_axis_split_noalloc(means, log_scales, quats, opacity_logits, count, mask, split_idx, status,
                            n_split=None, features=None, alpha=0.5, gamma=0.85, beta=0.6, stream=None):
    """long_axis_split with the library's fixed workspace: allocates nothing
    (capacity up to 2^28 rows). Calls that overlap on one GPU race."""
    _las("long_axis_split_noalloc", means, log_scales, quats, opacity_logits, count, mask, split_idx, status,
         n_split, features, alpha, gamma, beta, stream)


def _las(entry, means, log_scales, quats, opacity_logits, count, mask, split_idx, status, n_split, features,
         alpha, gamma, beta, stream):
    import torch

    _need(mask, torch.uint8, "mask")
    _need(split_idx, torch.int32, "split_idx")
    _need(status, torch.int32, "status")
    _need(n_split, torch.int64, "n_split")
    g = gaussians_struct(means, log_scales, quats, opacity_logits, count, features)
    if mask.numel() < g.capacity or split_idx.numel() < g.capacity:
        raise ValueError("mask and split_idx need capacity entries")
    if status.numel() < 1 or (n_split is not None and n_split.numel() < 1):
        raise ValueError("status and n_split need one entry")
    out = LasOut(_ptr(split_idx), _ptr(status), _ptr(n_split))
    prm = las_params(alpha, gamma, beta)
    _check(getattr(lib(), entry)(ctypes.byref(g), _ptr(mask), ctypes.byref(out), ctypes.byref(prm),
                                 _stream(stream)), entry)


ADAM_GROUPS = ("means", "log_scales", "quats", "opacity_logits", "features")


def long_axis_split_full(means, log_scales, quats, opacity_logits, count, mask, split_idx, status, moments,
                         n_split=None, features=None, alpha=0.5, gamma=0.85, beta=0.6, stream=None):
    """The full-record split: long_axis_split plus the optimiser state.

    moments: {group: (m, v)} for groups in ADAM_GROUPS, each tensor in the
    group's row layout (either of the pair may be None); both children's
    moment rows are cleared.
    """
    import torch

    _need(mask, torch.uint8, "mask")
    _need(split_idx, torch.int32, "split_idx")
    _need(status, torch.int32, "status")
    _need(n_split, torch.int64, "n_split")
    g = gaussians_struct(means, log_scales, quats, opacity_logits, count, features)
    if mask.numel() < g.capacity or split_idx.numel() < g.capacity:
        raise ValueError("mask and split_idx need capacity entries")
    widths = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "features": g.feat_dim}
    ptrs = {}
    for grp, pair in (moments or {}).items():
        if grp not in widths:
            raise ValueError(f"unknown moment group {grp}")
        for k, t in enumerate(pair):
            _need(t, torch.float32, f"moments[{grp}][{k}]")
            if t is not None and t.numel() < g.capacity * widths[grp]:
                raise ValueError(f"moments[{grp}][{k}] needs {g.capacity} x {widths[grp]} floats")
        ptrs[grp] = (ctypes.c_void_p * 2)(*[_ptr(t) for t in pair])
    adam = AdamMoments(*[ptrs.get(grp, (ctypes.c_void_p * 2)(None, None)) for grp in ADAM_GROUPS])
    out = LasOut(_ptr(split_idx), _ptr(status), _ptr(n_split))
    prm = las_params(alpha, gamma, beta)
    _check(lib().long_axis_split_full(ctypes.byref(g), ctypes.byref(adam), _ptr(mask), ctypes.byref(out),
                                      ctypes.byref(prm), _stream(stream)), "long_axis_split_full")


def split_mask(maps, views, gauss, view, pixel, weight, grad, count, mask, scores, grad_threshold=0.0,
               warmup=False, budget=None, n_selected=None, stream=None):
    """Split mask from edge scores into ``mask`` (uint8) and ``scores`` (int64,
    units of 2^-32); N = count[0] on the device; budget None = capacity."""
    import torch

    _need(maps, torch.float32, "maps")
    for t, dt, nm in ((gauss, torch.int32, "gauss"), (view, torch.int32, "view"), (pixel, torch.int32, "pixel"),
                      (weight, torch.float32, "weight"), (grad, torch.float32, "grad"), (count, torch.int64, "count"),
                      (mask, torch.uint8, "mask"), (scores, torch.int64, "scores")):
        if t is None:
            raise ValueError(f"{nm} is required")
        _need(t, dt, nm)
    _need(n_selected, torch.int64, "n_selected")
    n = int(gauss.numel())
    if not (view.numel() == pixel.numel() == weight.numel() == n):
        raise ValueError("gauss, view, pixel and weight need the same length")
    cap = int(mask.numel())
    if grad.numel() < cap or scores.numel() < cap:
        raise ValueError("grad and scores need capacity entries")
    tab, nv = view_table(*views)
    if nv:
        out_end = max(tab[v].out_offset + tab[v].width * tab[v].height for v in range(nv))
        if out_end > maps.numel():
            raise ValueError(f"views need {out_end} map floats, the tensor has {maps.numel()}")
    c = Contributions(_ptr(gauss), _ptr(view), _ptr(pixel), _ptr(weight), n)
    prm = SelectParams(float(grad_threshold), int(bool(warmup)), cap if budget is None else int(budget))
    _check(lib().split_mask(_ptr(maps), tab, nv, ctypes.byref(c), _ptr(grad), _ptr(count), cap,
                            ctypes.byref(prm), _ptr(mask), _ptr(scores), _ptr(n_selected), _stream(stream)),
           "split_mask")


class Step:
    """One densification step (edge maps + LAS) recorded as a HIP graph."""

    def __init__(self, images, views, out_maps, gaussian_args: dict, mask, split_idx, status, n_split=None,
                 precision="bf16", batched=True, seg_rows=0, wg_waves=0, alpha=0.5, gamma=0.85, beta=0.6,
                 stream=None):
        self._keep = (images, out_maps, mask, split_idx, status, n_split, gaussian_args)
        import torch

        self._tab, n = view_table(*views)
        _need(images, torch.uint8, "images")
        _need(out_maps, torch.float32, "out_maps")
        _check_extents(self._tab, n, images, out_maps)
        self._opts = edge_opts(precision, batched, seg_rows, wg_waves)
        self._g = gaussians_struct(**gaussian_args)
        _need(mask, torch.uint8, "mask")
        _need(split_idx, torch.int32, "split_idx")
        _need(status, torch.int32, "status")
        if mask.numel() < self._g.capacity or split_idx.numel() < self._g.capacity or status.numel() < 1:
            raise ValueError("mask and split_idx need capacity entries, status one")
        self._out = LasOut(_ptr(split_idx), _ptr(status), _ptr(n_split))
        self._prm = las_params(alpha, gamma, beta)
        h = ctypes.c_void_p()
        _check(lib().igsp_step_create(_ptr(images), self._tab, n, _ptr(out_maps), ctypes.byref(self._opts),
                                      ctypes.byref(self._g), _ptr(mask), ctypes.byref(self._out),
                                      ctypes.byref(self._prm), _stream(stream), ctypes.byref(h)),
               "igsp_step_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().igsp_step_launch(self._h, _stream(stream)), "igsp_step_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib().igsp_step_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lr_exponential(t: int, lr_init: float, lr_final: float, t_max: int) -> float:
    """Exponential learning-rate schedule (host): lr_init -> lr_final over t_max."""
    return float(lib().igsp_lr_exponential(int(t), float(lr_init), float(lr_final), int(t_max)))


def release_plans():
    lib().igsp_release_plans()
