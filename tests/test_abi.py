"""C ABI on the host (no GPU): the library loads, exports every symbol the
header declares, and rejects invalid arguments with the documented status
before touching the GPU. Pointers below are never dereferenced: validation
only compares their values."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2603_08661_amd as igsp
from paper_2603_08661_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igsp.h")

FAKE_IMG = 0x7F0000000000          # 16-byte aligned, never dereferenced
FAKE_OUT = 0x7F1000000000


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?([a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol():
    L = igsp.lib()
    names = declared_functions()
    assert set(names) == set(B.EXPORTS), names
    for n in names:
        assert hasattr(L, n), n
    assert L.igsp_version() == 1


def test_status_strings():
    for code in B.STATUS:
        assert igsp.status_string(code)
    assert "capacity" in igsp.status_string(-6)


def edge(views, n=None, images=FAKE_IMG, out=FAKE_OUT, opts=None):
    arr = (B.View * max(len(views), 1))(*[B.View(*v) for v in views])
    n = len(views) if n is None else n
    o = ctypes.byref(opts) if opts is not None else None
    return igsp.lib().edge_importance(images, arr, n, out, o, None)


GOOD = [(16, 8, 0, 0), (5, 3, 16 * 8 * 3, 16 * 8)]


@pytest.mark.parametrize("views,n,kw,code", [
    (GOOD, -1, {}, -2),
    (GOOD, 0, {"images": 0, "out": 0}, 0),           # n = 0: no-op even with NULLs
    (GOOD, None, {"images": 0}, -1),
    (GOOD, None, {"out": 0}, -1),
    (GOOD, None, {"images": FAKE_IMG + 3}, -3),
    ([(2, 8, 0, 0)], None, {}, -2),
    ([(8, 2, 0, 0)], None, {}, -2),
    ([(65536, 32768, 0, 0)], None, {}, -2),            # W*H = 2^31
    ([(8, 8, -1, 0)], None, {}, -2),
    ([(8, 8, 0, -5)], None, {}, -2),
    ([(16, 16, 0, 0)], None, {"out": FAKE_IMG + 100}, -4),
    ([(16, 16, 0, 0)], None, {"out": FAKE_IMG - 4 * 256 + 4}, -4),
])
def test_edge_validation(views, n, kw, code):
    assert edge(views, n, **kw) == code


@pytest.mark.parametrize("field,val", [("precision", 3), ("precision", -1), ("batched", 5), ("batched", -1), ("seg_rows", 4),
                                       ("seg_rows", 5000), ("wg_waves", 3), ("wg_waves", 16)])
def test_edge_bad_options(field, val):
    o = B.EdgeOpts(0, 1, 0, 0, None, None, None)
    setattr(o, field, val)
    assert edge(GOOD, opts=o) == -5


def las(g=None, mask=0x1000, out=None, prm=None):
    g = g or B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 100)
    out = out or B.LasOut(0x60, 0x70, None)
    L = igsp.lib()
    return L.long_axis_split(ctypes.byref(g) if g else None, mask, ctypes.byref(out),
                             ctypes.byref(prm) if prm else None, None)


def test_las_validation():
    L = igsp.lib()
    assert L.long_axis_split(None, 0x1000, None, None, None) == -1
    assert las(mask=0) == -1
    for k in ("means", "log_scales", "quats", "opacity_logits", "count"):
        g = B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 100)
        setattr(g, k, 0)
        assert las(g=g) == -1, k
    assert las(out=B.LasOut(0, 0x70, None)) == -1
    assert las(out=B.LasOut(0x60, 0, None)) == -1
    assert las(g=B.Gaussians(0x10, 0x20, 0x30, 0x40, None, -1, 0x50, 100)) == -5
    assert las(g=B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 4, 0x50, 100)) == -1   # feat_dim > 0, NULL features
    assert las(g=B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, -1)) == -2
    assert las(g=B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 2 ** 31)) == -2
    for a, gm, b in ((0.0, 0.85, 0.6), (0.5, 1.5, 0.6), (0.5, 0.85, -0.1), (math.nan, 0.85, 0.6),
                     (0.5, 0.85, math.inf)):
        assert las(prm=B.LasParams(a, gm, b)) == -5


def test_las_noalloc_validation():
    """The allocation-free split validates like long_axis_split and rejects a
    capacity above its fixed workspace before touching the GPU."""
    L = igsp.lib()
    out = B.LasOut(0x60, 0x70, None)

    def call(g, mask=0x1000):
        return L.long_axis_split_noalloc(ctypes.byref(g), mask, ctypes.byref(out), None, None)

    assert L.long_axis_split_noalloc(None, 0x1000, None, None, None) == -1
    assert call(B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 100), mask=0) == -1
    assert call(B.Gaussians(0x10, 0, 0x30, 0x40, None, 0, 0x50, 100)) == -1
    assert call(B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, -1)) == -2
    assert call(B.Gaussians(0x10, 0x20, 0x30, 0x40, None, -1, 0x50, 100)) == -5
    assert call(B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 2 ** 28 + 1)) == -10
    assert call(B.Gaussians(0x10, 0x20, 0x30, 0x40, None, 0, 0x50, 2 ** 31 - 1)) == -10
    assert "workspace" in igsp.status_string(-10)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libigsp.so")
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.lib()


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2603_08661_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".cpp", ".h", ".c")) or f == "Makefile":
                txt = open(os.path.join(dp, f)).read()
                assert not re.search(r"\boracle\b|igsp_oracle|liboracle", txt), f


def test_view_struct_layout_matches_header():
    assert ctypes.sizeof(B.View) == 24
    assert ctypes.sizeof(B.EdgeOpts) == 48
    assert ctypes.sizeof(B.Gaussians) == 64
    assert ctypes.sizeof(B.LasOut) == 24
    assert np.dtype([("w", "<i4"), ("h", "<i4"), ("i", "<i8"), ("o", "<i8")]).itemsize == 24


def test_null_stage_event_rejected():
    ev = (ctypes.c_void_p * 4)(1, 2, None, 4)
    o = B.EdgeOpts(0, 1, 0, 0, None, None, ctypes.cast(ev, ctypes.c_void_p))
    assert edge(GOOD, opts=o) == -1


def test_tuning_table_lookup_and_override(tmp_path):
    """The shipped table and the caller's cache are read once per process
    (a fresh interpreter here): entries of the view batch's size class pick
    the form and tile, the cache wins over the table, and malformed lines or
    out-of-range values are ignored."""
    import subprocess
    import sys

    # 1000 x 800: 800000 px -> log2 19; mean width 1000 -> log2 9; no GPU -> arch "unknown"
    row = ('{{"arch":"unknown","precision":2,"batched":1,"log2_px":19,"log2_w":9,'
           '"seg_rows":{s},"wg_waves":{w},"form":{f},"ms":1.0}}')
    table = tmp_path / "table.jsonl"
    table.write_text("not json\n" + row.format(s=96, w=2, f=3) + "\n"
                     + row.format(s=96, w=3, f=3).replace('"precision":2', '"precision":1') + "\n")
    cache = tmp_path / "cache.jsonl"
    code = ("import paper_2603_08661_amd as g; v=([1000],[800],[0],[0]);"
            "print(g.edge_resolve(v,'bf16'), g.edge_resolve(v,'fp16'), g.edge_resolve(v,'bf16',seg_rows=32),"
            " g.edge_resolve(v,'bf16','staged'))")
    env = dict(os.environ, IGSP_TUNE_DEFAULTS=str(table), IGSP_TUNE_CACHE=str(cache))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout.strip()
    # no entry: 4 wavefronts per work-group and, for one 1000 x 800 view (5 strips), the shortest
    # segment height, since no height gives the stencil launch 16 wavefronts per CU
    assert out == ("('persistent', 96, 2) ('staged', 10, 4) ('persistent', 32, 4) ('staged', 10, 4)"), out
    cache.write_text(row.format(s=48, w=8, f=2) + "\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout.strip()
    assert out.startswith("('staged', 48, 8)"), out


def test_split_mask_validation():
    L = igsp.lib()
    good_c = B.Contributions(0x10, 0x20, 0x30, 0x40, 5)
    prm = B.SelectParams(0.0, 0, 100)
    arr = (B.View * 1)(B.View(4, 4, 0, 0))

    def call(c=good_c, p=prm, cap=100, maps=0x50, grad=0x60, count=0x70, mask=0x80, scores=0x90, nv=1):
        return L.split_mask(maps, arr, nv, ctypes.byref(c) if c else None, grad, count, cap,
                            ctypes.byref(p) if p else None, mask, scores, None, None)

    assert call(c=None) == -1 and call(p=None) == -1
    assert call(grad=0) == -1 and call(count=0) == -1 and call(mask=0) == -1 and call(scores=0) == -1
    assert call(maps=0) == -1                                     # entries but no maps
    assert call(c=B.Contributions(0x10, 0, 0x30, 0x40, 5)) == -1
    assert call(c=B.Contributions(0, 0, 0, 0, -1)) == -2
    assert call(cap=-1) == -2 and call(cap=2 ** 31) == -2 and call(nv=-1) == -2
    assert call(p=B.SelectParams(0.0, 2, 100)) == -5
    assert call(p=B.SelectParams(0.0, 0, -1)) == -5
    assert call(p=B.SelectParams(float("nan"), 0, 100)) == -5
    assert ctypes.sizeof(B.Contributions) == 40 and ctypes.sizeof(B.SelectParams) == 16


def test_shipped_tuning_table_is_well_formed_and_covers_the_benchmark():
    """Every entry of the shipped table names a form, tile and size class the
    library accepts (batched request, staged or persistent answer, a segment
    height of the autotuner's list, 1-8 waves), and every batched benchmark
    geometry (in each precision it is measured in) finds an entry: the
    table is what the benchmark's default launches read."""
    import json

    import synth

    path = os.path.join(ROOT, "paper_2603_08661_amd", "tuned", "gfx950.jsonl")
    rows = [json.loads(line) for line in open(path) if line.strip()]
    assert rows, "empty tuning table"
    keys = set()
    for r in rows:
        assert r["arch"] == "gfx950"
        assert r["precision"] in (0, 1, 2) and r["batched"] == 1 and r["form"] in (2, 3)
        assert r["seg_rows"] in (10, 16, 22, 28, 40, 64, 88, 100, 124, 148, 196, 244) and r["wg_waves"] in (1, 2, 4, 8)
        assert r["ms"] > 0
        keys.add((r["precision"], r["log2_px"], r["log2_w"]))
    assert len(keys) == len(rows), "duplicate size classes"

    def ilog2(v):
        return int(v).bit_length() - 1

    prec_code = {"fp32": 0, "fp16": 1, "bf16": 2}
    for name in ("view_256x192", "view_1297x840", "views200_w1000_1560", "views150_2473x1643_mixed",
                 "step_views300_las3m"):
        w = synth.workload(name)
        widths, heights = (np.asarray(a, np.int64) for a in w.sizes())
        key_px = ilog2(max(int((widths * heights).sum()), 1))
        key_w = ilog2(max(int(widths.sum()) // len(widths), 1))
        for p in w.extra.get("precisions", [w.precision]):
            assert (prec_code[p], key_px, key_w) in keys, (name, p, key_px, key_w)


def test_default_segment_height_follows_the_launch_size():
    """With no tuned entry, the segment height is the tallest of 64, 40, 28,
    22, 16 rows that gives the stencil launch 16 wavefronts per CU (no device
    here: 256 CUs, 4096 wavefronts), else 10; the plain form counts one
    view's launch, the batched forms all views together."""
    import subprocess
    import sys

    code = ("import paper_2603_08661_amd as g\n"
            "def v(n, w, h): return ([w] * n, [h] * n, [0] * n, [0] * n)\n"
            "print([g.edge_resolve(v(*a), 'bf16', f)[1] for a, f in ("
            "((300, 2000, 1300), 'staged'), ((60, 1000, 800), 'staged'), ((40, 1000, 800), 'staged'),"
            "((300, 2000, 1300), 'plain'), ((1, 3840, 2160), 'plain'), ((1, 256, 192), 'staged'))])\n")
    env = dict(os.environ, IGSP_TUNE_DEFAULTS="", IGSP_TUNE_CACHE="")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout.strip()
    # 300 x 9 strips x 21 segments of 64 rows = 56700; 60 x 5 x 13 = 3900 < 4096 <= 60 x 5 x 20 = 6000;
    # 40 x 5 x 20 = 4000, 40 x 5 x 29 = 5800 (28 rows); one 2000 x 1300 view: 9 x 130 = 1170 at 10 rows;
    # 3840 x 2160: 16 x 216 = 3456 at 10 rows
    assert out == "[64, 40, 28, 10, 10, 10]", out
