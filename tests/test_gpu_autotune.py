"""The tile-shape autotuner: it returns a candidate shape, persists it to the
cache file, and later calls with default tile options use it -- their maps
equal an explicit call with the tuned shape bit for bit, and match the oracle."""
import json

import numpy as np
import pytest

import oracle
import synth
from parity import compare_view, view_map

pytestmark = pytest.mark.gpu


def test_autotune_shape_is_used_and_cached(tmp_path, monkeypatch):
    import torch

    import paper_2603_08661_amd as igsp

    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("IGSP_TUNE_CACHE", str(cache))
    dev = torch.device("cuda:0")
    imgs = [synth.image(90 + k, w, h, 12, True) for k, (w, h) in enumerate([(733, 311), (402, 517), (257, 129)])]
    vb = synth.pack_views(imgs, in_align=16, out_align=4)
    img = torch.from_numpy(np.concatenate([vb.rgb, np.zeros(32, np.uint8)])).to(dev)
    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    out = torch.zeros(vb.out_floats, dtype=torch.float32, device=dev)
    seg, wgw, form = igsp.edge_autotune(img, views, out, precision="bf16")
    assert seg in (10, 16, 22, 28, 40, 64, 88, 100, 124, 148, 196, 244) and wgw in (1, 2, 4, 8)
    assert form in ("staged", "persistent")
    rows = [json.loads(line) for line in cache.read_text().splitlines()]
    assert any(r["seg_rows"] == seg and r["wg_waves"] == wgw and r["precision"] == igsp.BF16
               and r["form"] == igsp.FORMS[form] for r in rows)

    a = torch.zeros_like(out)
    b = torch.zeros_like(out)
    igsp.edge_importance(img, views, a, precision="bf16")  # default options -> tuned form and shape
    igsp.edge_importance(img, views, b, precision="bf16", batched=form, seg_rows=seg, wg_waves=wgw)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a, b)
    for v in range(vb.n):
        compare_view(view_map(a, vb, v), oracle.edge_view(vb.view(v)), "bf16")
