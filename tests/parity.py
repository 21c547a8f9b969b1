"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare it with the CPU oracle element by element.

Tolerances (the arithmetic behind them):
  * Suppression decisions are made in FP32 on exact integer gradients in every
    storage mode, so a decision can differ from the oracle's exact one only
    where the oracle's decision margin c(p) is within FP32 rounding of zero:
    pixels with c(p) < NMS_EPS are exempt, every other pixel must match.
  * Maps: over pixels with the same decision, |E_gpu - E_ref| / max(1, E_ref)
    <= 1e-3 (FP32 storage) or 1e-2 (FP16 / BF16 storage: each stored value
    carries a relative rounding of 2^-11 / 2^-9, the map is a ratio of two
    such values). FP32 also meets a plain absolute bound of 1e-3.
  * The median is an exact selection of stored values, so it equals the
    oracle's median rounded to the storage format (plus FP32 rounding of the
    magnitude, 2^-22 relative).
"""
from __future__ import annotations

import numpy as np

import oracle
import synth

NMS_EPS = 1e-6
E_TOL = {"fp32": 1e-3, "fp16": 1e-2, "bf16": 1e-2}
MED_RTOL = {"fp32": 2.0 ** -20, "fp16": 2.0 ** -10, "bf16": 2.0 ** -8}


def gpu_edge(vb: synth.ViewBatch, precision="fp32", batched=True, seg_rows=0, wg_waves=0, reps=1):
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    pad = (-vb.rgb.size) % 16 + 16
    img = torch.from_numpy(np.concatenate([vb.rgb, np.zeros(pad, np.uint8)])).to(dev)
    out = torch.full((max(vb.out_floats, 1),), -7.0, dtype=torch.float32, device=dev)
    med = torch.zeros(vb.n, dtype=torch.float32, device=dev)
    nsv = torch.zeros(vb.n, dtype=torch.int32, device=dev)
    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    for _ in range(reps):
        igsp.edge_importance(img, views, out, precision=precision, batched=batched, seg_rows=seg_rows,
                             wg_waves=wg_waves, medians=med, survivors=nsv)
    torch.cuda.synchronize()
    return out.cpu().numpy(), med.cpu().numpy(), nsv.cpu().numpy()


def view_map(flat: np.ndarray, vb: synth.ViewBatch, v: int) -> np.ndarray:
    W, H, o = int(vb.widths[v]), int(vb.heights[v]), int(vb.out_offset[v])
    return flat[o:o + W * H].reshape(H, W)


def compare_view(E_gpu: np.ndarray, ref: dict, precision: str, med_gpu=None, nsv_gpu=None) -> dict:
    """Assert parity of one view's map against the oracle's stages; return stats."""
    keep_g = E_gpu > 0
    keep_r = ref["keep"] > 0
    mism = keep_g != keep_r
    exempt = ref["margin"] < NMS_EPS
    bad = mism & ~exempt
    assert not bad.any(), f"{int(bad.sum())} non-exempt NMS mismatches, e.g. at {np.argwhere(bad)[:5].tolist()}"
    assert np.isfinite(E_gpu).all() and (E_gpu >= 0).all()
    same = ~mism
    Er = ref["E"]
    diff = np.abs(E_gpu.astype(np.float64) - Er)
    scaled = float((diff[same] / np.maximum(1.0, Er[same])).max()) if same.any() else 0.0
    plain = float(diff[same].max()) if same.any() else 0.0
    assert scaled <= E_TOL[precision], f"scaled map error {scaled} > {E_TOL[precision]}"
    if precision == "fp32":
        assert plain <= 1e-3, f"plain map error {plain}"
    stats = {"mismatch": int(mism.sum()), "exempt": int(exempt.sum()), "px": int(E_gpu.size),
             "scaled_err": scaled, "plain_err": plain}
    if med_gpu is not None and ref["n"] > 0 and not mism.any():
        rel = abs(float(med_gpu) - ref["med"]) / ref["med"]
        assert rel <= MED_RTOL[precision], f"median {med_gpu} vs {ref['med']} (rel {rel})"
        stats["med_rel"] = rel
    if nsv_gpu is not None:
        assert abs(int(nsv_gpu) - ref["n"]) <= int(mism.sum())
    if ref["n"] > 0 and not mism.any():
        # the survivor holding the median maps to exactly 1
        assert (E_gpu == 1.0).any()
    if ref["n"] == 0:
        assert (E_gpu == 0).all()
    return stats


def check_batch(vb: synth.ViewBatch, precision="fp32", batched=True, views=None, **kw) -> list:
    E, med, nsv = gpu_edge(vb, precision, batched, **kw)
    out = []
    for v in (range(vb.n) if views is None else views):
        ref = oracle.edge_view(vb.view(v))
        out.append(compare_view(view_map(E, vb, v), ref, precision, med[v], nsv[v]))
    return out
