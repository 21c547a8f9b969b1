"""Edge-map error against the FP64 oracle, per storage precision, on full-size
views: every pixel of six views of the 150-view workload (2473x1643 and its
2x downsample, first, middle and last views) and of the single 1297x840
view, computed in the benchmark's batched form.

Reported per precision (one printed line each; run with -s):
  * suppression decisions that differ from the oracle's, and how many pixels
    are exempt (oracle decision margin below the stated epsilon);
  * max |E - E_ref| and max |E - E_ref| / max(1, E_ref) over pixels with equal
    decisions, and the largest E_ref (the map is unbounded, so a 2-byte
    storage's relative rounding gives an absolute error that grows with E);
  * max relative error of the per-view median;
  * how many pixels are off by more than 1e-2, and the smallest E_ref among
    them.
The parity bars themselves are the ones every other edge test applies."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_view, gpu_edge, view_map

pytestmark = pytest.mark.gpu

SAMPLE = [0, 1, 74, 75, 148, 149]


def _batch():
    w = synth.workload("views150_2473x1643_mixed")
    imgs = [w.render(views=SAMPLE)]
    one = synth.workload("view_1297x840").render()
    # the sampled full-size views and the single view, packed together
    views = [imgs[0].view(k) for k in range(imgs[0].n)] + [one.view(0)]
    return synth.pack_views(views, in_align=256, out_align=64)


def test_error_per_precision():
    vb = _batch()
    refs = [oracle.edge_view(vb.view(k)) for k in range(vb.n)]
    e_max = max(float(r["E"].max()) for r in refs)
    for p in ("fp32", "fp16", "bf16"):
        E, med, nsv = gpu_edge(vb, p)
        px = mism = exempt = over = 0
        plain = scaled = med_rel = 0.0
        e_over = np.inf
        for k in range(vb.n):
            st = compare_view(view_map(E, vb, k), refs[k], p, med[k], nsv[k])
            px += st["px"]
            mism += st["mismatch"]
            exempt += st["exempt"]
            plain = max(plain, st["plain_err"])
            scaled = max(scaled, st["scaled_err"])
            med_rel = max(med_rel, st.get("med_rel", 0.0))
            Eg, Er = view_map(E, vb, k).astype(np.float64), refs[k]["E"]
            big = (np.abs(Eg - Er) > 1e-2) & ((Eg > 0) == (Er > 0))
            over += int(big.sum())
            if big.any():
                e_over = min(e_over, float(Er[big].min()))
        print(f"{p}: {vb.n} views, {px} px; decision mismatches {mism} ({mism / px:.2e}), exempt {exempt}; "
              f"max |E-E_ref| {plain:.3e}, max scaled {scaled:.3e} (largest E_ref {e_max:.1f}); "
              f"median max rel {med_rel:.3e}; |E-E_ref| > 1e-2 at {over} px ({over / px:.2e}), "
              f"all with E_ref >= {e_over:.2f}", flush=True)
        assert mism <= exempt
        if p == "fp32":
            assert plain <= 1e-3
