"""Maximum view size: a view of 45601 x 42301 = 1.93 G pixels (the ABI's
limit is W * H < 2^31), far beyond what the oracle can hold, checked through
a property that holds at any size.

Mirror tiling: L(x, y) = S(fold(x, W), fold(y, H)) with fold the reflect-101
index map and L's sides k(W - 1) + 1, so L's own borders are reflection axes
of the tiling. Every stage of the method then sees at (x, y) of L exactly
what it sees at (fold x, fold y) of S (the blur is symmetric, the Sobel
difference odd and the magnitude even under each reflection), so:
  * the suppression decisions of L are S's read through the folds, exactly;
  * L's survivors are S's survivors, each counted m_x * m_y times (its
    column's and row's multiplicity in the tiling: an edge column or row of
    S appears once per period, any other twice), so L's median is the
    weighted lower median of S's magnitudes, computed here by the oracle;
  * L's map is S's map times one constant, sqrt(med_S / med_L) (FP32, BF16
    storage: the map is sqrt(q / median)), up to the rounding of the final
    division and root.
S's map itself is checked against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import MED_RTOL, compare_view

pytestmark = pytest.mark.gpu


def _fold(i, n):
    P = 2 * (n - 1)
    i = np.mod(i, P)
    return np.where(i < n, i, P - i)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_max_size_view_is_mirror_tiling(precision):
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    Ws, Hs = 1201, 901
    S = synth.image(4242, Ws, Hs, 60, True)
    Wl, Hl = 38 * (Ws - 1) + 1, 47 * (Hs - 1) + 1       # 45601 x 42301
    assert Wl * Hl < 2 ** 31
    print(f"max-size view {Wl} x {Hl} = {Wl * Hl / 1e9:.3f} G px, {precision}", flush=True)
    # the small view on its own, against the oracle
    s_img = torch.from_numpy(np.concatenate([S.reshape(-1), np.zeros(16, np.uint8)])).to(dev)
    s_out = torch.zeros(Ws * Hs, dtype=torch.float32, device=dev)
    s_med = torch.zeros(1, dtype=torch.float32, device=dev)
    igsp.edge_importance(s_img, ([Ws], [Hs], [0], [0]), s_out, precision=precision, medians=s_med)
    torch.cuda.synchronize()
    compare_view(s_out.cpu().numpy().reshape(Hs, Ws), oracle.edge_view(S), precision)
    # the large view, built on the device from S through the folds
    fx = torch.from_numpy(_fold(np.arange(Wl), Ws)).to(dev)
    fy = torch.from_numpy(_fold(np.arange(Hl), Hs)).to(dev)
    St = torch.from_numpy(S).to(dev)
    L = torch.empty((Hl * Wl * 3 + 16,), dtype=torch.uint8, device=dev)
    Lv = L[:Hl * Wl * 3].view(Hl, Wl, 3)
    for y0 in range(0, Hl, 4096):                       # row blocks keep the temporaries small
        y1 = min(Hl, y0 + 4096)
        Lv[y0:y1] = St[fy[y0:y1]][:, fx]
    out = torch.empty(Hl * Wl, dtype=torch.float32, device=dev)
    med = torch.zeros(1, dtype=torch.float32, device=dev)
    nsv = torch.zeros(1, dtype=torch.int32, device=dev)
    igsp.edge_importance(L, ([Wl], [Hl], [0], [0]), out, precision=precision, medians=med, survivors=nsv)
    torch.cuda.synchronize()
    # median of L: the oracle's survivors of S weighted by their multiplicity in L
    ref = oracle.edge_view(S)
    mx = np.bincount(_fold(np.arange(Wl), Ws), minlength=Ws).astype(np.int64)
    my = np.bincount(_fold(np.arange(Hl), Hs), minlength=Hs).astype(np.int64)
    keep = ref["keep"] > 0
    mult = (my[:, None] * mx[None, :])[keep]
    Mk = ref["M"][keep].astype(np.float64)
    order = np.argsort(Mk, kind="stable")
    cum = np.cumsum(mult[order])
    n_total = int(cum[-1])
    k = (n_total - 1) // 2
    m_med = Mk[order][np.searchsorted(cum, k + 1)]
    med_dn = np.sqrt(m_med) / 256000.0
    assert int(nsv.item()) == n_total
    rel = abs(med.item() - med_dn) / med_dn
    assert rel <= MED_RTOL[precision], f"median of L {med.item()} vs weighted oracle median {med_dn} (rel {rel})"
    # maps: same decisions, values S's times one constant
    # E = sqrt(q / median) and the medians come back in DN, sqrt(median) / 256000
    c = float(np.float64(s_med.item()) / np.float64(med.item()))
    s_map = s_out.view(Hs, Ws)
    ov = out.view(Hl, Wl)
    bad_keep, worst = 0, 0.0
    for y0 in range(0, Hl, 4096):
        y1 = min(Hl, y0 + 4096)
        a = ov[y0:y1]
        b = s_map[fy[y0:y1]][:, fx]
        bad_keep += int(((a > 0) != (b > 0)).sum().item())
        both = b > 0
        r = (a[both].double() / (b[both].double() * c) - 1.0).abs()
        worst = max(worst, float(r.max().item()) if r.numel() else 0.0)
    assert bad_keep == 0, f"{bad_keep} suppression decisions differ from the mirror tiling"
    assert worst <= 4e-6, f"map of L vs S's map x constant: relative {worst}"
    print(f"survivors {n_total}, median rel {rel:.2e}, worst value rel {worst:.2e}", flush=True)
    del L, Lv, out
    torch.cuda.empty_cache()
