"""GPU parity of long_axis_split against the CPU oracle (through the C ABI).

Bit-exact: status, K, new count, split indices, the longest axis, copied
fields, untouched rows and the canary rows past N + K. Floating point:
means |d| <= 16 * 2^-24 * (|p| + |offset|), log-scales <= 4 * 2^-24 *
max(1, |s'|), opacity logits <= 1e-6 * max(1, |o'|).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
CANARY = 12345.0


def run_las(g: synth.GaussianSet, N: int, mask: np.ndarray, cap: int, feats=None, calls=1, **prm):
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")

    def padded(a, rows):
        out = np.full((rows,) + a.shape[1:], CANARY, np.float32)
        out[:min(rows, a.shape[0])] = a[:rows]
        return out

    host = {"means": padded(g.means, cap), "log_scales": padded(g.log_scales, cap),
            "quats": padded(g.quats, cap), "opacity_logits": padded(g.opacity_logits, cap)}
    if feats is not None:
        host["features"] = padded(feats, cap)
    t = {k: torch.from_numpy(v.copy()).to(dev) for k, v in host.items()}
    count = torch.tensor([N], dtype=torch.int64, device=dev)
    mk = np.zeros(cap, np.uint8)
    mk[:min(cap, mask.size)] = mask[:cap]
    tmask = torch.from_numpy(mk).to(dev)
    sidx = torch.full((max(cap, 1),), -1, dtype=torch.int32, device=dev)
    status = torch.full((1,), 99, dtype=torch.int32, device=dev)
    nsplit = torch.full((1,), -1, dtype=torch.int64, device=dev)
    for _ in range(calls):
        igsp.long_axis_split(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], count, tmask, sidx,
                             status, n_split=nsplit, features=t.get("features"), **prm)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in t.items()}
    res.update(count=int(count.item()), status=int(status.item()), K=int(nsplit.item()),
               split_idx=sidx.cpu().numpy(), host=host, mask=mk)
    return res


def compare(res, N, cap, feats=None, **prm):
    h = res["host"]
    ref = oracle.las(N, h["means"], h["log_scales"], h["quats"], h["opacity_logits"], res["mask"][:N],
                     feats=h.get("features"), **{k: v for k, v in prm.items()})
    assert res["status"] == (0 if ref["status"] == 0 else -6)
    assert res["K"] == ref["K"]
    assert res["count"] == ref["count"]
    if ref["status"] != 0:
        for k in ("means", "log_scales", "quats", "opacity_logits"):
            assert (res[k] == h[k]).all(), k
        assert (res["split_idx"] == -1).all()
        return ref
    K = ref["K"]
    assert (res["split_idx"][:K] == ref["split_idx"]).all()
    assert (res["split_idx"][K:] == -1).all()
    sel = ref["split_idx"].astype(np.int64)
    child = N + np.arange(K)
    touched = np.zeros(cap, bool)
    touched[sel] = True
    touched[child] = True
    for k in ("means", "log_scales", "quats", "opacity_logits"):
        assert (res[k][~touched] == h[k][~touched]).all(), f"untouched rows changed in {k}"
    # quaternion: parent kept in place, copied bit-exactly to the second child
    assert (res["quats"][sel] == h["quats"][sel]).all() and (res["quats"][child] == h["quats"][sel]).all()
    if feats is not None:
        assert (res["features"][child] == h["features"][sel]).all()
        assert (res["features"][sel] == h["features"][sel]).all()
    rows = np.concatenate([sel, child])
    # means
    p = np.concatenate([h["means"][sel], h["means"][sel]]).astype(np.float64)
    s = h["log_scales"][sel].astype(np.float64)
    a = prm.get("alpha", 0.5)
    off = a * np.exp(s.max(axis=1))
    off2 = np.concatenate([off, off])[:, None]
    d = np.abs(res["means"][rows].astype(np.float64) - ref["means"][rows])
    bound = 16 * U * (np.abs(p) + off2)
    assert (d <= bound).all(), f"means err {(d / np.maximum(bound, 1e-30)).max()} x bound"
    ds = np.abs(res["log_scales"][rows].astype(np.float64) - ref["log_scales"][rows])
    assert (ds <= 4 * U * np.maximum(1, np.abs(ref["log_scales"][rows]))).all(), ds.max()
    do = np.abs(res["opacity_logits"][rows].astype(np.float64) - ref["opacity_logits"][rows])
    assert (do <= 1e-6 * np.maximum(1, np.abs(ref["opacity_logits"][rows]))).all(), do.max()
    return ref


@pytest.mark.parametrize("name", ["view_256x192", "view_1297x840", "step_views300_las3m"])
def test_workloads(name):
    w = synth.workload(name)
    g = w.gaussian_set()
    mk = w.split_mask()
    N = w.n_gauss
    cap = N + w.n_split + 300                     # 300 canary rows past N + K
    res = run_las(g, N, mk, cap)
    ref = compare(res, N, cap)
    assert ref["K"] == w.n_split
    assert (res["means"][N + w.n_split:] == CANARY).all()


@pytest.mark.parametrize("N,frac,extra", [(0, 0.0, 5), (1, 1.0, 0), (2047, 1.0, 0), (2048, 0.5, 1),
                                          (2049, 0.0, 10), (5000, 0.3, 3), (8193, 0.5, 0), (60000, 0.05, 0),
                                          (64000, 0.024, 0), (64000, 0.024, 1), (70001, 0.01, 0)])
def test_sizes_and_densities(N, frac, extra):
    """Capacities up to 65536 rows take the one-launch split of one
    work-group (rounds of 8192 rows), larger ones the three launches; 64000
    rows with 1536 selected sit on either side of that line."""
    g = synth.gaussians(17, max(N, 1))
    K = int(round(frac * N))
    mk = synth.mask(18, max(N, 1), K)[:N]
    cap = N + K + extra
    compare(run_las(g, N, mk, cap), N, cap)


def test_capacity_overflow_writes_nothing():
    g = synth.gaussians(3, 4000)
    mk = synth.mask(4, 4000, 400)
    cap = 4000 + 399
    res = run_las(g, 4000, mk, cap)
    assert res["status"] == -6 and res["count"] == 4000 and res["K"] == 400
    compare(res, 4000, cap)
    ok = run_las(g, 4000, mk, 4400)             # exactly fills capacity
    assert ok["status"] == 0 and ok["count"] == 4400


def test_features_and_params():
    N, F = 3000, 48
    g = synth.gaussians(5, N)
    mk = synth.mask(6, N, 700)
    f = np.random.default_rng(0).normal(size=(N, F)).astype(np.float32)
    prm = dict(alpha=0.4, gamma=0.9, beta=0.75)
    res = run_las(g, N, mk, N + 700, feats=f, **prm)
    compare(res, N, N + 700, feats=f, **prm)


def test_special_rows():
    N = 6
    g = synth.gaussians(8, N)
    g.log_scales[0] = [-3, -3, -3]            # isotropic: axis 0
    g.log_scales[1] = [-5, -2, -2]            # tie between 1 and 2: axis 1
    g.quats[2] = [0, 0, 0, 0]                 # zero quaternion: identity
    g.quats[3] = [3, 0, 0, 4]                 # unnormalised
    g.opacity_logits[4] = -60.0               # deep negative logit
    g.log_scales[5] = [np.nan, -1, -2]        # NaN stays in its own row
    mk = np.ones(N, np.uint8)
    res = run_las(g, N, mk, 2 * N)
    assert res["status"] == 0 and res["count"] == 2 * N
    sub = [0, 1, 2, 3, 4]
    ref = oracle.las(N, res["host"]["means"], res["host"]["log_scales"], res["host"]["quats"],
                     res["host"]["opacity_logits"], mk)
    for i in sub:
        for row in (i, N + i):
            assert np.allclose(res["means"][row], ref["means"][row], atol=1e-6)
            assert abs(res["opacity_logits"][row] - ref["opacity_logits"][row]) <= 1e-6 * max(1, abs(ref["opacity_logits"][row]))
    assert np.isnan(res["log_scales"][5]).any() and np.isnan(res["log_scales"][N + 5]).any()
    assert np.isfinite(res["means"][:5]).all() and np.isfinite(res["means"][N:N + 5]).all()


def test_two_calls_grow_count_on_device():
    N = 1000
    g = synth.gaussians(9, N)
    mk = synth.mask(10, N, 100)
    res = run_las(g, N, mk, 1300, calls=2)
    # second call splits the same first-N selection again; the new rows are
    # not selected (mask zero past N), so count grows by K twice
    assert res["status"] == 0 and res["count"] == 1200
    assert res["K"] == 100
    h = res["host"]
    r1 = oracle.las(N, h["means"], h["log_scales"], h["quats"], h["opacity_logits"], mk)
    r2 = oracle.las(1100, r1["means"].astype(np.float32), r1["log_scales"].astype(np.float32),
                    r1["quats"].astype(np.float32), r1["opacity_logits"].astype(np.float32), mk)
    assert r2["count"] == 1200
    assert np.abs(res["means"][:1200] - r2["means"][:1200]).max() < 1e-5


def _run_full(g, N, mask, cap, F, seed, groups, over_capacity=False, misalign=False):
    """long_axis_split_full with F feature floats and random moments for the
    given groups; returns (result dict as run_las, moments before, after).
    misalign: every array starts 4 bytes past a 16-byte boundary."""
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    widths = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "features": F}
    feats = rng.normal(size=(N, F)).astype(np.float32)

    def padded(a, rows):
        out = np.full((rows,) + a.shape[1:], CANARY, np.float32)
        out[:min(rows, a.shape[0])] = a[:rows]
        return out

    host = {"means": padded(g.means, cap), "log_scales": padded(g.log_scales, cap),
            "quats": padded(g.quats, cap), "opacity_logits": padded(g.opacity_logits, cap),
            "features": padded(feats, cap)}
    def dev_array(a):
        if not misalign:
            return torch.from_numpy(a.copy()).to(dev)
        flat = torch.zeros(a.size + 1, dtype=torch.float32, device=dev)
        view = flat[1:].view(a.shape)
        view.copy_(torch.from_numpy(a))
        assert view.data_ptr() % 16 == 4
        return view

    t = {k: dev_array(v) for k, v in host.items()}
    mom_host = {grp: [rng.normal(size=(cap, widths[grp])).astype(np.float32).squeeze(-1 if widths[grp] == 1 else ())
                      for _ in range(2)] for grp in groups}
    mom = {grp: tuple(dev_array(a) for a in pair) for grp, pair in mom_host.items()}
    count = torch.tensor([N], dtype=torch.int64, device=dev)
    mk = np.zeros(cap, np.uint8)
    mk[:N] = mask[:N]
    tmask = torch.from_numpy(mk).to(dev)
    sidx = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    status = torch.full((1,), 99, dtype=torch.int32, device=dev)
    nsplit = torch.full((1,), -1, dtype=torch.int64, device=dev)
    igsp.long_axis_split_full(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], count, tmask, sidx,
                              status, mom, n_split=nsplit, features=t["features"])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in t.items()}
    res.update(count=int(count.item()), status=int(status.item()), K=int(nsplit.item()),
               split_idx=sidx.cpu().numpy(), host=host, mask=mk)
    after = {grp: [a.cpu().numpy() for a in pair] for grp, pair in mom.items()}
    return res, mom_host, after


@pytest.mark.parametrize("N,K,F,groups", [
    (3000, 700, 48, ("means", "log_scales", "quats", "opacity_logits", "features")),
    (70001, 9000, 48, ("means", "opacity_logits", "features")),
    (2049, 2049, 3, ("log_scales", "features")),
    (5000, 0, 48, ("means", "features")),
    (9000, 2500, 8, ("means", "log_scales", "quats", "opacity_logits", "features")),   # 32 rows per wave step
    (3000, 900, 260, ("quats", "features")),    # a row wider than a wavefront of 16-byte lanes
])
def test_full_record_split(N, K, F, groups):
    g = synth.gaussians(21, N)
    mk = synth.mask(22, N, K)
    cap = N + K + 77
    res, before, after = _run_full(g, N, mk, cap, F, 23, groups)
    ref = compare(res, N, cap, feats=res["host"]["features"])
    for grp in groups:
        for k in range(2):
            want = oracle.las_moments(N, ref["split_idx"], {"x": before[grp][k]})["x"]
            assert (after[grp][k] == want).all(), (grp, k)
    # canary rows past N + K keep the parameters' canary and their moments
    assert (res["features"][N + K:] == CANARY).all()


@pytest.mark.parametrize("N,K,F", [(6000, 1500, 48), (4100, 300, 8)])
def test_full_record_split_unaligned_arrays(N, K, F):
    """Arrays that do not start on a 16-byte boundary take the row-by-row
    paths (dense tiles and sparse tiles alike) with the same results."""
    groups = ("means", "log_scales", "quats", "opacity_logits", "features")
    g = synth.gaussians(27, N)
    mk = synth.mask(28, N, K)
    cap = N + K + 9
    res, before, after = _run_full(g, N, mk, cap, F, 29, groups, misalign=True)
    ref = compare(res, N, cap, feats=res["host"]["features"])
    for grp in groups:
        for k in range(2):
            want = oracle.las_moments(N, ref["split_idx"], {"x": before[grp][k]})["x"]
            assert (after[grp][k] == want).all(), (grp, k)


def test_full_record_split_capacity_overflow_touches_nothing():
    N, K, F = 4000, 400, 48
    g = synth.gaussians(24, N)
    mk = synth.mask(25, N, K)
    cap = N + K - 1
    res, before, after = _run_full(g, N, mk, cap, F, 26, ("means", "features"))
    assert res["status"] == -6 and res["count"] == N
    for grp in ("means", "features"):
        for k in range(2):
            assert (after[grp][k] == before[grp][k]).all()
    assert (res["features"] == res["host"]["features"]).all()
