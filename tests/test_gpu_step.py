"""The densification step recorded as a HIP graph (edge maps then
Long-Axis-Split in one graph launch).

Every replay is checked against the oracle -- maps view by view
(parity.compare_view) and the Gaussians, split indices, count and status
(test_gpu_las.compare) -- and against the eager sequence bit for bit, with
eager work and synchronisation between the replays. One test builds the step
exactly as the benchmark does for its default workload (300 views, BF16,
3M Gaussians) and checks a replay of that graph against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_view, view_map
from test_gpu_las import compare

pytestmark = pytest.mark.gpu


def _setup(precision):
    import torch

    dev = torch.device("cuda:0")
    imgs = [synth.image(70 + k, w, h, 10, True) for k, (w, h) in enumerate([(300, 200), (517, 133), (64, 61)])]
    vb = synth.pack_views(imgs, in_align=16, out_align=4)
    img = torch.from_numpy(np.concatenate([vb.rgb, np.zeros(32, np.uint8)])).to(dev)
    N, K = 20000, 4000
    g = synth.gaussians(71, N, -4.5, 0.7)
    cap = N + K + 64
    mk = np.zeros(cap, np.uint8)
    mk[:N] = synth.mask(72, N, K)
    host = {}
    for k in ("means", "log_scales", "quats", "opacity_logits"):
        a = getattr(g, k)
        host[k] = np.zeros((cap,) + a.shape[1:], np.float32)
        host[k][:N] = a

    def fresh():
        t = {k: torch.from_numpy(v.copy()).to(dev) for k, v in host.items()}
        t["count"] = torch.tensor([N], dtype=torch.int64, device=dev)
        return t

    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    return vb, img, views, fresh, torch.from_numpy(mk).to(dev), cap, host, mk, N


def _las_result(gt, sidx, status, nsplit, host, mk):
    res = {k: gt[k].cpu().numpy() for k in host}
    res.update(count=int(gt["count"].item()), status=int(status.item()), K=int(nsplit.item()),
               split_idx=sidx.cpu().numpy(), host=host, mask=mk)
    return res


@pytest.mark.parametrize("precision,form", [("bf16", "persistent"), ("fp32", "persistent"), ("bf16", "staged"),
                                            ("fp16", "persistent"), ("fp16", "staged"), ("fp32", "staged")])
def test_graph_replays_match_oracle_and_eager(precision, form):
    import torch

    import paper_2603_08661_amd as igsp

    vb, img, views, fresh, mask, cap, host, mk, N = _setup(precision)
    dev = img.device
    refs = [oracle.edge_view(vb.view(v)) for v in range(vb.n)]
    # eager reference
    ga = fresh()
    out_a = torch.zeros(vb.out_floats, dtype=torch.float32, device=dev)
    sidx_a = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    st_a = torch.zeros(1, dtype=torch.int32, device=dev)
    igsp.edge_importance(img, views, out_a, precision=precision, batched="staged")
    igsp.long_axis_split(ga["means"], ga["log_scales"], ga["quats"], ga["opacity_logits"], ga["count"], mask,
                         sidx_a, st_a)
    torch.cuda.synchronize()

    gb = fresh()
    pristine = {k: v.clone() for k, v in gb.items()}
    out_b = torch.zeros(vb.out_floats, dtype=torch.float32, device=dev)
    sidx_b = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    st_b = torch.zeros(1, dtype=torch.int32, device=dev)
    ns_b = torch.full((1,), -1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream()
    step = igsp.Step(img, views, out_b, gb, mask, sidx_b, st_b, n_split=ns_b, precision=precision, batched=form,
                     stream=stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            for k in gb:
                gb[k].copy_(pristine[k])
            out_b.zero_()
            sidx_b.fill_(-1)
            step.launch(stream)
        stream.synchronize()
        _ = (torch.arange(1000, device=dev) * 2).sum().item()    # eager work between replays
        torch.cuda.synchronize()
        # against the oracle
        E = out_b.cpu().numpy()
        for v in range(vb.n):
            compare_view(view_map(E, vb, v), refs[v], precision)
        ref = compare(_las_result(gb, sidx_b, st_b, ns_b, host, mk), N, cap)
        assert ref["K"] == 4000
        # and against the eager sequence, bit for bit
        assert torch.equal(out_a, out_b), rep
        assert torch.equal(sidx_a, sidx_b) and torch.equal(st_a, st_b)
        for k in ga:
            assert torch.equal(ga[k], gb[k]), (rep, k)
    assert int(gb["count"].item()) == N + 4000
    step.close()


def test_graph_step_of_the_benchmark_workload():
    """The graph the benchmark times: its default workload (300 views of
    widths 1000-2473, BF16 storage, the tuned form and tile; LAS on 3M
    Gaussians with 20% selected), built through the same calls. One replay;
    sampled views checked pixel by pixel and the whole split against the
    oracle."""
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    w = synth.workload("step_views300_las3m")
    prec = w.precision
    vb = w.render()
    print(f"rendered {vb.n} views, {vb.pixels / 1e6:.1f} MPx", flush=True)
    img = torch.from_numpy(np.concatenate([vb.rgb, np.zeros(16, np.uint8)])).to(dev)
    out = torch.zeros(vb.out_floats, dtype=torch.float32, device=dev)
    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    g = w.gaussian_set()
    mk = w.split_mask()
    N, K = w.n_gauss, w.n_split
    cap = N + K + 300
    host = {}
    G = {}
    for k in ("means", "log_scales", "quats", "opacity_logits"):
        a = getattr(g, k)
        host[k] = np.full((cap,) + a.shape[1:], 12345.0, np.float32)
        host[k][:N] = a
        G[k] = torch.from_numpy(host[k]).to(dev)
    G["count"] = torch.tensor([N], dtype=torch.int64, device=dev)
    mkc = np.zeros(cap, np.uint8)
    mkc[:N] = mk
    mask = torch.from_numpy(mkc).to(dev)
    sidx = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    nsplit = torch.full((1,), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    bform, seg, wgw = igsp.edge_resolve(views, prec, "batched", 0, 0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        step = igsp.Step(img, views, out, G, mask, sidx, status, n_split=nsplit, precision=prec, batched=bform,
                         seg_rows=seg, wg_waves=wgw, stream=stream)
    step.launch(stream)
    stream.synchronize()
    print(f"replayed: form {bform}, tile {seg}x{wgw}", flush=True)
    E = out.cpu().numpy()
    area = vb.widths.astype(np.int64) * vb.heights
    sample = sorted({0, 1, int(np.argmax(area)), int(np.argmin(area)), vb.n // 2, vb.n - 2, vb.n - 1})
    for v in sample:
        st = compare_view(view_map(E, vb, v), oracle.edge_view(vb.view(v)), prec)
        print(f"view {v} ({vb.widths[v]}x{vb.heights[v]}): {st}", flush=True)
    res = _las_result(G, sidx, status, nsplit, host, mkc)
    ref = compare(res, N, cap)
    assert ref["K"] == K and res["count"] == N + K
    assert (res["means"][N + K:] == 12345.0).all()        # canary rows past N + K
    step.close()
