"""The densification step recorded as a HIP graph: every replay equals the
eager sequence bit for bit (same kernels, same inputs), with eager work and
synchronisation between the replays."""
import numpy as np
import pytest

import synth

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

    def fresh():
        def pad(a):
            out = np.zeros((cap,) + a.shape[1:], np.float32)
            out[:N] = a
            return torch.from_numpy(out).to(dev)
        return {"means": pad(g.means), "log_scales": pad(g.log_scales), "quats": pad(g.quats),
                "opacity_logits": pad(g.opacity_logits),
                "count": torch.tensor([N], dtype=torch.int64, device=dev)}

    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    return vb, img, views, fresh, torch.from_numpy(mk).to(dev), cap


@pytest.mark.parametrize("precision,form", [("bf16", "persistent"), ("fp32", "persistent"), ("bf16", "staged"),
                                            ("fp16", "persistent")])
def test_graph_replays_equal_eager(precision, form):
    import torch

    import paper_2603_08661_amd as igsp

    vb, img, views, fresh, mask, cap = _setup(precision)
    dev = img.device
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
    stream = torch.cuda.Stream()
    step = igsp.Step(img, views, out_b, gb, mask, sidx_b, st_b, precision=precision, batched=form, stream=stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            for k in gb:
                gb[k].copy_(pristine[k])
            out_b.zero_()
            step.launch(stream)
        stream.synchronize()
        _ = (torch.arange(1000, device=dev) * 2).sum().item()    # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out_a, out_b), rep
        assert torch.equal(sidx_a, sidx_b) and torch.equal(st_a, st_b)
        for k in ga:
            assert torch.equal(ga[k], gb[k]), (rep, k)
    assert int(gb["count"].item()) == 20000 + 4000
    step.close()
