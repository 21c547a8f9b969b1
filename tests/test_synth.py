"""Seeded input generator: determinism, sizes, value ranges, exact mask counts."""
import numpy as np
import pytest

import synth


def test_image_deterministic_and_in_range():
    a = synth.image(1000003, 256, 192, 12)
    b = synth.image(1000003, 256, 192, 12)
    c = synth.image(1000004, 256, 192, 12)
    assert a.shape == (192, 256, 3) and a.dtype == np.uint8
    assert (a == b).all()
    assert (a != c).mean() > 0.5
    # scene-like: full dynamic range used, not constant
    assert a.std() > 20


def test_noise_statistics():
    # a flat colour region inside a view has per-channel std close to sigma
    im = synth.image(7, 200, 150, n_poly=0, noise_sigma=5.0).astype(np.float64)
    # background gradient is smooth: remove it with a 2nd difference along x
    d = im[:, 2:, :] - 2 * im[:, 1:-1, :] + im[:, :-2, :]
    est = d.std() / np.sqrt(6.0)  # var of 2nd difference of iid noise = 6 sigma^2
    assert 4.5 < est < 5.5


def test_batch_matches_single_and_offsets():
    w = synth.workload("views200_w1000_1560")
    vb = w.render(views=[0, 1, 2])
    for k, v in enumerate([0, 1, 2]):
        ref = synth.image(int(w.seeds[v]), int(w.full_w[v]), int(w.full_h[v]), w.n_poly, w.texture)
        assert (vb.view(k) == ref).all()
    assert (vb.in_offset % 256 == 0).all()


def test_down2_sizes():
    w = synth.workload("views150_2473x1643_mixed")
    Wd, Hd = w.sizes()
    assert set(zip(Wd.tolist(), Hd.tolist())) == {(2473, 1643), (1236, 821)}
    assert int((w.down2 != 0).sum()) == 75


def test_view_size_ranges():
    w = synth.workload("views200_w1000_1560")
    W, H = w.sizes()
    assert W.min() >= 1000 and W.max() <= 1560
    asp = W / H
    assert asp.min() > 1.49 and asp.max() < 1.78
    w5 = synth.workload("step_views300_las3m")
    W5, _ = w5.sizes()
    assert W5.min() >= 1000 and W5.max() <= 2473 and w5.n_views == 300


@pytest.mark.parametrize("N,K", [(10_000, 1_000), (1000, 0), (1000, 1000), (37, 5)])
def test_mask_exact_count(N, K):
    m = synth.mask(11, N, K)
    assert m.dtype == np.uint8 and int(m.sum()) == K and set(np.unique(m)) <= {0, 1}
    assert (m == synth.mask(11, N, K)).all()


def test_gaussian_distributions():
    g = synth.gaussians(5, 200_000, -4.5, 0.7)
    assert abs(g.log_scales.mean() + 4.5) < 0.01 and abs(g.log_scales.std() - 0.7) < 0.01
    assert np.abs(np.linalg.norm(g.quats, axis=1) - 1).max() < 1e-6
    assert np.abs(g.means).max() <= 1.0
    u = 1 / (1 + np.exp(-g.opacity_logits.astype(np.float64)))
    assert abs(u.mean() - 0.5) < 0.01
    g2 = synth.gaussians(5, 200_000, -4.5, 0.7)
    assert (g.quats == g2.quats).all()
