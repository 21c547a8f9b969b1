"""Pins for the CPU oracle's Long-Axis-Split (Sec. 2.2, Algorithms 1 and 2).

Hand-derived worked examples (tests/golden/las_examples.json), a library
routine for the quaternion-to-matrix step (scipy's Rotation), the defining
property of the opacity update, and geometric invariants of the split.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "las_examples.json")
A, G, B = oracle.ALPHA, oracle.GAMMA, oracle.BETA


def one_row(case):
    return (np.array([case["mean"]], np.float32), np.array([case["log_scale"]], np.float32),
            np.array([case["quat_wxyz"]], np.float32), np.array([case["opacity_logit"]], np.float32))


@pytest.mark.parametrize("ci", [0, 1, 2])
def test_golden_examples(ci):
    case = json.load(open(GOLD))["cases"][ci]
    m, s, q, o = one_row(case)
    cap = 2
    pad = lambda a: np.concatenate([a, np.zeros_like(a)])  # noqa: E731
    r = oracle.las(1, pad(m), pad(s), pad(q), pad(o), np.array([1], np.uint8))
    assert r["status"] == 0 and r["K"] == 1 and r["count"] == cap
    assert r["axis"].tolist() == [case["axis"]] and r["split_idx"].tolist() == [0]
    # inputs are rounded to float32 first, so compare at float32 input precision
    tol = 1e-6
    assert np.allclose(r["means"][0], case["child_a_mean"], atol=tol)
    assert np.allclose(r["means"][1], case["child_b_mean"], atol=tol)
    assert np.allclose(r["log_scales"][0], case["log_scale_new"], atol=tol)
    assert np.allclose(r["log_scales"][1], case["log_scale_new"], atol=tol)
    assert abs(r["opacity_logits"][0] - case["opacity_logit_new"]) < tol
    assert (r["quats"][1] == q[0]).all()


def test_constants_are_the_papers():
    assert (A, G, B) == (0.5, 0.85, 0.6)


def test_quat_to_R_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(200):
        q = rng.normal(size=4)
        R = oracle.quat_to_R(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy: (x, y, z, w)
        assert np.abs(R - ref).max() < 1e-14
    assert (oracle.quat_to_R([0, 0, 0, 0]) == np.eye(3)).all()


def test_opacity_update_defining_property():
    sig = lambda x: 1.0 / (1.0 + math.exp(-x))  # noqa: E731
    for o in np.linspace(-30, 30, 121):
        on = oracle.opacity_update(o, B)
        assert abs(sig(on) - B * sig(o)) <= 1e-15 + 1e-13 * B * sig(o)
    # where the literal logit(beta*sigmoid(o)) is well conditioned, it agrees
    for o in np.linspace(-5, 5, 41):
        p = B * sig(o)
        assert abs(oracle.opacity_update(o, B) - math.log(p / (1 - p))) < 1e-13
    # deep negative logits stay finite (sigmoid underflows in the literal form)
    assert math.isfinite(oracle.opacity_update(-200.0, B))
    assert abs(oracle.opacity_update(-200.0, B) - (-200.0 + math.log(B))) < 1e-12


def _scene(N, cap, frac, seed=3, mu=-4.0, sd=0.5):
    g = synth.gaussians(seed, cap, mu, sd)
    mk = synth.mask(seed + 1, N, int(round(frac * N)))
    return g, mk


@pytest.mark.parametrize("N,frac", [(2000, 0.1), (500, 1.0), (300, 0.0)])
def test_split_invariants(N, frac):
    K = int(round(frac * N))
    g, mk = _scene(N, N + K, frac)
    r = oracle.las(N, g.means, g.log_scales, g.quats, g.opacity_logits, mk)
    assert r["status"] == 0 and r["K"] == K and r["count"] == N + K
    sel = np.nonzero(mk)[0]
    assert r["split_idx"].tolist() == sel.tolist()                # ascending, = mask's nonzeros
    unsel = np.setdiff1d(np.arange(N), sel)
    assert (r["means"][unsel] == g.means[unsel]).all()            # untouched rows bit-exact
    assert (r["log_scales"][unsel] == g.log_scales[unsel]).all()
    assert (r["opacity_logits"][unsel] == g.opacity_logits[unsel]).all()
    for rr, i in enumerate(sel):
        j = N + rr
        p = g.means[i].astype(np.float64)
        s = g.log_scales[i].astype(np.float64)
        l = int(np.argmax(s))
        assert r["axis"][rr] == l
        ca, cb = r["means"][i], r["means"][j]
        assert np.abs((ca + cb) / 2 - p).max() < 1e-15
        assert abs(np.linalg.norm(ca - cb) - 2 * A * math.exp(s[l])) < 1e-14
        Rm = Rotation.from_quat(np.r_[g.quats[i, 1:], g.quats[i, 0]].astype(np.float64)).as_matrix()
        for jx in range(3):
            if jx != l:
                assert abs(np.dot(ca - p, Rm[:, jx])) < 1e-14
        ds = r["log_scales"][i] - s
        exp_ds = np.where(np.arange(3) == l, math.log(A), math.log(G))
        assert np.abs(ds - exp_ds).max() < 1e-14
        assert (r["log_scales"][j] == r["log_scales"][i]).all()
        assert (r["quats"][j] == g.quats[i]).all() and (r["quats"][i] == g.quats[i]).all()
        sig = lambda x: 1 / (1 + math.exp(-x))  # noqa: E731
        assert abs(sig(r["opacity_logits"][i]) - B * sig(float(g.opacity_logits[i]))) < 1e-15


def test_ties_take_lowest_axis_and_zero_quat_is_identity():
    cap = 4
    m = np.zeros((cap, 3), np.float32)
    s = np.array([[-3, -3, -3], [-5, -2, -2], [0, 0, 0], [0, 0, 0]], np.float32)
    q = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]], np.float32)
    o = np.zeros(cap, np.float32)
    r = oracle.las(2, m, s, q, o, np.array([1, 1], np.uint8))
    assert r["axis"].tolist() == [0, 1]
    assert np.allclose(r["means"][0], [A * math.exp(-3), 0, 0])       # identity used
    assert np.allclose(r["means"][1], [0, A * math.exp(-2), 0])


def test_capacity_overflow_is_all_or_nothing():
    N = 100
    g, mk = _scene(N, N + 5, 0.1)          # K = 10 > 5 free rows
    r = oracle.las(N, g.means, g.log_scales, g.quats, g.opacity_logits, mk)
    assert r["status"] == -6 and r["count"] == N and r["split_idx"].size == 0
    assert (r["means"] == g.means).all() and (r["log_scales"] == g.log_scales).all()


def test_global_rotation_covariance():
    N = 200
    g, mk = _scene(N, N + 20, 0.1, seed=9)
    r = oracle.las(N, g.means, g.log_scales, g.quats, g.opacity_logits, mk)
    Q = Rotation.from_euler("xyz", [0.3, -1.1, 2.0])
    qQ = Q.as_quat()                                   # (x, y, z, w)
    rq = (Q * Rotation.from_quat(np.c_[g.quats[:, 1:], g.quats[:, :1]])).as_quat()
    quats2 = np.c_[rq[:, 3:], rq[:, :3]].astype(np.float32)
    means2 = Q.apply(g.means.astype(np.float64)).astype(np.float32)
    r2 = oracle.las(N, means2, g.log_scales, quats2, g.opacity_logits, mk)
    sel = np.nonzero(mk)[0]
    for rr, i in enumerate(sel):
        for row in (i, N + rr):
            # children of the rotated scene are the rotated children (up to float32 input rounding)
            diff = r2["means"][row] - Q.apply(r["means"][row])
            assert np.abs(diff).max() < 1e-6
    assert qQ.shape == (4,)


def test_features_copied():
    N, F = 50, 6
    g, mk = _scene(N, N + 5, 0.1)
    f = np.random.default_rng(0).normal(size=(N + 5, F)).astype(np.float32)
    r = oracle.las(N, g.means, g.log_scales, g.quats, g.opacity_logits, mk, feats=f)
    for rr, i in enumerate(np.nonzero(mk)[0]):
        assert (r["feats"][N + rr] == f[i]).all() and (r["feats"][i] == f[i]).all()


def test_capacity_boundary_exact():
    N = 100
    g, mk = _scene(N, N + 10, 0.1)          # K = 10
    ok = oracle.las(N, g.means, g.log_scales, g.quats, g.opacity_logits, mk)
    assert ok["status"] == 0 and ok["count"] == N + 10        # exactly fills capacity
    short = oracle.las(N, g.means[:N + 9], g.log_scales[:N + 9], g.quats[:N + 9],
                       g.opacity_logits[:N + 9], mk)
    assert short["status"] == -6 and short["count"] == N      # one row short: nothing split


def test_moments_reading_worked_example():
    """Hand-worked: N = 4, rows 0 and 2 selected, capacity 7. Rows 0, 2 (the
    first children) and 4, 5 (the second children) are cleared; rows 1, 3
    (not split) and 6 (past N + K) keep their values."""
    m = np.arange(1.0, 22.0).reshape(7, 3)
    out = oracle.las_moments(4, [0, 2], {"m": m})["m"]
    expect = m.copy()
    expect[[0, 2, 4, 5]] = 0.0
    assert (out == expect).all()
    assert (out[[1, 3, 6]] == [[4, 5, 6], [10, 11, 12], [19, 20, 21]]).all()
    assert (m == np.arange(1.0, 22.0).reshape(7, 3)).all()   # input untouched
