"""Pins for the CPU oracle's edge-score pipeline (Sec. 2.1).

Each test ties the oracle to something outside itself: closed forms derived by
hand (tests/golden/edge_closed_forms.json), library routines (scipy's
convolution and Sobel filters, numpy's reflect padding, atan2), invariants of
the definition (rotation/mirror covariance, scale and offset invariance), and
a brute-force re-formulation of the suppression step written a different way
(angle-based direction table instead of exact integer bins).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "edge_closed_forms.json")


def flat(v, W=16, H=12):
    im = np.zeros((H, W, 3), np.uint8)
    im[:] = v
    return im


def rnd(seed, H, W, lo=0, hi=256):
    return np.random.default_rng(seed).integers(lo, hi, (H, W, 3), dtype=np.uint8)


# ---------------------------------------------------------------- taps / gray

def test_blur_taps_binomial_sum_to_one():
    w = oracle.blur_taps()
    assert w.tolist() == [1, 4, 6, 4, 1]          # binomial C(4, k)
    assert sum(Fraction(int(t), 16) for t in w) == 1   # normalised taps sum to exactly 1
    assert int(np.outer(w, w).sum()) == 256


def test_gray_channel_order_and_weights():
    o = oracle.edge_view(flat((255, 0, 0)))
    assert (o["gray"] == 299 * 255).all()
    o = oracle.edge_view(flat((0, 255, 0)))
    assert (o["gray"] == 587 * 255).all()
    o = oracle.edge_view(flat((0, 0, 255)))
    assert (o["gray"] == 114 * 255).all()
    o = oracle.edge_view(flat((77, 77, 77)))
    assert (o["gray"] == 77000).all()             # weights sum to 1 (x1000)


def test_blur_impulse_response_is_kernel():
    im = np.zeros((15, 17, 3), np.uint8)
    im[7, 8] = 10
    o = oracle.edge_view(im)
    w = oracle.blur_taps()
    ref = np.zeros((15, 17), np.int64)
    ref[5:10, 6:11] = np.outer(w, w) * 10000
    assert (o["b"] == ref).all()


@pytest.mark.parametrize("seed,H,W", [(0, 13, 17), (1, 3, 3), (2, 4, 9), (3, 31, 5)])
def test_blur_and_sobel_match_scipy_mirror(seed, H, W):
    # scipy's 'mirror' mode is reflect-101 (d c b | a b c d | c b a)
    im = rnd(seed, H, W)
    o = oracle.edge_view(im)
    i64 = im.astype(np.int64)
    gray = 299 * i64[..., 0] + 587 * i64[..., 1] + 114 * i64[..., 2]
    assert (o["gray"] == gray).all()
    w = oracle.blur_taps()
    b = ndi.convolve(gray, np.outer(w, w), mode="mirror")
    assert (o["b"] == b).all()
    assert (o["gx"] == ndi.sobel(b, axis=1, mode="mirror")).all()
    assert (o["gy"] == ndi.sobel(b, axis=0, mode="mirror")).all()
    assert (o["M"] == o["gx"] ** 2 + o["gy"] ** 2).all()


# ---------------------------------------------------------------- closed forms

def test_ramp_closed_form():
    g = json.load(open(GOLD))["ramp"]
    W, H = g["W"], g["H"]
    im = np.zeros((H, W, 3), np.uint8)
    im[:] = np.arange(W, dtype=np.uint8)[None, :, None]
    o = oracle.edge_view(im)
    for y in range(H):
        assert o["gx"][y].tolist() == g["gx_row"]
    assert (o["gy"] == 0).all()
    cols = sorted(set(np.nonzero(o["keep"])[1].tolist()))
    assert cols == g["survivor_columns"]
    assert (o["E"][o["keep"] > 0] == g["E_at_survivors"]).all()
    assert o["n"] == H


def test_diagonal_ramp_gradient():
    W, H = 24, 20
    im = np.zeros((H, W, 3), np.uint8)
    im[:] = (np.arange(W)[None, :] + np.arange(H)[:, None]).astype(np.uint8)[..., None]
    o = oracle.edge_view(im)
    inner = (slice(3, H - 3), slice(3, W - 3))
    assert (o["gx"][inner] == 8 * 256000).all() and (o["gy"][inner] == 8 * 256000).all()
    assert (o["bin"][inner] == 2).all()


@pytest.mark.parametrize("k,W,H", [(10, 20, 12), (5, 14, 7), (20, 40, 9)])
def test_step_edge_one_pixel_ridge(k, W, H):
    g = json.load(open(GOLD))["step"]
    im = np.zeros((H, W, 3), np.uint8)
    im[:, k:] = 255
    o = oracle.edge_view(im)
    if (k, W, H) == (g["k"], g["W"], g["H"]):
        for col, val in g["gx_over_64x255000"].items():
            assert (o["gx"][:, int(col)] == val * 64 * 255000).all()
        assert sorted(set(np.nonzero(o["keep"])[1].tolist())) == g["survivor_columns"]
    assert (o["keep"][:, k - 1] == 1).all()
    assert o["keep"].sum() == H            # exactly one pixel per row
    assert (o["E"][:, k - 1] == 1.0).all() and o["E"].sum() == H
    # bright-to-dark: the ridge moves to the dark side, column k
    o2 = oracle.edge_view(255 - im)
    assert (o2["keep"][:, k] == 1).all() and o2["keep"].sum() == H
    # a horizontal step (transpose) leaves row k-1
    o3 = oracle.edge_view(np.ascontiguousarray(im.transpose(1, 0, 2)))
    assert (o3["keep"][k - 1, :] == 1).all() and o3["keep"].sum() == H


def test_constant_image_is_zero():
    o = oracle.edge_view(flat((40, 120, 200), 23, 11))
    assert o["n"] == 0 and (o["E"] == 0).all() and (o["M"] == 0).all()


# ---------------------------------------------------------------- binning

def _atan2_bin(gx, gy):
    """Textbook Canny quantisation: angle mod 180 rounded to the nearest 45."""
    a = np.degrees(np.arctan2(gy, gx)) % 180.0
    q = np.round(a / 45.0).astype(int) % 4   # 0:0deg 1:45deg 2:90deg 3:135deg
    # 45 degrees with y down is gx, gy of the same sign
    return np.choose(q, [0, 2, 1, 3]), a


def test_bins_equal_atan2_rounding():
    rng = np.random.default_rng(0)
    for mag in (10, 1000, 2 ** 20, 2 ** 28):
        gx = rng.integers(-mag, mag + 1, 20000)
        gy = rng.integers(-mag, mag + 1, 20000)
        ok = (gx != 0) | (gy != 0)
        gx, gy = gx[ok], gy[ok]
        ref, ang = _atan2_bin(gx.astype(np.float64), gy.astype(np.float64))
        # skip the (measure-zero) cases float64 atan2 cannot place reliably
        far = np.abs(((ang - 22.5) % 45.0) - 22.5) < 22.5 - 1e-9
        got = np.array([oracle.bin_of(a, b) for a, b in zip(gx, gy)])
        assert (got[far] == ref[far]).all()


# ---------------------------------------------------------------- NMS brute force

def _nms_direction_table(gx, gy):
    """Suppression written another way: the full gradient angle is rounded to
    one of 8 compass directions, the step is read from a table, neighbours
    come from numpy's reflect padding, and the keep rule is applied."""
    H, W = gx.shape
    M = gx.astype(object) ** 2 + gy.astype(object) ** 2     # exact Python ints
    Mp = np.pad(M, 1, mode="reflect")
    ang = np.degrees(np.arctan2(gy.astype(np.float64), gx.astype(np.float64)))
    sector = np.round(ang / 45.0).astype(int) % 8
    table = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    keep = np.zeros((H, W), np.uint8)
    for y in range(H):
        for x in range(W):
            if M[y, x] == 0:
                continue
            dx, dy = table[sector[y, x]]
            lo = Mp[y + 1 - dy, x + 1 - dx]
            hi = Mp[y + 1 + dy, x + 1 + dx]
            keep[y, x] = 1 if (M[y, x] > lo and M[y, x] >= hi) else 0
    return keep


@pytest.mark.parametrize("case", ["noise", "checker", "lines", "scene", "tiny", "ties"])
def test_nms_matches_direction_table(case):
    if case == "noise":
        im = rnd(3, 24, 31)
    elif case == "checker":
        yy, xx = np.mgrid[0:16, 0:18]
        im = np.repeat((((yy // 2 + xx // 3) % 2) * 200 + 20).astype(np.uint8)[..., None], 3, 2)
    elif case == "lines":
        im = np.zeros((17, 19, 3), np.uint8)
        im[:, 5] = 255
        im[9, :] = 128
        im[np.arange(17), np.arange(17)] = 60
    elif case == "scene":
        im = synth.image(99, 48, 40, 8, True)
    elif case == "tiny":
        im = rnd(8, 3, 4)
    else:
        im = rnd(9, 12, 12, 100, 103)      # low-contrast noise: many near-equal magnitudes
    o = oracle.edge_view(im)
    ref = _nms_direction_table(o["gx"], o["gy"])
    assert (o["keep"] == ref).all()


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", [0, 1])
def test_rotation_and_mirror_covariance(seed):
    im = synth.image(1000 + seed, 37, 29, 6, True)
    o = oracle.edge_view(im)
    for k in (1, 2, 3):
        r = oracle.edge_view(np.ascontiguousarray(np.rot90(im, k)))
        assert (r["keep"] == np.rot90(o["keep"], k)).all()
        assert (r["E"] == np.rot90(o["E"], k)).all()
        assert (r["M"] == np.rot90(o["M"], k)).all()
    for ax in (0, 1):
        r = oracle.edge_view(np.ascontiguousarray(np.flip(im, ax)))
        assert (r["keep"] == np.flip(o["keep"], ax)).all()
        assert (r["E"] == np.flip(o["E"], ax)).all()


def test_scale_and_offset_invariance():
    im = (synth.image(5, 40, 30, 8, True) // 2).astype(np.uint8)   # values <= 127
    o = oracle.edge_view(im)
    o2 = oracle.edge_view((im * 2).astype(np.uint8))
    assert (o2["keep"] == o["keep"]).all() and (o2["E"] == o["E"]).all()
    o3 = oracle.edge_view((im + 100).astype(np.uint8))                # no clipping
    assert (o3["keep"] == o["keep"]).all() and (o3["E"] == o["E"]).all()


# ---------------------------------------------------------------- median

@pytest.mark.parametrize("seed,H,W", [(0, 40, 50), (1, 7, 9), (2, 64, 64)])
def test_median_is_lower_median_of_survivors(seed, H, W):
    im = synth.image(seed, W, H, 5, True)
    o = oracle.edge_view(im)
    n = o["n"]
    vals = o["m"][o["keep"] > 0]
    assert vals.size == n and n > 0
    k = (n - 1) // 2
    assert o["med"] == np.partition(vals, k)[k]
    E = o["E"][o["keep"] > 0]
    assert (E < 1).sum() <= k < (E <= 1).sum()
    assert (E == 1.0).any()
    assert (o["E"][o["keep"] == 0] == 0).all()


def test_batch_equals_single_views_any_threads():
    w = synth.workload("views200_w1000_1560")
    vb = w.render(views=[0, 1], in_align=1, out_align=1)
    # shrink to keep the test fast: crop two small views
    imgs = [vb.view(0)[:60, :81], vb.view(1)[:33, :47]]
    pb = synth.pack_views(imgs, in_align=3, out_align=5)
    for t in (1, 2):
        r = oracle.edge_batch(pb.rgb, pb.widths, pb.heights, pb.in_offset, pb.out_offset,
                              pb.out_floats, threads=t)
        for v, im in enumerate(imgs):
            o = oracle.edge_view(im)
            H, W = im.shape[:2]
            got = r["E"][int(pb.out_offset[v]):int(pb.out_offset[v]) + W * H].reshape(H, W)
            assert (got == o["E"]).all() and r["n"][v] == o["n"] and r["med"][v] == o["med"]


def test_rejects_views_below_3x3():
    with pytest.raises(ValueError):
        oracle.edge_view(np.zeros((2, 5, 3), np.uint8))


# ---------------------------------------------------------------- exact brute force, whole pipeline

def _brute_refl(i, n):
    """Reflect-101 by repeated mirroring about the border pixels."""
    while i < 0 or i >= n:
        i = -i if i < 0 else 2 * (n - 1) - i
    return i


def _brute_gradients(im):
    """Gray, the 5x5 blur as one 25-term sum and the Sobel pair, in plain
    Python integers with explicit reflect-101. Returns (gx, gy) as lists."""
    H, W = im.shape[:2]
    refl = _brute_refl
    g = [[299 * int(im[y, x, 0]) + 587 * int(im[y, x, 1]) + 114 * int(im[y, x, 2]) for x in range(W)]
         for y in range(H)]
    w = [1, 4, 6, 4, 1]
    b = [[sum(w[j] * w[k] * g[refl(y + j - 2, H)][refl(x + k - 2, W)] for j in range(5) for k in range(5))
          for x in range(W)] for y in range(H)]

    def B(y, x):
        return b[refl(y, H)][refl(x, W)]

    gx = [[sum(c * (B(y + dy, x + 1) - B(y + dy, x - 1)) for dy, c in ((-1, 1), (0, 2), (1, 1))) for x in range(W)]
          for y in range(H)]
    gy = [[sum(c * (B(y + 1, x + dx) - B(y - 1, x + dx)) for dx, c in ((-1, 1), (0, 2), (1, 1))) for x in range(W)]
          for y in range(H)]
    return gx, gy


def _brute_pipeline(im):
    """Every step of Sec. 2.1 in plain Python integers on a small image, with
    formulations that differ from the oracle's: explicit reflect-101 by
    repeated mirroring, the 5x5 blur as one 25-term sum, the orientation from
    the exact comparison (|gx| + |gy|)^2 vs 2 g^2, the median by sorting.
    Returns (keep, M, M of the median survivor or None)."""
    H, W = im.shape[:2]
    refl = _brute_refl
    gx, gy = _brute_gradients(im)
    M = [[gx[y][x] ** 2 + gy[y][x] ** 2 for x in range(W)] for y in range(H)]

    def sgn(v):
        return (v > 0) - (v < 0)

    keep = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            a, c = gx[y][x], gy[y][x]
            s = (abs(a) + abs(c)) ** 2
            if s < 2 * a * a:
                d = (sgn(a), 0)
            elif s < 2 * c * c:
                d = (0, sgn(c))
            else:
                d = (sgn(a), sgn(c))
            m = M[y][x]
            lo = M[refl(y - d[1], H)][refl(x - d[0], W)]
            hi = M[refl(y + d[1], H)][refl(x + d[0], W)]
            keep[y][x] = int(m > 0 and m > lo and m >= hi)
    surv = sorted(M[y][x] for y in range(H) for x in range(W) if keep[y][x])
    mmed = surv[(len(surv) - 1) // 2] if surv else None
    return np.array(keep, np.uint8), np.array(M, dtype=object), mmed


def _tiny_images():
    rng = np.random.default_rng(17)
    out = [rng.integers(0, 256, (8, 8, 3), dtype=np.uint8) for _ in range(12)]
    out += [rng.integers(120, 124, (8, 8, 3), dtype=np.uint8) for _ in range(4)]     # many ties
    yy, xx = np.mgrid[0:8, 0:8]
    out.append(np.repeat(((xx + yy) % 2 * 255).astype(np.uint8)[..., None], 3, 2))  # checkerboard
    st = np.zeros((8, 8, 3), np.uint8)
    st[:, 4:] = 200
    out.append(st)                                                                    # step
    out.append(np.repeat((xx * 30).astype(np.uint8)[..., None], 3, 2))               # ramp
    out.append(rng.integers(0, 256, (3, 5, 3), dtype=np.uint8))                      # smallest views
    out.append(rng.integers(0, 256, (5, 3, 3), dtype=np.uint8))
    return out


@pytest.mark.parametrize("k", range(21))
def test_whole_pipeline_against_exact_brute_force(k):
    im = _tiny_images()[k]
    keep, M, mmed = _brute_pipeline(im)
    o = oracle.edge_view(im)
    assert (o["M"] == M.astype(np.int64)).all()
    assert (o["keep"] == keep).all()
    assert o["n"] == int(keep.sum())
    if mmed is None:
        assert (o["E"] == 0).all()
        return
    # the median survivor's magnitude, exactly; in DN of an unnormalised Sobel: sqrt(M_med) / 256000
    assert int(o["Mmed"]) == mmed
    assert o["med"] == pytest.approx(math.sqrt(mmed) / 256000.0, rel=1e-15)
    # the map squared is M / M_med exactly (up to the FP64 root and division)
    for y, x in zip(*np.nonzero(keep)):
        want = Fraction(int(M[y, x]), mmed)
        assert o["E"][y, x] ** 2 == pytest.approx(float(want), rel=4e-16 * 8)
    assert (o["E"][keep == 0] == 0).all()
