"""Pins for the oracle's suppression decision margin c(p) (Sec. 2.1 step 3).

The GPU decides suppression in FP32 on exact integer gradients, so its
decisions can differ from the exact ones only near a tie. The parity tests
forgive a decision mismatch where the oracle's margin

    c(p) = min(|sqrt M(p) - sqrt M(p - d)|, |sqrt M(p) - sqrt M(p + d)|,
               ||gy| - t |gx||, ||gx| - t |gy||) / sqrt M(p),   t = sqrt 2 - 1

(+inf where M(p) = 0) is below a small epsilon, so a wrong margin would widen
or narrow those exemptions without any other test noticing. It is pinned here
three ways, none of which reuses the oracle's code:

  * recomputed from exact Python-integer gradients (the brute-force gradients
    of the whole-pipeline test, or the oracle's gradients, which scipy pins)
    with 60-digit decimal square roots and t = sqrt 2 - 1, to 1e-12 relative;
  * closed forms worked by hand: the blurred step (its two central pixels tie,
    c = 0; the pixels beside them are limited by the angle term, c = t), the
    diagonal ramp (flat magnitude, c = 0), and small gradient fields whose
    margin is a known angle term ((5 sqrt 2 - 7) / sqrt 29), a known neighbour
    term along an axis (1/10) and along a diagonal (1 - 2 sqrt 2 / 3);
  * soundness: the margin means what the exemption assumes -- moving every
    input of a pixel's decision (the gradient pair, and the three magnitudes'
    roots) by less than the stated fraction of c(p) sqrt M(p) never changes
    the decision.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import synth
from test_oracle_edge import _brute_gradients, _brute_refl, _tiny_images

getcontext().prec = 60
T_EXACT = Decimal(2).sqrt() - 1
T = math.sqrt(2.0) - 1.0


def _sgn(v):
    return int(v > 0) - int(v < 0)


def _exact_margin(gx, gy):
    """c(p) from exact integer gradients (lists or int64 arrays), every root
    and the constant t to 60 significant digits; the orientation from the
    same decimal t (|gy| < t |gx|: horizontal, |gx| < t |gy|: vertical, else
    diagonal)."""
    H, W = len(gx), len(gx[0])
    G = [[(int(gx[y][x]), int(gy[y][x])) for x in range(W)] for y in range(H)]
    M = [[a * a + c * c for a, c in row] for row in G]
    out = np.full((H, W), np.inf)
    for y in range(H):
        for x in range(W):
            m = M[y][x]
            if m == 0:
                continue
            sx, sy = G[y][x]
            a, c = abs(sx), abs(sy)
            if c < T_EXACT * a:
                dx, dy = _sgn(sx), 0
            elif a < T_EXACT * c:
                dx, dy = 0, _sgn(sy)
            else:
                dx, dy = _sgn(sx), _sgn(sy)
            lo = M[_brute_refl(y - dy, H)][_brute_refl(x - dx, W)]
            hi = M[_brute_refl(y + dy, H)][_brute_refl(x + dx, W)]
            r = Decimal(m).sqrt()
            terms = (abs(r - Decimal(lo).sqrt()), abs(r - Decimal(hi).sqrt()),
                     abs(c - T_EXACT * a), abs(a - T_EXACT * c))
            out[y, x] = float(min(terms) / r)
    return out


def _assert_margin_equal(got, want):
    inf = np.isinf(want)
    assert (np.isinf(got) == inf).all()
    # FP64 roots of values below 2^57 and the differences of two of them:
    # absolute error a few 2^-53 after the division by sqrt M(p)
    err = np.abs(got[~inf] - want[~inf])
    assert (err <= 1e-12 * want[~inf] + 2e-15).all(), float(err.max())


# ---------------------------------------------------------------- exact recomputation

@pytest.mark.parametrize("k", range(21))
def test_margin_equals_exact_recomputation_on_tiny_images(k):
    im = _tiny_images()[k]
    gx, gy = _brute_gradients(im)
    o = oracle.edge_view(im)
    _assert_margin_equal(o["margin"], _exact_margin(gx, gy))


@pytest.mark.parametrize("seed,W,H", [(31, 48, 40), (32, 37, 29)])
def test_margin_equals_exact_recomputation_on_scenes(seed, W, H):
    o = oracle.edge_view(synth.image(seed, W, H, 8, True))
    want = _exact_margin(o["gx"], o["gy"])
    _assert_margin_equal(o["margin"], want)
    assert (want == 0).any() or (want < 1e-2).any()   # the cases that matter do occur


def test_margin_on_random_gradient_fields():
    rng = np.random.default_rng(5)
    for mag in (3, 1000, 2 ** 27):
        gx = rng.integers(-mag, mag + 1, (9, 11))
        gy = rng.integers(-mag, mag + 1, (9, 11))
        _assert_margin_equal(oracle.nms(gx, gy)["margin"], _exact_margin(gx, gy))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k,W,H", [(10, 20, 12), (5, 14, 7)])
def test_margin_of_blurred_step(k, W, H):
    # gx at columns k-3 .. k+2 is 1, 5, 10, 10, 5, 1 (x 64 x 255000), gy = 0:
    # the pixels at k-1 and k tie (c = 0); at k-3, k-2, k+1, k+2 the angle
    # term ||gy| - t|gx|| / |gx| = t is below every neighbour term
    # (|1-0|/1, |1-5|/1, |5-1|/5, |5-10|/5); every other pixel has M = 0
    im = np.zeros((H, W, 3), np.uint8)
    im[:, k:] = 255
    c = oracle.edge_view(im)["margin"]
    for x in range(W):
        col = c[:, x]
        if x in (k - 1, k):
            assert (col == 0).all()
        elif x in (k - 3, k - 2, k + 1, k + 2):
            assert np.allclose(col, T, rtol=1e-15, atol=0)
        else:
            assert np.isinf(col).all()


def test_margin_of_diagonal_ramp_is_zero():
    W, H = 24, 20
    im = np.zeros((H, W, 3), np.uint8)
    im[:] = (np.arange(W)[None, :] + np.arange(H)[:, None]).astype(np.uint8)[..., None]
    c = oracle.edge_view(im)["margin"]
    # the gradient is (8, 8) x 256000 from 3 px inside the borders, so pixels
    # whose diagonal neighbours are inside that region tie with both
    assert (c[4:H - 4, 4:W - 4] == 0).all()


def _field(centre, nbrs, fill=(0, 0)):
    """5x5 gradient field: `centre` at (2, 2), nbrs = {(dx, dy): (gx, gy)}."""
    gx = np.full((5, 5), fill[0], np.int64)
    gy = np.full((5, 5), fill[1], np.int64)
    gx[2, 2], gy[2, 2] = centre
    for (dx, dy), (a, b) in nbrs.items():
        gx[2 + dy, 2 + dx], gy[2 + dy, 2 + dx] = a, b
    return oracle.nms(gx, gy)


def test_margin_known_angle_term():
    # (5, 2): |gy| = 2 < 5 t, horizontal, d = (1, 0); left M = 9, right M = 20;
    # terms |sqrt29 - 3|, |sqrt29 - sqrt20|, 5t - 2, 5 - 2t: the third is least
    o = _field((5, 2), {(-1, 0): (3, 0), (1, 0): (4, 2)})
    want = (5 * math.sqrt(2) - 7) / math.sqrt(29)
    assert o["margin"][2, 2] == pytest.approx(want, rel=1e-13)
    assert o["keep"][2, 2] == 1


def test_margin_known_neighbour_term_on_an_axis():
    # (10, 0), d = (1, 0); left (9, 0), right (2, 0): terms 1, 8, 10t, 10
    o = _field((10, 0), {(-1, 0): (9, 0), (1, 0): (2, 0)})
    assert o["margin"][2, 2] == pytest.approx(0.1, rel=1e-14)
    # the same centre with the neighbours swapped: the -d neighbour is the
    # larger side's partner now, still 1 / 10, and the pixel is kept either way
    o = _field((10, 0), {(-1, 0): (2, 0), (1, 0): (9, 0)})
    assert o["margin"][2, 2] == pytest.approx(0.1, rel=1e-14)


def test_margin_known_neighbour_term_on_a_diagonal():
    # (3, 3): diagonal with gx gy > 0, d = (1, 1); p - d = up-left M = 16,
    # p + d = down-right M = 1; the other six neighbours are large (M = 100)
    # and must not enter: c = (3 sqrt 2 - 4) / (3 sqrt 2) = 1 - 2 sqrt 2 / 3
    big = (10, 0)
    nb = {(dx, dy): big for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)}
    nb[(-1, -1)] = (4, 0)
    nb[(1, 1)] = (1, 0)
    o = _field((3, 3), nb)
    assert o["bin"][2, 2] == 2
    assert o["margin"][2, 2] == pytest.approx(1 - 2 * math.sqrt(2) / 3, rel=1e-14)
    # the anti-diagonal (3, -3): d = (1, -1), p - d = down-left, p + d = up-right
    nb = {(dx, dy): big for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)}
    nb[(-1, 1)] = (4, 0)
    nb[(1, -1)] = (1, 0)
    o = _field((3, -3), nb)
    assert o["bin"][2, 2] == 3
    assert o["margin"][2, 2] == pytest.approx(1 - 2 * math.sqrt(2) / 3, rel=1e-14)


def test_margin_is_infinite_only_at_zero_gradient():
    o = _field((0, 0), {(1, 0): (7, 1), (-1, 0): (2, 9)})
    assert np.isinf(o["margin"][2, 2]) and o["keep"][2, 2] == 0
    assert np.isfinite(o["margin"][o["M"] > 0]).all()


# ---------------------------------------------------------------- soundness

def _decide(gx, gy, rp, rlo_of, rhi_of):
    """The suppression rule on perturbed inputs (plain floats): orientation
    from (gx, gy), then root magnitudes compared with the tie rule."""
    a, c = abs(gx), abs(gy)
    if c < T * a:
        d = (_sgn(gx), 0)
    elif a < T * c:
        d = (0, _sgn(gy))
    else:
        d = (_sgn(gx), _sgn(gy))
    lo, hi = rlo_of(d), rhi_of(d)
    return int(rp > lo and rp >= hi and rp > 0), d


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_margin_bounds_every_decision_flip(seed):
    rng = np.random.default_rng(100 + seed)
    im = synth.image(200 + seed, 40, 32, 8, True) if seed < 2 else rng.integers(118, 123, (24, 24, 3), np.uint8)
    o = oracle.edge_view(im)
    H, W = o["M"].shape
    R = np.sqrt(o["M"].astype(np.float64))
    checked = 0
    for y in range(H):
        for x in range(W):
            c = o["margin"][y, x]
            if not np.isfinite(c) or c < 1e-9:
                continue
            r = R[y, x]
            gx, gy = float(o["gx"][y, x]), float(o["gy"][y, x])
            for _ in range(6):
                u = rng.choice([-1.0, 1.0], 5) * rng.uniform(0.9, 1.0, 5)
                dg, dm = 0.24 * c * r, 0.49 * c * r
                pert = {}

                def root(dd, sgn):
                    q = (_brute_refl(y + sgn * dd[1], H), _brute_refl(x + sgn * dd[0], W))
                    if q not in pert:
                        pert[q] = R[q] + dm * rng.choice([-1.0, 1.0])
                    return pert[q]

                k, d = _decide(gx + u[0] * dg, gy + u[1] * dg, r + u[2] * dm,
                               lambda dd: root(dd, -1), lambda dd: root(dd, +1))
                assert k == o["keep"][y, x], (y, x, c)
            checked += 1
    assert checked > 100
