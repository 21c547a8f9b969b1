"""Arithmetic identities the GPU kernels rely on, checked exhaustively or on
dense random samples on the CPU (no GPU): the suppression decision as one
unsigned compare of float bit patterns."""
import numpy as np


def _keep_float(m, A, B, neg):
    # the oracle's rule: M(p) > M(p - d) and M(p) >= M(p + d) and M(p) > 0,
    # with (p - d, p + d) = (A, B) if d = +e, else (B, A)
    strict, loose = np.where(neg, B, A), np.where(neg, A, B)
    return (m > strict) & (m >= loose) & (m > 0)


def _keep_bits(m, A, B, neg):
    u = lambda x: x.view(np.uint32).astype(np.uint64)  # noqa: E731
    sgn = np.where(neg, -1, 0).astype(np.int64)
    bA = (u(A) + 1 + sgn).astype(np.uint64)
    bB = (u(B) - sgn).astype(np.uint64)
    return u(m) >= np.maximum(np.maximum(bA, bB), 1)


def test_suppression_bit_compare_matches_float_rule():
    rng = np.random.default_rng(7)
    n = 2_000_000
    # magnitudes: integers (squares of exact gradients) and their neighbours,
    # many exact ties and zeros, plus adjacent floats
    base = rng.integers(0, 50, n).astype(np.float32) ** 2
    m = base.copy()
    A = np.where(rng.random(n) < 0.3, base, rng.integers(0, 50, n).astype(np.float32) ** 2)
    B = np.where(rng.random(n) < 0.3, base, rng.integers(0, 50, n).astype(np.float32) ** 2)
    nudge = rng.integers(-1, 2, n)
    A = np.where(A > 0, np.nextafter(A, np.where(nudge > 0, np.inf, 0)).astype(np.float32), A)
    A = np.where(nudge == 0, base, A)
    big = rng.random(n) < 0.1
    m = np.where(big, rng.random(n).astype(np.float32) * 3e16, m).astype(np.float32)
    B = np.where(big, m, B).astype(np.float32)
    neg = rng.random(n) < 0.5
    assert (_keep_float(m, A, B, neg) == _keep_bits(m, A, B, neg)).all()


def test_suppression_bit_compare_small_exhaustive():
    vals = np.array([0.0, 1.0, 2.0, 4.0, 5.0, 8.0, 9.0, np.nextafter(np.float32(4.0), np.float32(0))],
                    np.float32)
    m, A, B = np.meshgrid(vals, vals, vals, indexing="ij")
    m, A, B = m.ravel(), A.ravel(), B.ravel()
    for neg in (False, True):
        nn = np.full(m.shape, neg)
        assert (_keep_float(m, A, B, nn) == _keep_bits(m, A, B, nn)).all()
