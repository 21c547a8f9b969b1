"""Pins of the split-mask oracle: a hand-worked example, brute force on small
random problems (a pairwise count instead of a sort), order independence of
the exact fixed-point scores, and the warm-up / budget / invalid-entry rules."""
import numpy as np

import oracle


def _problem(seed, N=40, n_views=2, n=400, W=(7, 5), H=(6, 9)):
    rng = np.random.default_rng(seed)
    W, H = np.array(W[:n_views]), np.array(H[:n_views])
    off = np.r_[0, np.cumsum(W * H)[:-1]]
    maps = rng.random(int((W * H).sum())).astype(np.float32)
    maps[rng.random(maps.size) < 0.6] = 0.0                  # most pixels suppressed
    g = rng.integers(-2, N + 3, n).astype(np.int32)          # some out of range on purpose
    v = rng.integers(0, n_views + 1, n).astype(np.int32)
    p = rng.integers(-1, 60, n).astype(np.int32)
    w = rng.random(n).astype(np.float32)
    return maps, W, H, off, g, v, p, w


def test_hand_worked_scores_and_mask():
    # view 0: 2 x 2 map [0.5, 0, 0.25, 1.0]; view 1 (offset 4): 1 x 3 map [2, 0, 0.75]
    maps = np.array([0.5, 0.0, 0.25, 1.0, 2.0, 0.0, 0.75], np.float32)
    W, H, off = [2, 3], [2, 1], [0, 4]
    #          g   v  p   w        product (exact in float32) -> units of 2^-32
    rows = [(0, 0, 0, 0.25),   # 0.125  -> 2^29
            (0, 1, 2, 0.5),    # 0.375  -> 3 * 2^29
            (1, 0, 1, 1.0),    # 0      -> nothing
            (1, 0, 3, 0.125),  # 0.125  -> 2^29
            (2, 1, 0, 0.0625), # 0.125  -> 2^29
            (3, 0, 4, 1.0),    # pixel 4 outside the 2 x 2 view -> ignored
            (5, 0, 0, 1.0)]    # Gaussian 5 >= N = 4 -> ignored
    g, v, p, w = (np.array(c) for c in zip(*rows))
    sc = oracle.split_scores(maps, W, H, off, g, v, p, w.astype(np.float32), N=4)
    assert sc.tolist() == [4 * 2 ** 29, 2 ** 29, 2 ** 29, 0]
    grad = np.array([1e-4, 5e-4, 2e-4, 9e-4], np.float32)
    # threshold 1.5e-4: candidates 1, 2, 3; budget 6 -> K = 2: the tie 1 == 2 goes to index 1, then 2
    mask, K = oracle.split_select(sc, grad, 4, 1.5e-4, False, 6)
    assert K == 2 and mask.tolist() == [0, 1, 1, 0]
    mask, K = oracle.split_select(sc, grad, 4, 1.5e-4, False, 5)   # K = 1: lower index wins the tie
    assert K == 1 and mask.tolist() == [0, 1, 0, 0]
    mask, K = oracle.split_select(sc, grad, 4, 1.5e-4, True, 5)    # warm-up: Gaussian 0 competes
    assert K == 1 and mask.tolist() == [1, 0, 0, 0]
    mask, K = oracle.split_select(sc, grad, 4, 1.0, False, 100)    # no candidate
    assert K == 0 and mask.sum() == 0
    mask, K = oracle.split_select(sc, grad, 4, 0.0, False, 3)      # budget below N
    assert K == 0 and mask.sum() == 0


def _brute(scores, cand, K):
    """Selected iff fewer than K candidates rank above it (score, then index)."""
    n = scores.size
    sel = np.zeros(n, np.uint8)
    for i in range(n):
        if not cand[i]:
            continue
        above = sum(1 for j in range(n) if cand[j] and (scores[j] > scores[i] or (scores[j] == scores[i] and j < i)))
        sel[i] = above < K
    return sel


def test_selection_against_brute_force():
    for seed in range(30):
        maps, W, H, off, g, v, p, w = _problem(seed)
        N = 40
        sc = oracle.split_scores(maps, W, H, off, g, v, p, w, N)
        rng = np.random.default_rng(100 + seed)
        grad = rng.random(N).astype(np.float32)
        thr = float(rng.random())
        warm = bool(seed % 3 == 0)
        budget = int(rng.integers(N - 5, 2 * N))
        mask, K = oracle.split_select(sc, grad, N, thr, warm, budget)
        cand = np.ones(N, bool) if warm else grad >= np.float32(thr)
        assert K == min(int(cand.sum()), max(0, budget - N))
        assert (mask == _brute(sc, cand, K)).all()


def test_scores_independent_of_entry_order_and_exact():
    maps, W, H, off, g, v, p, w = _problem(7, n=2000)
    a = oracle.split_scores(maps, W, H, off, g, v, p, w, 40)
    perm = np.random.default_rng(1).permutation(g.size)
    b = oracle.split_scores(maps, W, H, off, g[perm], v[perm], p[perm], w[perm], 40)
    assert (a == b).all()
    # each valid entry's term, summed by a plain Python loop
    ref = [0] * 40
    for gi, vi, pi, wi in zip(g, v, p, w):
        if 0 <= gi < 40 and 0 <= vi < len(W) and 0 <= pi < W[vi] * H[vi]:
            e = np.float32(maps[off[vi] + pi]) * np.float32(wi)
            if e > 0:
                ref[gi] += int(np.floor(float(e) * 2.0 ** 32))
    assert a.tolist() == ref


def test_fixed_point_scores_select_what_real_sums_select():
    """How much the fixed-point reading of the score (each product rounded to
    float32, then floored to units of 2^-32) moves the selection, against
    scores summed in FP64 from the exact products of the stored float32
    inputs. 200k Gaussians, 20 views of 1024 x 768 with log-normal maps (65%
    of pixels zero), discs of radius 1-5 px, 40% candidates, K = 20%. A
    Gaussian can change sides only if its real score lies within its own
    rounding bound plus the K-th score's of the K-th real score; every one
    that changes must be such a one, and there are at most a few."""
    import synth

    rng = np.random.default_rng(77)
    nv, W, H, N = 20, 1024, 768, 200_000
    Ws, Hs = np.full(nv, W), np.full(nv, H)
    off = np.arange(nv, dtype=np.int64) * W * H
    maps = rng.lognormal(0.0, 1.0, nv * W * H).astype(np.float32)
    maps[rng.random(maps.size) < 0.65] = 0.0
    c = synth.contributions(4242, N, Ws, Hs, 3)
    q = oracle.split_scores(maps, Ws, Hs, off, c.gauss, c.view, c.pixel, c.weight, N)
    # real-valued scores: FP64 products of the same float32 inputs, no rounding to float32, no floor
    e = maps[off[c.view] + c.pixel].astype(np.float64) * c.weight.astype(np.float64)
    real = np.bincount(c.gauss, weights=e, minlength=N)
    # per-Gaussian bound of |q 2^-32 - real|: float32 rounding of each product (2^-24 relative)
    # and the floor (2^-32 absolute), summed over its contributions
    bound = np.bincount(c.gauss, weights=e * 2.0 ** -24 + 2.0 ** -32, minlength=N)
    assert np.all(np.abs(q * 2.0 ** -32 - real) <= bound)
    grad = synth.grad_accum(4243, N)
    thr = float(np.quantile(grad, 0.6))
    K = N // 5
    budget = N + K
    mq, kq = oracle.split_select(q, grad, N, thr, False, budget)
    cand = grad >= np.float32(thr)
    idx = np.flatnonzero(cand)
    order = np.lexsort((idx, -real[idx]))
    mr = np.zeros(N, np.uint8)
    mr[idx[order[:K]]] = 1
    assert kq == K
    changed = np.flatnonzero(mq != mr)
    t = real[idx[order[K - 1]]]                          # the K-th real score
    bk = bound[idx[order[K - 1]]]
    assert np.all(np.abs(real[changed] - t) <= bound[changed] + bk + 1e-300)
    assert changed.size <= 4, changed.size
    print(f"selection differs for {changed.size} of {N} Gaussians ({K} selected)")
