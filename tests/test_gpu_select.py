"""GPU parity of split_mask against the oracle (through the C ABI): scores,
mask and K bit-exact (the scores are exact fixed-point sums), over ties,
budgets, warm-up, out-of-range entries and sizes around the tile."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _maps(seed, W, H):
    rng = np.random.default_rng(seed)
    off = np.r_[0, np.cumsum(np.asarray(W) * np.asarray(H))[:-1]].astype(np.int64)
    maps = (rng.lognormal(0.0, 0.8, int(off[-1] + W[-1] * H[-1]))).astype(np.float32)
    maps[rng.random(maps.size) < 0.65] = 0.0           # suppressed pixels
    return maps, off


def run(N, cap, W, H, c, grad, thr, warm, budget, maps, off, extra_bad=False):
    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    g, v, p, w = c.gauss.copy(), c.view.copy(), c.pixel.copy(), c.weight.copy()
    if extra_bad:      # entries the call must ignore
        g = np.r_[g, N, N + 5, 0, 1].astype(np.int32)
        v = np.r_[v, 0, 0, len(W), 0].astype(np.int32)
        p = np.r_[p, 0, 0, 0, W[0] * H[0]].astype(np.int32)
        w = np.r_[w, 1, 1, 1, 1].astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    gradp = np.zeros(cap, np.float32)
    gradp[:N] = grad
    mask = torch.full((cap,), 7, dtype=torch.uint8, device=dev)
    scores = torch.full((cap,), -1, dtype=torch.int64, device=dev)
    nsel = torch.full((1,), -1, dtype=torch.int64, device=dev)
    count = torch.tensor([N], dtype=torch.int64, device=dev)
    views = (np.asarray(W), np.asarray(H), np.zeros(len(W), np.int64), off)
    igsp.split_mask(T(maps), views, T(g), T(v), T(p), T(w), T(gradp), count, mask, scores, grad_threshold=thr,
                    warmup=warm, budget=budget, n_selected=nsel)
    torch.cuda.synchronize()
    ref_s = oracle.split_scores(maps, W, H, off, g, v, p, w, N)
    ref_m, ref_k = oracle.split_select(ref_s, grad, N, thr, warm, budget)
    got_s, got_m = scores.cpu().numpy(), mask.cpu().numpy()
    assert (got_s[:N] == ref_s).all(), "scores"
    assert (got_s[N:] == -1).all() and (got_m[N:] == 7).all(), "rows past N touched"
    assert int(nsel.item()) == ref_k
    assert (got_m[:N] == ref_m).all(), f"mask: {int((got_m[:N] != ref_m).sum())} rows differ"
    return ref_k


@pytest.mark.parametrize("order", ["rows", "spread"])
@pytest.mark.parametrize("N,radius,thr,warm,budget_extra", [
    (1000, 3, 3e-4, False, 300),
    (2048, 2, 1e-4, False, 10 ** 6),      # budget above the candidates: every candidate
    (2049, 3, 2e-4, True, 500),           # warm-up
    (5000, 1, 5e-4, False, 0),            # budget == N: nothing
    (70001, 4, 1.5e-4, False, 7000),
])
def test_split_mask_parity(N, radius, thr, warm, budget_extra, order):
    W, H = [320, 257, 96], [200, 133, 61]
    maps, off = _maps(N, W, H)
    c = synth.contributions(N + 1, N, W, H, radius, order)
    grad = synth.grad_accum(N + 2, N)
    K = run(N, N + 123, W, H, c, grad, thr, warm, N + budget_extra, maps, off, extra_bad=True)
    print(N, "K", K, "contributions", c.n)


def test_split_mask_ties_and_zero_scores():
    """Most Gaussians get no contribution (score 0): the K-th key sits in a
    large tie, resolved by index order across tiles."""
    N = 9000
    W, H = [64], [64]
    maps, off = _maps(3, W, H)
    c = synth.contributions(4, 500, W, H, 2)           # only Gaussians < 500 contribute
    grad = np.full(N, 1.0, np.float32)
    for budget in (N + 100, N + 600, N + 4097, N + 8999):
        run(N, N, W, H, c, grad, 0.5, False, budget, maps, off)


def test_split_mask_repeated_calls_and_empty():
    N = 3000
    W, H = [100], [80]
    maps, off = _maps(5, W, H)
    c = synth.contributions(6, N, W, H, 3)
    grad = synth.grad_accum(7, N)
    for _ in range(3):          # the plan's radix histogram is restored by each call
        run(N, N, W, H, c, grad, 1e-4, False, N + 700, maps, off)
    empty = synth.Contributions(*(np.zeros(0, t) for t in (np.int32, np.int32, np.int32, np.float32)))
    run(N, N, W, H, empty, grad, 1e-4, False, N + 700, maps, off)     # all scores 0: index order
    run(0, 16, W, H, c, np.zeros(0, np.float32), 0.0, False, 100, maps, off)   # N = 0


@pytest.mark.parametrize("scale", [2e-9, 1.0, 3.0e6])
def test_split_mask_key_widths(scale):
    """The radix selection starts at the highest digit any candidate key
    uses: keys of one byte (scores of a few units of 2^-32), of about 40 bits
    (the usual range), and of 58-60 bits (the top digit of the 64-bit key)."""
    N = 6000
    W, H = [150, 90], [120, 77]
    maps, off = _maps(11, W, H)
    maps = (maps * np.float32(scale)).astype(np.float32)
    c = synth.contributions(12, N, W, H, 3)
    grad = synth.grad_accum(13, N)
    ref = oracle.split_scores(maps, W, H, off, c.gauss, c.view, c.pixel, c.weight, N)
    bits = int(ref.max()).bit_length()
    assert (scale < 1e-6 and bits <= 8) or (scale == 1.0 and 30 < bits < 48) or (scale > 1e6 and bits > 56), bits
    for budget in (N + 1, N + 1500, N + 5999):
        run(N, N + 7, W, H, c, grad, 1e-4, False, budget, maps, off)


@pytest.mark.parametrize("order", ["rows", "spread"])
@pytest.mark.parametrize("case", ["threshold", "ties_everywhere"])
def test_split_mask_above_one_grid_of_tiles(order, case):
    """N = 2.5M rows: 1221 tiles of 2048 rows against a grid of 1024
    work-groups, so the count, compact and mask kernels stride past the grid,
    each thread of the tile scan sums two tiles, and the radix passes stride
    over more candidates than the grid holds threads. 'threshold': every
    Gaussian contributes, 40% pass the gradient test, 20% are selected (the
    K-th key lies inside the scores). 'ties_everywhere': only the first 300k
    Gaussians contribute, warm-up makes every row a candidate and K = 1.2M,
    so the K-th key is the zero score shared by 2.2M rows in every tile,
    taken in index order across all of them."""
    N = 2_500_000
    W, H = [1297, 2000, 640], [840, 1300, 480]
    maps, off = _maps(77, W, H)
    grad = synth.grad_accum(78, N)
    if case == "threshold":
        c = synth.contributions(79, N, W, H, 1, order)
        thr, warm, budget = float(np.quantile(grad, 0.6)), False, N + N // 5
    else:
        c = synth.contributions(80, 300_000, W, H, 2, order)
        thr, warm, budget = 0.0, True, N + 1_200_000
    print(f"{case}/{order}: {c.n} contributions", flush=True)
    K = run(N, N + 777, W, H, c, grad, thr, warm, budget, maps, off)
    assert K == budget - N
