"""The exponential learning-rate schedule (Sec. 3): the library's host
function against the oracle, and both against the paper's endpoints and the
closed forms of an exponential decay."""
import math

import pytest

import oracle
import paper_2603_08661_amd as igsp


@pytest.mark.parametrize("lr0,lr1", [(0.020, 0.002), (0.000128, 0.0000128)])   # scale, position (Sec. 3)
def test_endpoints_midpoint_ratio(lr0, lr1):
    T = 30000
    for f in (igsp.lr_exponential, oracle.lr_exponential):
        assert f(0, lr0, lr1, T) == pytest.approx(lr0, rel=1e-15)
        assert f(T, lr0, lr1, T) == pytest.approx(lr1, rel=1e-15)
        assert f(T // 2, lr0, lr1, T) == pytest.approx(math.sqrt(lr0 * lr1), rel=1e-14)   # geometric mean
        assert f(-5, lr0, lr1, T) == pytest.approx(lr0) and f(T + 9, lr0, lr1, T) == pytest.approx(lr1)
        # constant ratio over equal steps (an exponential): gamma = lr1 / lr0 = 0.1 per T
        assert f(7000, lr0, lr1, T) / f(4000, lr0, lr1, T) == pytest.approx(0.1 ** (3000 / T), rel=1e-13)


def test_library_matches_oracle_and_rejects_bad_input():
    for t in range(0, 30001, 997):
        assert igsp.lr_exponential(t, 0.02, 0.002, 30000) == pytest.approx(oracle.lr_exponential(t, 0.02, 0.002, 30000),
                                                                          rel=1e-14)
    assert math.isnan(igsp.lr_exponential(1, 0.0, 0.1, 10)) and math.isnan(igsp.lr_exponential(1, 0.1, 0.1, 0))
