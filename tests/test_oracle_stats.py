"""Population statistics of the oracle (percentile ranks and PMF counts of
goals, Sec. 4.2), pinned by the characterisations of the definitions: the
nearest-rank value v of rank r has fewer than r values below it and at least
r values at or below it; histogram counts are the number of values in each
bin's half-open range, found by direct comparison with the bin edges."""
import numpy as np
import pytest


@pytest.mark.parametrize("N", [1, 2, 5, 50, 999])
def test_nearest_rank_characterisation(orc, N):
    rng = np.random.default_rng(N)
    vals = rng.integers(-50, 60, size=N) * 1000 + rng.integers(0, 3, size=N)  # many ties
    q = [1, 50000, 250000, 500000, 750000, 999999, 1000000]
    got = orc.nearest_rank_quantiles(vals, q)
    for qi, v in zip(q, got):
        r = max(1, -(-qi * N // 1000000))
        below = int((vals < v).sum())
        at_or_below = int((vals <= v).sum())
        assert below < r <= at_or_below, (N, qi, v)


def test_nearest_rank_paper_counts(orc):
    """For 50 particles the 5 % rank falls on the third smallest value
    (ceil(2.5)); for 12,500 particles on the 625th."""
    vals = np.arange(50)[::-1] * 7
    assert orc.nearest_rank_quantiles(vals, [50000])[0] == 14
    vals = np.arange(12500)
    assert orc.nearest_rank_quantiles(vals, [50000])[0] == 624


@pytest.mark.parametrize("bins", [1, 7, 64])
def test_histogram_against_edges(orc, bins):
    rng = np.random.default_rng(bins)
    vals = rng.integers(-1000, 5000, size=3000)
    lo, hi = -500, 4321
    h = orc.goal_histogram(vals, bins, lo, hi)
    for b in range(bins):
        # bin b holds g with b <= (g - lo) * bins / (hi - lo) < b + 1
        cnt = sum(1 for g in vals if lo <= g < hi and b * (hi - lo) <= (g - lo) * bins < (b + 1) * (hi - lo))
        assert h[b] == cnt
    assert h.sum() == int(((vals >= lo) & (vals < hi)).sum())
