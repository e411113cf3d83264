"""Host logic of learned scheduling (CPU): the candidate binning policies the
tuner times.  A policy is (edges, depths): samples whose prediction lies in
[edges[b-1], edges[b]) start with a first pass of depths[b] steps."""
import numpy as np
import pytest

from paper_2506_03266_amd import learned


def _valid(pol, lo=1, hi=15):
    edges, depths = pol
    return (len(depths) == len(edges) + 1 and all(lo <= d <= hi for d in depths)
            and list(edges) == sorted(edges) and list(depths) == sorted(depths))


@pytest.mark.parametrize("k", [1, 2, 4, 5])
@pytest.mark.parametrize("wide", [False, True])
def test_candidates_are_valid_and_start_with_the_fallback(k, wide):
    pred = np.random.default_rng(k).normal(1.6, 0.1, 500)
    pols = learned.candidate_policies(pred, k, wide)
    assert pols[0] == ((), (k,))            # one group: the FIFO fallback, timed first
    assert all(_valid(p) for p in pols)
    assert len(set(pols)) == len(pols)      # no policy timed twice
    depths = {d for _, ds in pols for d in ds}
    assert min(depths) >= max(1, k - (2 if wide else 1)) and max(depths) <= k + (2 if wide else 1)


def test_wide_candidates_cover_every_two_and_three_depth_split():
    pred = np.linspace(1.0, 2.0, 101)
    k = 5
    pols = learned.candidate_policies(pred, k, True)
    pairs = {ds for e, ds in pols if len(ds) == 2}
    triples = {ds for e, ds in pols if len(ds) == 3}
    assert pairs == {(a, c) for a in range(3, 8) for c in range(a + 1, 8)}
    assert triples == {(a, c, d) for a in range(3, 8) for c in range(a + 1, 8) for d in range(c + 1, 8)}
    # split points are the prediction deciles
    edges = {e[0] for e, ds in pols if len(ds) == 2}
    assert edges == {float(q) for q in np.quantile(pred, np.arange(1, 10) / 10)}


def test_narrow_candidates():
    pred = np.linspace(0.0, 1.0, 11)
    pols = learned.candidate_policies(pred, 4, False)
    assert {ds for _, ds in pols} == {(4,), (3, 4), (4, 5), (3, 4, 5)}
    assert len(pols) == 1 + 9 * 2 + 36
