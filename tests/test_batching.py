"""Host-side chunk planning of event batches (no GPU): events smallest first, chunks of
at most a target number of (event, bin) pairs, an oversized event alone."""
import numpy as np
import pytest

from paper_2602_12052_amd.autotune import plan_chunks


def check_plan(bins, target, chunks):
    bins = [int(b) for b in bins]
    flat = [e for c in chunks for e in c]
    # every event exactly once, in stable smallest-first order
    assert sorted(flat) == list(range(len(bins)))
    assert flat == sorted(range(len(bins)), key=lambda e: bins[e])
    for i, c in enumerate(chunks):
        assert c, "empty chunk"
        n = sum(bins[e] for e in c)
        assert n <= target or len(c) == 1
        # greedy: the next chunk's first event would not have fitted into this one
        if i + 1 < len(chunks):
            assert n + bins[chunks[i + 1][0]] > target


@pytest.mark.parametrize("seed", range(6))
def test_plan_chunks_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 80))
    bins = np.exp(rng.uniform(np.log(5), np.log(1000), n)).astype(int)
    if seed % 2:
        bins[rng.integers(0, n, 3)] = 7          # ties keep their order
    target = int(rng.choice([1, 64, 512, 2000, 10 ** 6]))
    check_plan(bins, target, plan_chunks(bins, target))


def test_plan_chunks_cases():
    # the largest event is over the target: a chunk of its own
    assert plan_chunks([300, 10, 900, 250], 512) == [[1, 3], [0], [2]]
    # a chunk may reach the target exactly; one pair more closes it; zero-bin events
    # ride along with the smallest
    assert plan_chunks([256, 0, 255, 1], 512) == [[1, 3, 2, 0]]
    assert plan_chunks([256, 0, 256, 1], 512) == [[1, 3, 0], [2]]
    assert plan_chunks([], 512) == []
    assert plan_chunks([5, 5, 5], 10 ** 9) == [[0, 1, 2]]
    with pytest.raises(ValueError):
        plan_chunks([1, 2], 0)
