"""Pins of the base case (Sec. 2.2: below a threshold a sequential sampler
draws the sample): draw-until-k-distinct over a tile of S slots, output
ascending, complement when 2k > S.  Brute force: every k-subset of a small
tile must be equally likely."""
import math
from itertools import combinations

import numpy as np
import pytest
from scipy import stats


@pytest.mark.parametrize("S,k", [(4, 2), (5, 2), (6, 3), (7, 5), (8, 1), (8, 7), (9, 4),
                                  (12, 3), (12, 9), (3, 3), (1, 1), (10, 10), (11, 6)])
def test_all_subsets_equally_likely(kgref, S, k):
    subsets = {c: i for i, c in enumerate(combinations(range(S), k))}
    nsub = len(subsets)
    reps = max(60 * nsub, 3000)
    counts = np.zeros(nsub, dtype=np.int64)
    for t in range(reps):
        keys = kgref.leaf(k, S, seed=99, ordinal=t % 997, tile=t // 997)
        tup = tuple(int(x) for x in keys)
        assert list(tup) == sorted(set(tup)) and len(tup) == k
        assert all(0 <= x < S for x in tup)
        counts[subsets[tup]] += 1
    if nsub > 1:
        assert stats.chisquare(counts).pvalue > 1e-5


def test_leaf_sorted_distinct_large(kgref):
    for S, k in [(2**29, 512), (2**21, 600), (2**32, 1000), (2**32, 2**31 + 5), (1000, 999),
                 (3000, 1500), (3000, 1501), (2**20 + 7, 900)]:
        if k > 10**6:
            continue
        keys = kgref.leaf(k, S, seed=1, ordinal=3, tile=5)
        assert len(keys) == k
        assert np.all(np.diff(keys.astype(np.int64)) > 0)
        assert keys[0] >= 0 and int(keys[-1]) < S


def test_leaf_position_marginals_uniform(kgref):
    # Each slot is chosen with probability k/S: chi-square over slot hits.
    S, k, reps = 40, 7, 6000
    hits = np.zeros(S, dtype=np.int64)
    for t in range(reps):
        hits[kgref.leaf(k, S, seed=5, ordinal=t, tile=0).astype(np.int64)] += 1
    assert stats.chisquare(hits).pvalue > 1e-5
    assert hits.sum() == k * reps


def test_leaf_stream_definition_first_draws(kgref):
    """Without repeats and rejections the first k masked words are the sample:
    draw t is word t mod 4 of block t/4 of stream (seed, ordinal, tile, TLEAF):
    Philox counter (ordinal, t/4, tile, TLEAF)."""
    S, k, seed, o, t = 2**30, 9, 12345, 17, 4
    words = []
    for j in range(3):
        words += [int(w) for w in kgref.philox([o, j, t, kgref.TAG_TLEAF], [seed & 0xFFFFFFFF, seed >> 32])]
    want = sorted(w & (S - 1) for w in words[:k])
    assert len(set(want)) == k
    assert [int(x) for x in kgref.leaf(k, S, seed, o, t)] == want
