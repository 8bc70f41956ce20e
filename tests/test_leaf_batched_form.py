"""The GPU base case does not draw one value at a time: it takes the first J
draws at once, sorts and de-duplicates them, and grows J by k - D(J) while
only D(J) < k distinct values are seen (each draw adds at most one new
value, so k distinct values cannot appear before draw J + k - D(J)).  Tiles
too large for one LDS pass are split into key sub-ranges, and dense tiles
draw the excluded slots.  This test runs that batched procedure, written out
here with numpy over Philox blocks from the oracle, and requires the same
sorted set as the oracle's sequential definition (Sec. 2.2 base case)."""
import numpy as np
import pytest


def philox_words(kgref, seed, ordinal, tile, nblocks):
    # counter (ordinal, block, tile, TLEAF)
    rec = np.zeros((nblocks, 6), dtype=np.uint32)
    rec[:, 0] = ordinal
    rec[:, 1] = np.arange(nblocks, dtype=np.uint32)
    rec[:, 2] = tile
    rec[:, 3] = kgref.TAG_TLEAF
    rec[:, 4] = seed & 0xFFFFFFFF
    rec[:, 5] = seed >> 32
    return kgref.eval_many(1, rec, np.uint32, 4).reshape(-1)


def batched_leaf(kgref, k, S, seed, ordinal, tile, cap):
    comp = 2 * k > S
    ke = S - k if comp else k
    bits = 0 if S <= 1 else int(S - 1).bit_length()
    mask = (1 << bits) - 1
    span = 1 << bits
    if ke == 0:
        return np.arange(S, dtype=np.uint64)
    nsub = 1
    while nsub < span and nsub * cap < ke:
        nsub *= 2
    J = ke
    while True:
        words = philox_words(kgref, seed, ordinal, tile, (J + 3) // 4)[:J].astype(np.uint64) & mask
        valid = words[words < S]
        W = span // nsub
        over = False
        parts = []
        for sb in range(nsub):
            inr = valid[(valid >= sb * W) & (valid < (sb + 1) * W)]
            if len(inr) > cap:
                over = True
                break
            parts.append(np.unique(inr))
        if over:
            nsub *= 2
            continue
        D = sum(len(p) for p in parts)
        if D == ke:
            chosen = np.concatenate(parts) if parts else np.zeros(0, np.uint64)
            break
        J += ke - D
    if not comp:
        return chosen
    return np.setdiff1d(np.arange(S, dtype=np.uint64), chosen)


@pytest.mark.parametrize("k,S,cap", [(512, 2**29, 1024), (530, 2**29, 1024), (600, 2**21, 1024),
                                     (900, 1000, 1024), (1500, 2048, 1024), (400, 500, 128), (1100, 2**30, 1024),
                                     (3000, 2**20, 256), (3000, 5000, 128), (700, 701, 128), (1, 1, 128),
                                     (5, 7, 128), (2000, 2**32, 512), (64, 3000, 128)])
def test_batched_equals_sequential(kgref, k, S, cap):
    for tile in range(3):
        want = kgref.leaf(k, S, seed=77, ordinal=5, tile=tile)
        got = batched_leaf(kgref, k, S, 77, 5, tile, cap)
        assert np.array_equal(got, want), (k, S, cap, tile)
