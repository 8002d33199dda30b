"""The schedule of the symmetric pair kernel, modelled on the CPU.

The kernel cuts the points into groups of 256 (four 64-point tiles); with G groups, the wave of
group g and distance chunk c meets group h = (g + d) mod G for the distances d of its chunk,
symmetrically for 1 <= d < G/2 and one-sidedly at d = 0 and d = G/2 (even G).  It writes the
target sums of chunk c into slice c and the source sums of distance d into slice nchunks_d + d - 1.
This model repeats the kernel's index arithmetic (the plan of `sym_plan` and the loops of
`ghat_sym_kernel`) and checks, for every tile count and chunking, that each ordered pair of tiles
is formed exactly once and each slice entry is written exactly once, so the S product, which adds
every slice, sees each pair's contribution once and reads no stale memory.
"""

import collections

import pytest


def plan(N, nchunks_d):
    G = (N + 255) // 256
    Dmax = G // 2
    even = G % 2 == 0
    Dsym = max(0, Dmax - 1 if even else Dmax)
    want = nchunks_d if nchunks_d > 0 else min(1024, (65536 + G - 1) // max(G, 1))
    want = max(1, min(want, Dmax + 1))
    dpc = (Dmax + 1 + want - 1) // want
    nchd = (Dmax + 1 + dpc - 1) // dpc
    return G, Dmax, even, Dsym, dpc, nchd, nchd + Dsym


def run(N, nchunks_d):
    G, Dmax, even, Dsym, dpc, nchd, slices = plan(N, nchunks_d)
    ntiles = N // 64
    cover = collections.Counter()
    writes = collections.Counter()
    for g in range(G):
        for c in range(nchd):
            for d in range(c * dpc, min(Dmax + 1, c * dpc + dpc)):
                h = (g + d) % G
                sym = d != 0 and not (even and d == Dmax)
                for ts in range(4):
                    j0 = h * 256 + 64 * ts
                    if j0 >= N:
                        break
                    for m in range(4):
                        t0 = g * 256 + 64 * m
                        if t0 < N:
                            cover[(t0 // 64, j0 // 64)] += 1
                            if sym:
                                cover[(j0 // 64, t0 // 64)] += 1
                    if sym:
                        writes[(nchd + d - 1, j0 // 64)] += 1
            for m in range(4):
                if g * 256 + 64 * m < N:
                    writes[(c, (g * 256 + 64 * m) // 64)] += 1
    return ntiles, slices, cover, writes


@pytest.mark.parametrize("tiles", list(range(1, 34)) + [63, 64, 65, 100])
@pytest.mark.parametrize("nchunks_d", [0, 1, 2, 3, 1024])
def test_every_pair_once_every_slice_entry_once(tiles, nchunks_d):
    ntiles, slices, cover, writes = run(64 * tiles, nchunks_d)
    assert all(cover[(a, b)] == 1 for a in range(ntiles) for b in range(ntiles))
    assert len(cover) == ntiles * ntiles
    assert all(writes[(s, t)] == 1 for s in range(slices) for t in range(ntiles))
    assert len(writes) == slices * ntiles


def test_slice_count_of_the_starfish_scene():
    # 256,000 points: 1000 groups, 63 distance chunks of 8, 499 source-side slices
    assert plan(256000, 0) == (1000, 500, True, 499, 8, 63, 562)


# ----------------------------------------------------------------------------------------------
# The 3D kernel on 16-point sub-blocks (tiles may straddle bodies).  Against one staged source tile,
# lane l = 16 G + i takes in phase p (0..3) sub-block b = (G + p) mod 4 and at step t (0..15) the
# source 16 b + ((i + t) mod 16), read from LDS entry 48 b + i + t (each sub-block staged twice, at
# e and e + 16).  The running source-side sums rotate by one lane inside each row of 16 after every
# step (lane l receives lane (l & ~15) | ((l + 1) & 15)) and move one row down after every phase
# (lane l receives lane (l + 16) mod 64).  The model follows which source's sum each lane holds.
def sub_block_schedule():
    holder = list(range(64))  # holder[l]: the source whose running sum lane l holds
    pairs = collections.Counter()
    entries = set()
    for p in range(4):
        for t in range(16):
            for lane in range(64):
                G, i = lane >> 4, lane & 15
                b = (G + p) & 3
                e = 48 * b + i + t
                src = 16 * b + ((i + t) & 15)
                assert e - 48 * b in range(32)  # inside the sub-block's two staged copies
                assert (e - 48 * b) % 16 == src % 16
                assert holder[lane] == src  # the lane adds into the sum of the source it meets
                pairs[(lane, src)] += 1
                entries.add(e)
            holder = [holder[(lane & ~15) | ((lane + 1) & 15)] for lane in range(64)]
        holder = [holder[(lane + 16) & 63] for lane in range(64)]
    return pairs, holder, entries


def test_sub_block_schedule_meets_every_pair_once_and_returns_the_sums():
    pairs, holder, entries = sub_block_schedule()
    assert len(pairs) == 64 * 64 and set(pairs.values()) == {1}
    assert holder == list(range(64))  # lane j ends with source j's sum: plain coalesced stores
    assert max(entries) < 4 * 48


def test_sub_block_phases_see_one_sub_block_per_row():
    # within a phase each row of 16 lanes reads one sub-block, so a lane's source body (and its
    # body-centre constants) is fixed for the phase; the four rows read four different sub-blocks
    for p in range(4):
        blocks = [((lane >> 4) + p) & 3 for lane in range(64)]
        for G in range(4):
            assert len(set(blocks[16 * G:16 * G + 16])) == 1
        assert sorted(set(blocks)) == [0, 1, 2, 3]
