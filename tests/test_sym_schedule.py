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
