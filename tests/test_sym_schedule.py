"""The schedule of the symmetric pair kernels, modelled on the CPU.

The kernels cut the points into groups of 256 (four 64-point tiles); with G groups, group g meets
group h = (g + d) mod G for d = 0 .. G/2, symmetrically for 1 <= d < G/2 and one-sidedly at d = 0
and d = G/2 (even G).  Two forms share that pairing:

* one wave per block (W = 1): the wave of group g and distance chunk c meets the groups of its
  distances, writes its target sums of chunk c into target slice c and the source sums of distance
  d into slice nchunks_d + d - 1;
* W = 8 waves per block sharing each source tile: the G0 real groups are padded with empty ones to
  G, a multiple of W; block b holds target groups W b .. W b + W - 1 (one per wave) and walks block
  offsets hh: at hh every wave meets the same source group (W b + hh) mod G, wave w at distance
  hh - w (idle outside 0 .. G/2), and the waves' source-side sums of the tile are added in the block
  (in wave order) and written once, into source slice hh / W.  Chunk c covers offsets
  c dpc .. c dpc + dpc - 1; each wave writes its target sums of chunk c into target slice c.

This model repeats the kernels' index arithmetic (the plan of `sym_plan`, the tile walk and the loops
of the kernels) and checks, for every tile count and chunking, that each ordered pair of tiles is
formed exactly once and each slice entry is written exactly once, so the S product, which adds every
slice, sees each pair's contribution once and reads no stale memory.
"""

import collections

import pytest

def cdiv(a, b):
    return (a + b - 1) // b


def plan(N, nchunks_d, W):
    G0 = cdiv(N, 256)
    G = W * cdiv(G0, W)
    Dmax = G // 2
    even = G % 2 == 0
    # one wave: distances 0 .. Dmax; W waves: offsets 0 .. HH - 1 reach distance Dmax for every wave
    HH = Dmax + 1 if W == 1 else W * cdiv(Dmax + W, W)
    want = nchunks_d if nchunks_d > 0 else min(1024, cdiv(65536, G))
    want = max(1, min(want, HH))
    dpc = cdiv(HH, want)
    nchd = cdiv(HH, dpc)
    dsym = max(0, Dmax - 1 if even else Dmax)
    return G, Dmax, even, HH, dpc, nchd, nchd + (dsym if W == 1 else HH // W)


def tile_start(gb, G, hh, ts):
    """First point of tile ts of source group (gb + hh) mod G, with the kernels' single conditional
    subtraction in place of the remainder (valid because gb + hh < 2 G)."""
    h = gb + hh
    assert h < 2 * G
    if h >= G:
        h -= G
    assert h == (gb + hh) % G
    return h * 256 + 64 * ts


def seek(gb, G, N, hh1, hh, ts):
    """The kernels' tile walk: the next tile at or after (hh, ts), skipping groups past N."""
    while hh < hh1:
        if ts < 4 and tile_start(gb, G, hh, ts) < N:
            return True, hh, ts
        hh, ts = hh + 1, 0
    return False, hh, ts


def run_one_wave(N, nchunks_d):
    G, Dmax, even, HH, dpc, nchd, slices = plan(N, nchunks_d, 1)
    ntiles = N // 64
    cover = collections.Counter()
    writes = collections.Counter()
    for g in range(G):
        for c in range(nchd):
            for d in range(c * dpc, min(Dmax + 1, c * dpc + dpc)):
                h = g + d
                if h >= G:
                    h -= G
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


def run(N, nchunks_d, W):
    if W == 1:
        return run_one_wave(N, nchunks_d)
    G, Dmax, even, HH, dpc, nchd, slices = plan(N, nchunks_d, W)
    ntiles = N // 64
    cover = collections.Counter()
    writes = collections.Counter()
    for b in range(G // W):
        gb = W * b
        for c in range(nchd):
            hh1 = min(HH, c * dpc + dpc)
            have, hh, ts = seek(gb, G, N, hh1, c * dpc, 0)
            while have:
                h = (gb + hh) % G
                j0 = tile_start(gb, G, hh, ts)
                for w in range(W):
                    g, d = gb + w, hh - w
                    if not 0 <= d <= Dmax:
                        continue
                    assert (g + d) % G == h
                    sym = d != 0 and not (even and d == Dmax)
                    for m in range(4):
                        t0 = g * 256 + 64 * m
                        if t0 < N:
                            cover[(t0 // 64, j0 // 64)] += 1
                            if sym:
                                cover[(j0 // 64, t0 // 64)] += 1
                writes[(nchd + hh // W, j0 // 64)] += 1  # the block's sum over its waves
                have, hh, ts = seek(gb, G, N, hh1, hh, ts + 1)
            for w in range(W):
                for m in range(4):
                    t0 = (gb + w) * 256 + 64 * m
                    if t0 < N:
                        writes[(c, t0 // 64)] += 1
    return ntiles, slices, cover, writes


@pytest.mark.parametrize("W", [1, 8])
@pytest.mark.parametrize("tiles", list(range(1, 34)) + [63, 64, 65, 100, 131])
@pytest.mark.parametrize("nchunks_d", [0, 1, 2, 3, 1024])
def test_every_pair_once_every_slice_entry_once(tiles, nchunks_d, W):
    ntiles, slices, cover, writes = run(64 * tiles, nchunks_d, W)
    assert all(cover[(a, b)] == 1 for a in range(ntiles) for b in range(ntiles))
    assert len(cover) == ntiles * ntiles
    assert all(writes[(s, t)] == 1 for s in range(slices) for t in range(ntiles))
    assert len(writes) == slices * ntiles


def test_slice_count_of_the_starfish_scene():
    # 256,000 points, 1000 groups.  One wave per block: 63 chunks of 8 distances, 499 source-side
    # slices (one per symmetric distance).  Eight waves per block: 64 chunks of 8 block offsets, 64
    # source-side slices
    assert plan(256000, 0, 1) == (1000, 500, True, 501, 8, 63, 562)
    assert plan(256000, 0, 8) == (1000, 500, True, 512, 8, 64, 128)


def test_slice_count_of_the_sphere_scene():
    # 400,000 points (1000 spheres of 400), the tuned 42 chunks: 1563 groups (781 symmetric
    # distances), or 1568 with eight waves per block (99 source-side slices)
    assert plan(400000, 42, 1) == (1563, 781, False, 782, 19, 42, 823)
    assert plan(400000, 42, 8) == (1568, 784, True, 792, 19, 42, 141)


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


# ----------------------------------------------------------------------------------------------
# Staging of a source tile spread over the block (shared-source shapes): 64 / W sources per wave,
# value v of lane `lane` (v = lane + 64 k, k < ceil(values / 64)) is field v // (64 / W) of source
# (64 / W) * wave + v % (64 / W); fields are the DIM coordinates, |l|^2, then the real and the
# imaginary parts of the RT charges, stored at field * STRIDE + E(p) and + DUP (E(p) = p for 64-point
# tiles; (p // 16) * 48 + p % 16 for 16-point sub-blocks).
@pytest.mark.parametrize("W", [1, 8])
@pytest.mark.parametrize("DIM,RT,sub16", [(2, 1, False), (2, 4, False), (3, 1, False), (3, 2, False),
                                          (3, 1, True), (3, 2, True), (3, 4, True)])
def test_tile_staging_stores_every_value_once(W, DIM, RT, sub16):
    src = 64 // W
    fields = DIM + 1 + 2 * RT
    nvals = src * fields
    regs = cdiv(nvals, 64)
    stride, dup = (192, 16) if sub16 else (128, 64)
    seen = collections.Counter()
    entries = collections.Counter()
    for wave in range(W):
        for lane in range(64):
            for k in range(regs):
                v = lane + 64 * k
                if v >= nvals:
                    continue
                f, p = v // src, src * wave + v % src
                seen[(f, p)] += 1
                e = f * stride + ((p >> 4) * 48 + (p & 15) if sub16 else p)
                entries[e] += 1
                entries[e + dup] += 1
                assert e - f * stride + dup < stride  # inside the field's array
    assert len(seen) == fields * 64 and set(seen.values()) == {1}
    assert set(entries.values()) == {1}  # no two values share an LDS entry
    if W == 8 and fields <= 8:
        assert regs == 1  # one register per lane carries the next tile during the products
