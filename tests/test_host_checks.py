"""Host-side helpers of the GPU parity tests, checked on the CPU.

The complete tile-list check of the GPU tests expands the records' rectangles
into per-tile lists on the host; here that expansion is compared with the
oracle's own tile lists (explicit per-Gaussian tile enumeration), on two pairs
so the per-pair offsets are exercised, and a planted mistake must fail it.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Grid

from gpu_common import assert_lists_complete, lists_from_rects


def _records(b, g):
    """The L dict of gpu_lists, filled from the oracle (rectangles, keys) for
    every pair of the batch, and the oracle's per-tile lists."""
    sc = b.scenes[0]
    rects, keys, ref = [], [], []
    for p in b.pairs:
        tu0, ntu, tv0, ntv, _ = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
        rects.append(np.stack([tu0, ntu, tv0, ntv], 1))
        keys.append(oracle.depth_key32(sc.means, p.rx))
        lists, lkeys, _ = oracle.tile_lists(sc.means, sc.log_scales, p.rx, g)
        ref.append((lists, lkeys))
    P, T = len(b.pairs), g.n_tiles
    base = np.arange(P + 1, dtype=np.int64) * sc.n
    L = dict(base=base, T=T, rec_rect=np.concatenate(rects).astype(np.int64),
             rec_key=np.concatenate(keys).astype(np.uint32))
    # the GPU's sorted arrays: the oracle's lists laid out tile after tile
    ts, te, klo, val, pos = [], [], [], [], 0
    for lists, lkeys in ref:
        for t in range(T):
            ts.append(pos)
            pos += len(lists[t])
            te.append(pos)
            val.append(lists[t])
            klo.append(lkeys[t])
    L.update(ts=np.array(ts, np.int64), te=np.array(te, np.int64),
             klo=np.concatenate(klo).astype(np.uint32), val=np.concatenate(val).astype(np.uint32))
    return L, ref


@pytest.mark.parametrize("tw,th", [(8, 8), (16, 4)])
def test_host_list_expansion_matches_oracle_tile_lists(tw, th):
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=tw, tile_h=th)
    b = synth.tiny(grid=g, n=600)
    b.pairs.append(synth.Pair(np.array([2.5, 1.0, 2.0]), b.pairs[0].tx, b.pairs[0].freq_hz, 0))
    L, ref = _records(b, g)
    tile, key, gid = lists_from_rects(L, g.n_tiles_az, [0] * len(b.pairs))
    for k, (lists, lkeys) in enumerate(ref):
        for t in range(g.n_tiles):
            m = tile == k * g.n_tiles + t
            np.testing.assert_array_equal(gid[m], lists[t])
            np.testing.assert_array_equal(key[m], lkeys[t])
    lens = assert_lists_complete(L, g.n_tiles_az, [0] * len(b.pairs))
    assert lens.sum() > 0


def test_host_list_check_catches_planted_mistakes():
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=8, tile_h=8)
    b = synth.tiny(grid=g, n=600)
    L, _ = _records(b, g)
    nz = np.nonzero(L["te"] - L["ts"] >= 2)[0]
    t = int(nz[0])
    swapped = dict(L, val=L["val"].copy())          # two entries of one list out of order
    a = int(L["ts"][t])
    swapped["val"][[a, a + 1]] = swapped["val"][[a + 1, a]]
    with pytest.raises(AssertionError):
        assert_lists_complete(swapped, g.n_tiles_az, [0])
    moved = dict(L, te=L["te"].copy(), ts=L["ts"].copy())   # one entry counted in the next tile
    moved["te"][t] -= 1
    moved["ts"][t + 1] -= 1
    with pytest.raises(AssertionError):
        assert_lists_complete(moved, g.n_tiles_az, [0])
