"""Host-side checks of the persistent batched form's work order (no GPU).

The persistent kernel takes items from one queue in table order and lets an
item of phase p start once every tile of its planes' phases < p has
finished.  It drains the queue whatever the number of resident work-groups
only if every item's dependencies come earlier in the table; these tests
check that property of the order the library builds, that every (volume,
phase, tile) is listed exactly once, that paired tiles share their row
segment (both halves of a work-group then execute the same barriers), and
that merged volumes advance together.
"""
import ctypes

import numpy as np
import pytest

from paper_1503_07998_amd import _native as N


def order(planes, nseg, nstrip, pair, per_iter, iters, window=0):
    lib = N.lib()
    lib.mvd_internal_pq_order.restype = ctypes.c_long
    n = len(planes)
    arr = lambda v: (ctypes.c_int * n)(*v)
    args = [n, arr(planes), arr(nseg), arr(nstrip), arr(pair), arr(per_iter), arr(iters), window]
    cnt = lib.mvd_internal_pq_order(*args, None, 0)
    assert cnt > 0
    out = (ctypes.c_int * (4 * cnt))()
    assert lib.mvd_internal_pq_order(*args, out, cnt) == cnt
    return np.frombuffer(out, dtype=np.int32).reshape(cnt, 4)


CASES = [
    # planes, nseg, nstrip, pair, per_iter, iters, window
    ([3], [1], [1], [1], [3], [2], 0),
    ([200, 300, 150], [3, 1, 4], [1, 2, 1], [1, 1, 0], [4, 6, 8], [10, 10, 10], 0),
    ([7, 5], [2, 1], [3, 2], [1, 0], [3, 4], [2, 3], 2),
    ([512], [1], [1], [1], [3], [10], 64),
    ([4, 9, 1], [5, 1, 2], [1, 1, 1], [1, 1, 1], [2, 6, 4], [0, 1, 3], 3),
]


@pytest.mark.parametrize("planes,nseg,nstrip,pair,per_iter,iters,window", CASES)
def test_every_tile_once_and_dependencies_first(planes, nseg, nstrip, pair, per_iter, iters, window):
    it = order(planes, nseg, nstrip, pair, per_iter, iters, window)
    ntiles = [s * t for s, t in zip(nseg, nstrip)]
    want = sum(p * n * (1 + pi * k) for p, n, pi, k in zip(planes, ntiles, per_iter, iters))
    seen = set()
    done = {}   # (job, plane, phase) -> tiles listed so far
    for j, p, b0, b1 in it.tolist():
        assert 0 <= j < len(planes) and 0 <= p < 1 + per_iter[j] * iters[j]
        tiles = [b0] + ([b1] if b1 >= 0 else [])
        if not pair[j]:
            assert b1 == -1
        else:   # both tiles in one row segment: the same barrier sequence
            segs = {(b // nstrip[j]) % nseg[j] for b in tiles}
            assert len(segs) == 1
        for b in tiles:
            assert 0 <= b < planes[j] * ntiles[j]
            assert (j, p, b) not in seen, "a tile is listed twice"
            seen.add((j, p, b))
            y = b // ntiles[j]
            for q in range(p):   # every tile of every earlier phase of this plane is listed before
                assert done.get((j, y, q), 0) == ntiles[j], (j, p, b, q)
        for b in tiles:
            key = (j, b // ntiles[j], p)
            done[key] = done.get(key, 0) + 1
    assert len(seen) == want


def test_merged_volumes_advance_together():
    it = order([200, 300, 150], [3, 1, 4], [1, 2, 1], [1, 1, 0], [4, 6, 8], [10, 10, 10])
    n = len(it)
    for j in range(3):
        pos = np.nonzero(it[:, 0] == j)[0]
        # each volume's items spread over the whole table, not one after another
        assert pos[0] < 0.01 * n and pos[-1] > 0.99 * n
        frac = np.arange(len(pos)) / len(pos)
        assert np.abs(pos / n - frac).max() < 0.01


def test_windows_finish_planes_before_later_ones_start():
    it = order([12], [1], [2], [1], [3], [2], window=4)
    first_of, last_of = {}, {}
    for i, (j, p, b0, b1) in enumerate(it.tolist()):
        for b in (b0, b1):
            if b < 0:
                continue
            y = b // 2
            first_of.setdefault(y, i)
            last_of[y] = i
    for w0 in (0, 4):
        assert max(last_of[y] for y in range(w0, w0 + 4)) < min(first_of[y] for y in range(w0 + 4, w0 + 8))
