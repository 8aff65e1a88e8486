"""Pins of the oracle's metadata-from-bricks pass (Sec. 5.3: a client whose
server has no metadata computes it from the voxels of fetched bricks).

The references here are written differently from the oracle: a brute force
over every voxel of the level that keeps those whose footprint in L0 voxels
meets the leaf box grown by one voxel of that level, and the generator's own
per-leaf metadata (the server's answer) at level 0."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import leaf_grid

DIMS, SPACING, B, LEAF, DEPTH, NL = (40, 36, 20), (1.0, 1.0, 2.0), 8, (4, 4, 2), 4, 3


def _scene(seed=0, n_ch=2):
    V = oracle.make_volume(DIMS, SPACING, n_ch, 16, B, NL, LEAF, DEPTH)
    d, f, nb = oracle.level_info(V)
    rng = np.random.default_rng(seed)
    levels = [[rng.integers(0, 65536, size=(d[l][2], d[l][1], d[l][0]), dtype=np.uint16) for l in range(NL)]
              for _ in range(n_ch)]
    ng = leaf_grid(DIMS, LEAF, DEPTH)
    unknown = np.zeros((n_ch, int(np.prod(ng)), 2), np.uint16)
    unknown[..., 1] = 65535
    return V, levels, unknown, ng, d, f, nb


def _ids(V, c, l, nb):
    return [oracle.brick_id(V.n_levels, c, l, x, y, z)
            for z in range(nb[l][2]) for y in range(nb[l][1]) for x in range(nb[l][0])]


def _brute(arr, f, d, ng, leaf, inside):
    """Per leaf: min/max over level voxels v whose L0 footprint
    [v f, (v + 1) f) meets [x0 - f, x1 + f) on every axis."""
    out = {}
    for lz in range(ng[2]):
        for ly in range(ng[1]):
            for lx in range(ng[0]):
                if not inside(lx, ly, lz):
                    continue
                keep = []
                for a, li in enumerate((lx, ly, lz)):
                    x0, x1, fa = li * leaf[a], (li + 1) * leaf[a], int(f[a])
                    keep.append([v for v in range(int(d[a])) if v * fa < x1 + fa and (v + 1) * fa > x0 - fa])
                k = (lz * ng[1] + ly) * ng[0] + lx
                if not all(keep):
                    out[k] = (0, 0)
                    continue
                sub = arr[np.ix_(keep[2], keep[1], keep[0])]
                out[k] = (int(sub.min()), int(sub.max()))
    return out


@pytest.mark.parametrize("level", [0, 1, 2])
def test_matches_brute_force_per_level(level):
    V, levels, unknown, ng, d, f, nb = _scene()
    got = oracle.leaf_meta_from_bricks(V, levels, unknown, _ids(V, 1, level, nb))
    ext = [int(nb[level][a]) * B * int(f[level][a]) for a in range(3)]  # the brick grid's L0 extent
    inside = lambda x, y, z: x * LEAF[0] < ext[0] and y * LEAF[1] < ext[1] and z * LEAF[2] < ext[2]
    ref = _brute(levels[1][level], f[level], d[level], ng, LEAF, inside)
    assert len(ref) > 0
    for k, mm in ref.items():
        assert tuple(int(x) for x in got[1, k]) == mm, (level, k)
    # leaves outside every brick and the other channel keep their values
    rest = np.ones(len(unknown[0]), bool)
    rest[list(ref)] = False
    assert np.array_equal(got[1, rest], unknown[1, rest])
    assert np.array_equal(got[0], unknown[0])


def test_level0_equals_the_servers_metadata():
    """At level 0 the result is the conservative leaf metadata the data
    server gives (L0 values within one voxel of the leaf, clamped)."""
    src = synth.config1_volume()
    leaf, depth = (8, 8, 8), 3
    V = oracle.make_volume(src.dims, src.spacing, 1, src.bits, 16, src.n_levels, leaf, depth)
    _, _, nb = oracle.level_info(V)
    lg = leaf_grid(src.dims, leaf, depth)
    start = np.zeros((1, int(np.prod(lg)), 2), np.uint16)
    start[..., 1] = 255
    got = oracle.leaf_meta_from_bricks(V, src.levels, start, _ids(V, 0, 0, nb))
    assert np.array_equal(got[0], src.leaf_minmax(0, leaf, lg))


def test_finest_level_wins_in_any_order():
    V, levels, unknown, ng, d, f, nb = _scene(seed=3)
    fine = _ids(V, 0, 0, nb)[:5]
    coarse = _ids(V, 0, 1, nb)
    only_fine = oracle.leaf_meta_from_bricks(V, levels, oracle.leaf_meta_from_bricks(V, levels, unknown, coarse),
                                             fine)
    for order in (fine + coarse, coarse + fine, coarse[::-1] + fine[::-1]):
        assert np.array_equal(oracle.leaf_meta_from_bricks(V, levels, unknown, order), only_fine)


def test_coarse_estimate_is_within_the_fine_range_for_averaged_levels():
    """With levels made by 2x averaging (as the generators do), a coarse
    level's range of a leaf lies within the range of the L0 voxels its
    dilated box covers: the estimate can only miss extremes."""
    src = synth.config1_volume()
    leaf, depth = (8, 8, 8), 3
    V = oracle.make_volume(src.dims, src.spacing, 1, src.bits, 16, src.n_levels, leaf, depth)
    _, f, nb = oracle.level_info(V)
    lg = leaf_grid(src.dims, leaf, depth)
    start = np.zeros((1, int(np.prod(lg)), 2), np.uint16)
    l1 = oracle.leaf_meta_from_bricks(V, src.levels, start, _ids(V, 0, 1, nb))[0]
    a = src.levels[0][0]
    for k in range(len(l1)):
        lx, ly, lz = k % lg[0], (k // lg[0]) % lg[1], k // (lg[0] * lg[1])
        # L0 voxels under the level-1 box: one level-1 voxel (2 L0) beyond the leaf
        sl = [slice(max(i * leaf[ax] - 2, 0), min((i + 1) * leaf[ax] + 2, a.shape[2 - ax]))
              for ax, i in enumerate((lx, ly, lz))]
        sub = a[sl[2], sl[1], sl[0]]
        assert sub.min() <= l1[k, 0] <= l1[k, 1] <= sub.max()


def test_metadata_levels_across_calls_equal_one_call():
    """With the per-leaf metadata level, splitting the bricks over calls in
    any order (finest first, coarsest first, interleaved) gives the result
    of one call over all of them (finest wins), and each leaf's level is the
    finest level of a brick covering it (255 where none does).  Without the
    levels a later coarser call would overwrite finer metadata."""
    V, levels, unknown, ng, d, f, nb = _scene(seed=5)
    fine = _ids(V, 0, 0, nb)[::3] + _ids(V, 1, 0, nb)[:4]
    mid = _ids(V, 0, 1, nb)[::2]
    coarse = _ids(V, 0, 2, nb) + _ids(V, 1, 2, nb)
    lvl0 = np.full(unknown.shape[:2], 255, np.uint8)
    one, one_lvl = oracle.leaf_meta_from_bricks(V, levels, unknown, fine + mid + coarse, lvl0)
    assert np.array_equal(one, oracle.leaf_meta_from_bricks(V, levels, unknown, fine + mid + coarse))
    for parts in ((fine, mid, coarse), (coarse, mid, fine), (mid, fine, coarse), (coarse, fine, mid)):
        mm, lv = unknown, lvl0
        for p in parts:
            mm, lv = oracle.leaf_meta_from_bricks(V, levels, mm, p, lv)
        assert np.array_equal(mm, one) and np.array_equal(lv, one_lvl)
    # the levels are the finest covering brick's
    for ids, l in ((coarse, 2), (mid, 1), (fine, 0)):
        _, lv = oracle.leaf_meta_from_bricks(V, levels, unknown, ids, lvl0)
        assert set(np.unique(lv)) <= {l, 255} and (lv == l).any()
    # a coarser call after a finer one changes nothing where the finer one reached
    mm_f, lv_f = oracle.leaf_meta_from_bricks(V, levels, unknown, fine, lvl0)
    mm_fc, lv_fc = oracle.leaf_meta_from_bricks(V, levels, mm_f, coarse, lv_f)
    hit = lv_f == 0
    assert hit.any() and np.array_equal(mm_fc[hit], mm_f[hit]) and (lv_fc[hit] == 0).all()
    plain = oracle.leaf_meta_from_bricks(V, levels, mm_f, coarse)
    assert not np.array_equal(plain[hit], mm_f[hit])  # what the levels prevent
