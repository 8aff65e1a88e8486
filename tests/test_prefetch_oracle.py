"""Pins of the predictor-row reference (oracle/prefetch.py) on hand-worked
cases: brick grid indexing, history shifts, features of bricks seen by a
simple camera, labels and candidates."""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import prefetch as opf


def _geo():
    V = oracle.make_volume((64, 64, 64), (1, 1, 1), 2, 16, 16, 3, (8, 8, 8), 3)
    return V, opf.Geometry(V)


def test_geometry_by_hand():
    V, G = _geo()
    assert G.per_channel == 64 + 8 + 1 and G.P == 64
    assert G.dense(1, 1, 1, 0, 1) == 73 + 64 + (1 * 2 + 0) * 2 + 1
    assert G.cover(0, 1, 3, 2, 1) == G.dense(0, 1, 1, 1, 0)
    assert G.cover(1, 2, 3, 3, 3) == 73 + 72
    assert tuple(G.nleaf) == (8, 8, 8)


def test_record_by_hand():
    hist = np.array([0x11, 0x88, 0x00, 0x01], np.uint8)
    counts = np.array([3, 0, 0, 0], np.uint32)
    res_slot = np.array([2, -1, 0, 1], np.int64)
    stamp = np.array([6, 7, 7], np.uint32)  # slots 0, 1, 2
    out = opf.record(hist, counts, res_slot, stamp, 7)
    # brick 0: 0x11 -> 0x22 | requested | read (slot 2 stamped 7) = 0x33
    # brick 1: oldest bits drop out, not resident -> 0
    # brick 2: slot 0 stamped 6 -> not read this frame
    # brick 3: 0x01 -> 0x02, slot 1 stamped 7 -> read
    assert out.tolist() == [0x33, 0x00, 0x00, 0x12]


def _cam(eye, ty=0.5, aspect=1.0):
    return dict(proj="persp", eye=list(eye), F=[0.0, 0.0, 1.0], R=[1.0, 0.0, 0.0], U=[0.0, 1.0, 0.0],
                tx=ty * aspect, ty=ty)


def test_features_by_hand():
    V, G = _geo()
    n_nodes = oracle.node_count(V)[0]
    meta = np.zeros((n_nodes, 2, 2), np.uint16)
    # brick (1,1,1) covers leaves x, y, z in {2, 3}; three of them reach raw 200
    for (gx, gy, gz) in [(2, 2, 2), (3, 2, 2), (3, 3, 3)]:
        meta[G.leaf_off + (gz * 8 + gy) * 8 + gx, 0] = (0, 200)
    for (gx, gy, gz) in [(2, 3, 2), (2, 2, 3)]:
        meta[G.leaf_off + (gz * 8 + gy) * 8 + gx, 0] = (0, 100)
    tf = np.zeros((256, 4), np.float32)
    tf[128:, 3] = 0.5  # entries >= 128 visible
    chans = [dict(c=0, W0=0, W1=255 * 256)]  # raw value r -> table entry r
    hist = np.zeros(2 * G.per_channel, np.uint8)
    p111 = (1 * 4 + 1) * 4 + 1
    hist[G.dense(0, 0, 1, 1, 1)] = 0b1010_0101
    res = np.full(2 * G.per_channel, -1, np.int64)
    res[G.dense(0, 1, 0, 0, 0)] = 5
    cam = _cam((24.0, 24.0, -76.0))
    X, amb = opf.features(G, cam, 100, 1.0, chans, tf[None], meta, hist, res)
    f = X[p111]  # channel 0, brick (1,1,1), centre (24, 24, 24), 100 ahead of the eye
    # one pixel at unit distance = 2 * 0.5 / 100; at t = 100 it covers 1 voxel: 16 px per brick
    assert f[0] == 0.5
    assert f[1] == -1.0 / 8.0  # D_1 = 2 / 0.01 = 200
    assert f[2] == 0.0 and f[3] == 1.0 and f[4] == 0.0 and f[5] == 0.0
    assert f[6] == 1.5 / 4.0
    assert f[7] == 3.0 / 8.0
    assert f[8:16].tolist() == [1, 0, 1, 0, 0, 1, 0, 1]
    assert f[16:24].tolist() == [0, 1, 0, 0, 0, 0, 0, 0]
    assert not amb[p111]
    # brick (3,1,1): centre (56, 24, 24), 32 to the right
    g = X[(1 * 4 + 1) * 4 + 3]
    t = math.hypot(32.0, 100.0)
    assert abs(g[0] - math.log2(16.0 / (t * 0.01)) / 8.0) < 1e-15
    assert abs(g[4] - 0.32) < 1e-15 and g[3] == 1.0
    # channel 1 is not shown: no leaf fraction
    assert X[G.P + p111][7] == 0.0
    # a camera past the volume looking further +z sees nothing
    Y, _ = opf.features(G, _cam((24.0, 24.0, 100.0)), 100, 1.0, chans, tf[None], meta, hist, res)
    assert Y[:, 3].sum() == 0
    # the desired level rises with distance: at t = 400, levels 1 (D=200) and 2 (D=400) are due
    Z, amb2 = opf.features(G, _cam((24.0, 24.0, -376.0)), 100, 1.0, chans, tf[None], meta, hist, res)
    assert Z[p111][2] == 2.0 / 8.0 and amb2[p111]  # t = 400 sits on the level-2 threshold


def test_labels_and_candidates_by_hand():
    V, G = _geo()
    hist = np.zeros(2 * G.per_channel, np.uint8)
    hist[G.dense(0, 1, 1, 0, 0)] = 0x10  # level-1 brick (1,0,0) of channel 0 read 1 frame ago
    y, m = opf.labels(G, hist)
    # the level-1 brick (1,0,0) covers L0 bricks x in {2,3}, y in {0,1}, z in {0,1}
    rows = [(pz * 4 + py) * 4 + px for pz in (0, 1) for py in (0, 1) for px in (2, 3)]
    assert y[:, 1].sum() == 8 and all(y[r, 1] == 1 for r in rows)
    assert y[:, [0, 2]].sum() == 0 and m[:, :3].all() and not m[:, 3:].any()
    z = np.full((2 * G.P, 16), -10.0)
    z[0, 0] = math.log(4.0)         # p = 0.8 for L0 brick (0,0,0)
    z[1, 1] = math.log(9.0)         # p = 0.9 for level-1 brick (0,0,0) ...
    z[0, 1] = math.log(3.0)         # ... which also gets 0.75 from row 0
    z[5, 2] = 0.0                   # p = 0.5: not above 0.5
    res = np.full(2 * G.per_channel, -1, np.int64)
    res[G.dense(0, 0, 0, 0, 0)] = 0  # resident: not a candidate
    best = opf.candidates(G, z, 0.5, res)
    assert set(best) == {int(G.dense(0, 1, 0, 0, 0))}
    assert abs(best[int(G.dense(0, 1, 0, 0, 0))] - 0.9) < 1e-12
