"""Pins of the oracle's render-and-skip leaves (Alg. 1 isHomogeneous /
renderAndSkipNode; Sec. 6.1: a node is rendered from its value only when it
is homogeneous for all channels).  A channel is homogeneous in a leaf when
its metadata hold one value (min == max); a leaf where every visible channel
is empty or homogeneous, and one is not empty, is rendered from those values
without bricks.

References: the closed form of a constant multi-channel volume with nothing
resident (per-channel table values in exact rationals); exact equality with
the plain rendering where level 0 is read with exact metadata; a leaf
homogeneous in only some channels changes nothing at all (every channel
still samples its brick); request and read sets only shrink."""
from __future__ import annotations

import math
from fractions import Fraction
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import leaf_grid


def _rgba_exact(v: Fraction, W0, W1, tf):
    w0, w1 = Fraction(W0, 256), Fraction(W1, 256)
    x = min(max((v - w0) / (w1 - w0), Fraction(0)), Fraction(1))
    p = 255 * x
    i0 = min(int(math.floor(p)), 255)
    i1 = min(i0 + 1, 255)
    fr = p - i0
    return tuple(Fraction(float(tf[i0, k])) * (1 - fr) + Fraction(float(tf[i1, k])) * fr for k in range(4))


def _exact_meta(arrays, leaf, depth):
    """Exact dilated leaf [min, max] per channel (the blob server's answer)."""
    nz, ny, nx = arrays[0].shape
    ns = SimpleNamespace(levels=[[a] for a in arrays])
    grid = leaf_grid((nx, ny, nz), leaf, depth)
    return np.stack([synth.BlobVolume.leaf_minmax(ns, c, leaf, grid) for c in range(len(arrays))])


def _ramp(rgb, a):
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = rgb
    tf[:, 3] = np.linspace(0, a, 256, dtype=np.float32)
    return tf


@pytest.mark.parametrize("alphas", [(0.04, 0.02), (0.5, 0.3)])
def test_constant_channels_closed_form(alphas):
    """Two constant channels (values 200 and 90) with nothing resident: every
    leaf is homogeneous in both, so each of the n samples of an axis ray is
    the mix of the two table values, and the image is the closed form
    A = 1 - (1 - a_s)^n, C = C_s (1 - (1 - a_s)^n) / a_s, with n cut at the
    first sample where A >= 0.99; nothing is requested or read.  With the
    option off the image is empty and every channel-sample requests."""
    vals = (200, 90)
    arr = [np.full((16, 16, 16), v, np.uint8) for v in vals]
    V = oracle.make_volume((16, 16, 16), (1, 1, 1), 2, 8, 8, 1, (4, 4, 4), 2)
    lm = _exact_meta(arr, (4, 4, 4), 2)
    chans = [dict(c=c, lo=0, hi=0, W0=0, W1=255 * 256, tf=_ramp(rgb, a))
             for c, (rgb, a) in enumerate(zip(((0.2, 0.4, 0.6), (0.9, 0.1, 0.3)), alphas))]
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    none = np.full(oracle.brick_count(V), -1, np.int32)
    fr, _ = oracle.make_frame(cam, 16, 16, 0.5, chans, homogeneous=True)
    r = oracle.render(V, [[a] for a in arr], none, lm, fr, 1)
    ch = [_rgba_exact(Fraction(v), c["W0"], c["W1"], c["tf"]) for v, c in zip(vals, chans)]
    a_s = 1 - (1 - ch[0][3]) * (1 - ch[1][3])
    Cs = [a_s * (ch[0][3] * ch[0][k] + ch[1][3] * ch[1][k]) / (ch[0][3] + ch[1][3]) for k in range(3)]
    n = 32  # samples at z = -1/4 + k/2 inside [0, 16)
    for i in range(1, 33):
        if 1 - (1 - a_s) ** i >= Fraction(99, 100):
            n = i
            break
    A = 1 - (1 - a_s) ** n
    assert np.allclose(r["rgba"][..., 3], float(A), atol=1e-12, rtol=0)
    for k in range(3):
        assert np.allclose(r["rgba"][..., k], float(Cs[k] * A / a_s), atol=1e-12, rtol=0)
    assert r["counts"].sum() == 0 and r["used"].sum() == 0
    assert r["stats"]["channel_samples"] == 0
    fr0, _ = oracle.make_frame(cam, 16, 16, 0.5, chans)
    r0 = oracle.render(V, [[a] for a in arr], none, lm, fr0, 1)
    assert (r0["rgba"] == 0).all() and r0["counts"].sum() == 16 * 16 * 32 * 2


def _noise_channel(shape, seed):
    """Values 40..250 that vary inside every 4^3 leaf (no leaf is empty for a
    table with alpha > 0 from entry 1 on, none is homogeneous)."""
    rng = np.random.default_rng(seed)
    return rng.integers(40, 251, shape).astype(np.uint8)


@pytest.mark.parametrize("partial", [False, True])
def test_leaf_homogeneous_in_some_channels_samples_every_channel(partial):
    """Channel 0 is constant (homogeneous in every leaf), channel 1 varies in
    every leaf: no leaf is homogeneous for all channels, so the option changes
    nothing: images bit-identical, the same request multiset, the same read
    set, and channel 0's bricks are read.  With everything resident at level 0
    and with a random half resident over levels 0..2."""
    arr = [np.full((32, 32, 32), 150, np.uint8), _noise_channel((32, 32, 32), 3)]
    src = synth.ArrayVolume(arr, 8, (1, 1, 1), 3)
    V = oracle.make_volume(src.dims, src.spacing, 2, 8, 8, 3, (4, 4, 4), 3)
    lm = _exact_meta(arr, (4, 4, 4), 3)
    assert (lm[0, :, 0] == lm[0, :, 1]).all() and (lm[1, :, 0] < lm[1, :, 1]).all()
    nb = oracle.brick_count(V)
    if partial:
        res = np.full(nb, -1, np.int32)
        pick = np.nonzero(np.random.default_rng(4).random(nb) < 0.5)[0]
        res[pick] = np.arange(len(pick))
        hi = 2
    else:
        ids = oracle.dense_ids(V)
        res = np.full(nb, -1, np.int32)
        l0 = [i for i, x in enumerate(ids) if oracle.brick_id_decode(V.n_levels, int(x))[1] == 0]
        res[l0] = np.arange(len(l0))
        hi = 0
    chans = [dict(c=c, lo=0, hi=hi, W0=0, W1=255 * 256, tf=_ramp(rgb, 0.05))
             for c, rgb in enumerate(((0.2, 0.4, 0.6), (0.9, 0.1, 0.3)))]
    cam = synth.camera_persp((70.0, 55.0, 48.0), (16, 15, 17), (0, 0, 1), 45.0, 1.0)
    out = []
    for h in (False, True):
        fr, _ = oracle.make_frame(cam, 48, 48, 0.5, chans, lod_bias=0.6, homogeneous=h)
        out.append(oracle.render(V, src.levels, res, lm, fr, nb))
    p, h = out
    assert np.array_equal(p["rgba"], h["rgba"])
    assert np.array_equal(p["counts"], h["counts"]) and np.array_equal(p["used"], h["used"])
    ch0_slots = res[:nb // 2][res[:nb // 2] >= 0]
    assert h["used"][ch0_slots].any()


def _plateau_scene(leaf=(4, 4, 4), depth=4, n_channels=2):
    src = synth.plateau_volume(n_channels)
    V = oracle.make_volume(src.dims, src.spacing, n_channels, 8, 16, src.n_levels, leaf, depth)
    lm = _exact_meta([src.levels[c][0] for c in range(n_channels)], leaf, depth)
    chans = []
    for c in range(n_channels):
        tf = synth.tf_hue(c / n_channels, 0.06)
        tf[:, 3] = np.maximum(tf[:, 3], np.float32(0.004))  # a haze: value 0 is visible (not empty)
        chans.append(dict(c=c, lo=0, hi=src.n_levels - 1, W0=0, W1=255 * 256, tf=tf))
    return src, V, lm, chans


def test_render_and_skip_equals_plain_at_level_0():
    """Constant boxes on a visible zero background: with exact dilated
    metadata, a leaf homogeneous in both channels holds its value on every
    voxel a sample in it interpolates, so where level 0 is read the image is
    the plain one (FP64 rounding aside), with fewer brick reads and no
    requests either way."""
    src, V, lm, chans = _plateau_scene()
    hom = (lm[:, :, 0] == lm[:, :, 1]).all(axis=0)
    assert 0.3 < hom.mean() < 0.9
    full = np.arange(oracle.brick_count(V), dtype=np.int32)
    ch0 = [dict(ch, hi=0) for ch in chans]
    for cam in (synth.camera_ortho_axis((32, 32), 64, 64), synth.orbit_path(src.dims, src.spacing, 4)[1]):
        out = []
        for h in (False, True):
            fr, _ = oracle.make_frame(cam, 64, 64, 0.5, ch0, homogeneous=h)
            out.append(oracle.render(V, src.levels, full, lm, fr, oracle.brick_count(V)))
        p, h = out
        assert np.abs(p["rgba"] - h["rgba"]).max() < 1e-12
        assert p["counts"].sum() == 0 and h["counts"].sum() == 0
        assert h["stats"]["channel_samples"] < 0.7 * p["stats"]["channel_samples"]
        assert h["stats"]["samples"] == p["stats"]["samples"]


def test_requests_and_reads_only_shrink():
    """Only the coarsest level resident, levels 0..2 desired: render-and-skip
    leaves neither request nor read, so every brick's count is at most its
    plain count, the read set is a subset, and the totals drop; with unknown
    metadata ([0, max]) no leaf qualifies and nothing changes."""
    src, V, lm, chans = _plateau_scene()
    ids = oracle.dense_ids(V)
    res = np.full(oracle.brick_count(V), -1, np.int32)
    coarse = [i for i, x in enumerate(ids) if oracle.brick_id_decode(V.n_levels, int(x))[1] == V.n_levels - 1]
    res[coarse] = np.arange(len(coarse))
    cam = synth.orbit_path(src.dims, src.spacing, 4)[2]
    for meta, shrink in ((lm, True), (np.stack([np.zeros_like(lm[..., 0]), np.full_like(lm[..., 1], 255)], -1), False)):
        out = []
        for h in (False, True):
            fr, _ = oracle.make_frame(cam, 64, 64, 0.5, chans, lod_bias=0.8, homogeneous=h)
            out.append(oracle.render(V, src.levels, res, meta, fr, len(coarse)))
        p, h = out
        if shrink:
            assert (h["counts"] <= p["counts"]).all() and h["counts"].sum() < p["counts"].sum()
            assert (h["used"] <= p["used"]).all()
        else:
            assert np.array_equal(p["rgba"], h["rgba"]) and np.array_equal(p["counts"], h["counts"])
            assert np.array_equal(p["used"], h["used"])
