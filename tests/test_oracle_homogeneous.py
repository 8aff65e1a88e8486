"""Pins of the oracle's homogeneous-leaf rendering (Alg. 1 isHomogeneous /
renderAndSkipNode, read through the transfer function: a leaf whose whole
value range maps to one RGBA is rendered from its metadata, without voxels).

References: the interpolated table evaluated in exact rationals; the closed
form of a saturated constant volume with nothing resident; equality with the
plain rendering where every sample reads level 0."""
from __future__ import annotations

import math
from fractions import Fraction

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


def _plateau_tf(rng):
    """Piecewise-constant RGBA table: runs of random length, some with alpha 0."""
    tf = np.zeros((256, 4), np.float32)
    e = 0
    while e < 256:
        n = int(rng.integers(1, 40))
        val = rng.uniform(0, 1, 4).astype(np.float32)
        if rng.random() < 0.25:
            val[3] = 0.0
        tf[e:e + n] = val
        e += n
    return tf


def test_flatness_equals_constant_rgba_on_the_range():
    """[mn, mx] is homogeneous iff the interpolated RGBA is the same for every
    value in [mn, mx], with alpha non-zero.  RGBA is piecewise linear with
    breakpoints where the table position is an integer, so both ends and the
    breakpoints inside decide it (exact rationals)."""
    rng = np.random.default_rng(11)
    hits = 0
    for trial in range(80):
        tf = _plateau_tf(rng)
        raw_max = 255 if trial % 2 else 65535
        a, b = sorted(rng.integers(0, raw_max * 256, 2))
        if b - a < 64:
            b = a + 64
        W0, W1 = int(a), int(b)
        w0, w1 = Fraction(W0, 256), Fraction(W1, 256)
        for _ in range(40):
            mn, mx = sorted(int(x) for x in rng.integers(0, raw_max + 1, 2))
            if rng.random() < 0.5:
                mx = min(raw_max, mn + int(rng.integers(0, 3 * max(1, (b - a) // 256 // 255 + 1))))
            pts = {Fraction(mn), Fraction(mx)}
            for e in range(256):
                v = w0 + (w1 - w0) * Fraction(e, 255)
                if mn <= v <= mx:
                    pts.add(v)
            vals = {_rgba_exact(v, W0, W1, tf) for v in pts}
            flat = len(vals) == 1 and next(iter(vals))[3] != 0
            hits += flat
            assert oracle.tf_flat(mn, mx, W0, W1, tf) == flat, (W0, W1, mn, mx)
    assert hits > 50  # the case is exercised, not only its negation


def _axis_scene(vol):
    nz, ny, nx = vol.shape
    V = oracle.make_volume((nx, ny, nz), (1, 1, 1), 1, 8, 8, 1, (4, 4, 4), 2)
    lm = np.zeros((1, int(np.prod(oracle.node_count(V)[2][-1])), 2), np.uint16)
    lm[..., 0] = vol.min()
    lm[..., 1] = vol.max()
    return V, lm


@pytest.mark.parametrize("a", [0.05, 0.3])
def test_saturated_constant_volume_needs_no_bricks(a):
    """A constant volume above the window's top maps to the table's last
    entry everywhere: with homogeneous leaves on and nothing resident the
    image is the closed form A = 1 - (1-a)^n of the plain renderer with
    everything resident, and nothing is requested or read; with it off and
    nothing resident the image is empty and every sample requests."""
    vol = np.full((16, 16, 16), 200, np.uint8)
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = (0.2, 0.4, 0.6)
    tf[:, 3] = np.linspace(0, a, 256, dtype=np.float32)  # varies: only the clamped end is flat
    ch = [dict(c=0, lo=0, hi=0, W0=0, W1=100 * 256, tf=tf)]
    V, lm = _axis_scene(vol)
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    none = np.full(oracle.brick_count(V), -1, np.int32)
    fr, _ = oracle.make_frame(cam, 16, 16, 0.5, ch, homogeneous=True)
    r = oracle.render(V, [[vol]], none, lm, fr, 1)
    af = float(np.float32(a))
    n = min(32, math.ceil(math.log(0.01) / math.log(1 - af)))
    A = 1 - (1 - af) ** n
    assert np.allclose(r["rgba"][..., 3], A, atol=1e-12, rtol=0)
    assert np.allclose(r["rgba"][..., :3], np.array([0.2, 0.4, 0.6], np.float32).astype(np.float64) * A,
                       atol=1e-12, rtol=0)
    assert r["counts"].sum() == 0 and r["used"].sum() == 0
    fr0, _ = oracle.make_frame(cam, 16, 16, 0.5, ch)
    r0 = oracle.render(V, [[vol]], none, lm, fr0, 1)
    assert (r0["rgba"] == 0).all() and r0["counts"].sum() == 16 * 16 * 32
    full = np.arange(oracle.brick_count(V), dtype=np.int32)
    r1 = oracle.render(V, [[vol]], full, lm, fr0, oracle.brick_count(V))
    assert np.allclose(r1["rgba"], r["rgba"], atol=1e-12, rtol=0)


def _blob_scene():
    src = synth.config1_volume()
    leaf, depth = (8, 8, 8), 3
    V = oracle.make_volume(src.dims, src.spacing, 1, src.bits, 16, src.n_levels, leaf, depth)
    lm = src.leaf_minmax(0, leaf, leaf_grid(src.dims, leaf, depth))[None]
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = (0.9, 0.5, 0.1)
    tf[:16, 3] = np.linspace(0, 0.08, 16, dtype=np.float32)
    tf[16:, 3] = np.float32(0.08)  # a plateau: blob cores map to one RGBA
    W0, W1 = synth.window_fx(0.02 * 255, 0.4 * 255)  # 57 of 470 non-empty leaves homogeneous
    return src, V, lm, [dict(c=0, lo=0, hi=0, W0=W0, W1=W1, tf=tf)]


def test_equals_plain_rendering_where_level_0_is_read():
    """With every brick resident and level 0 desired, a homogeneous leaf's
    samples read values inside its exact metadata range, which the table maps
    to the plateau's RGBA: the image is the plain one (to FP64 rounding), with
    fewer voxel reads and no requests either way."""
    src, V, lm, ch = _blob_scene()
    full = np.arange(oracle.brick_count(V), dtype=np.int32)
    for cam in (synth.camera_ortho_axis((32, 32), 64, 64), synth.orbit_path(src.dims, src.spacing, 4)[1]):
        out = []
        for h in (False, True):
            fr, _ = oracle.make_frame(cam, 64, 64, 0.5, ch, homogeneous=h)
            out.append(oracle.render(V, src.levels, full, lm, fr, oracle.brick_count(V)))
        p, h = out
        assert np.abs(p["rgba"] - h["rgba"]).max() < 1e-12
        assert p["counts"].sum() == 0 and h["counts"].sum() == 0
        assert h["stats"]["channel_samples"] < 0.95 * p["stats"]["channel_samples"]


def test_requests_are_a_subset_of_the_plain_ones():
    """With only the coarsest level resident, homogeneous leaves request
    nothing: every brick's count is at most its plain count, and the total
    drops."""
    src, V, lm, ch = _blob_scene()
    _, _, nb = oracle.level_info(V)
    ids = oracle.dense_ids(V)
    res = np.full(oracle.brick_count(V), -1, np.int32)
    coarse = [i for i, x in enumerate(ids) if oracle.brick_id_decode(V.n_levels, int(x))[1] == V.n_levels - 1]
    res[coarse] = np.arange(len(coarse))
    cam = synth.orbit_path(src.dims, src.spacing, 4)[2]
    out = []
    for h in (False, True):
        fr, _ = oracle.make_frame(cam, 64, 64, 0.5, ch, homogeneous=h)
        out.append(oracle.render(V, src.levels, res, lm, fr, len(coarse)))
    p, h = out
    assert (h["counts"] <= p["counts"]).all()
    assert h["counts"].sum() < p["counts"].sum()
