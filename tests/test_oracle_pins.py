"""Pins of the CPU oracle against things other than itself: closed forms,
library routines, brute force on tiny inputs and the paper's invariants.

Paper sections cited: Sec. 3 (partial / full mapping and their propagation),
Sec. 5.3 (incremental residency update and LRU eviction), Sec. 7 (brick ID
layout), Sec. 6.1 / Alg. 1 (per-sample traversal, requests, substitution),
Sec. 6.2 (per-channel resolution ranges)."""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.ndimage import map_coordinates

import oracle
import synth
from tests.helpers import leaf_grid, single_sample_camera

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ brick IDs

def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_brick_id_golden():
    """Sec. 7: 24 bits of spatial offset (8 each for x, y, z) and 8 bits of
    page-table ID for (m x k) <= 256 page tables."""
    for row in _read_golden("brick_ids.txt"):
        k, c, l, bx, by, bz, expect = (int(x, 0) for x in row)
        assert oracle.brick_id(k, c, l, bx, by, bz) == expect
        assert oracle.brick_id_decode(k, expect) == (c, l, bx, by, bz)


@given(st.integers(1, 16), st.integers(0, 15), st.integers(0, 15), st.integers(0, 255),
       st.integers(0, 255), st.integers(0, 255))
@settings(max_examples=200, deadline=None)
def test_brick_id_roundtrip(k, c, l, bx, by, bz):
    l = l % k
    if c * k + l > 255:
        return
    i = oracle.brick_id(k, c, l, bx, by, bz)
    assert 0 <= i < 2 ** 32
    assert oracle.brick_id_decode(k, i) == (c, l, bx, by, bz)


# ------------------------------------------------------ level / tree shape

@pytest.mark.parametrize("dims,spacing,L,B,leaf,depth,C,bricks_per_ch,nodes,zdims", [
    ((64, 64, 64), (1, 1, 1), 3, 16, (8, 8, 8), 3, 1, 73, 585, [64, 32, 16]),
    ((2048, 2048, 64), (1, 1, 4), 7, 32, (16, 16, 4), 7, 4, 10837, 299605,
     [64, 64, 64, 32, 16, 8, 4]),
    ((8192, 8192, 192), (1, 1, 3), 9, 32, (16, 16, 8), 9, 16, 506197, None,
     [192, 192, 96, 48, 24, 12, 6, 3, 2]),
])
def test_level_and_tree_shapes(dims, spacing, L, B, leaf, depth, C, bricks_per_ch, nodes, zdims):
    V = oracle.make_volume(dims, spacing, C, 16, B, L, leaf, depth)
    d, f, nb = oracle.level_info(V)
    assert list(d[:, 2]) == zdims
    assert oracle.brick_count(V) == C * bricks_per_ch
    # the generator's own level schedule (a separate implementation) agrees
    sd, sf, _ = synth.level_schedule(dims, spacing, L)
    assert [tuple(x) for x in d] == [tuple(x) for x in sd]
    assert [tuple(x) for x in f] == [tuple(x) for x in sf]
    # brick IDs fit: at most 256 bricks per axis, m*k <= 256
    assert nb.max() <= 256 and C * L <= 256
    if nodes is not None:
        assert oracle.node_count(V)[0] == nodes


# ------------------------------------------------ sampling, TF, compositing

def _scene_V(levels, bits, B, leaf, depth, spacing=(1, 1, 1)):
    nz, ny, nx = levels[0][0].shape
    return oracle.make_volume((nx, ny, nz), spacing, len(levels), bits, B, len(levels[0]), leaf,
                              depth)


def _all_resident(V):
    return np.arange(oracle.brick_count(V), dtype=np.int32)


def _leaf_mm_full(V, levels):
    """Leaf metadata covering the full value range (nothing is empty)."""
    _, _, n = oracle.node_count(V)
    nl = int(np.prod(n[-1]))
    mm = np.zeros((V.n_channels, nl, 2), np.uint16)
    mm[:, :, 1] = 65535 if V.bits == 16 else 255
    return mm


def _probe(levels, bits, point, chans, lo=0, hi=0, B=4, leaf=(4, 4, 4), depth=2, res=None,
           leaf_mm=None):
    """A of a single-sample ray at `point` through O1."""
    V = _scene_V(levels, bits, B, leaf, depth)
    fr, keep = oracle.make_frame(single_sample_camera(point), 1, 1, 1000.0, chans)
    r = oracle.render(V, levels, _all_resident(V) if res is None else res,
                      _leaf_mm_full(V, levels) if leaf_mm is None else leaf_mm, fr,
                      oracle.brick_count(V))
    return r["rgba"][0, 0]


def test_trilinear_matches_library_routine():
    """Trilinear with voxel centres at i+1/2 and clamp-to-edge equals
    scipy.ndimage.map_coordinates(order=1, mode='nearest') at u - 1/2."""
    rng = np.random.default_rng(5)
    a = rng.integers(0, 65536, size=(7, 9, 10)).astype(np.uint16)  # ragged dims
    levels = [[a]]
    ramp = synth.tf_ramp()
    W0, W1 = 0, 65535 * 256
    ch = [dict(c=0, lo=0, hi=0, W0=W0, W1=W1, tf=ramp)]
    pts = np.stack([rng.uniform(0, 10, 60), rng.uniform(0, 9, 60), rng.uniform(0, 7, 60)], 1)
    pts = np.vstack([pts, [[0.1, 0.2, 0.3], [9.9, 8.9, 6.9], [0.5, 0.5, 0.5]]])
    for p in pts:
        A = _probe(levels, 16, p, ch, depth=2)[3]
        ref = map_coordinates(a.astype(np.float64), [[p[2] - 0.5], [p[1] - 0.5], [p[0] - 0.5]],
                              order=1, mode="nearest")[0]
        # single sample: A = alpha = TF ramp at x = v / 65535 (table in fp32)
        assert abs(A * 65535.0 - ref) < 0.02, (p, A * 65535, ref)


def test_centre_sample_is_mean_of_eight():
    a = np.array([[[10, 20], [30, 40]], [[50, 60], [70, 80]]], dtype=np.uint8)
    ch = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=synth.tf_ramp())]
    A = _probe([[a]], 8, (1.0, 1.0, 1.0), ch, B=2, leaf=(1, 1, 1), depth=1)[3]
    assert abs(A * 255.0 - 45.0) < 1e-4


def test_trilinear_reproduces_linear_field():
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    a = (1000 + 300 * x + 200 * y + 500 * z).astype(np.uint16)
    ch = [dict(c=0, lo=0, hi=0, W0=0, W1=65535 * 256, tf=synth.tf_ramp())]
    rng = np.random.default_rng(2)
    for _ in range(30):
        p = rng.uniform([0.5, 0.5, 0.5], [7.5, 6.5, 5.5])  # interior: no clamping
        A = _probe([[a]], 16, p, ch, B=4, leaf=(4, 4, 2), depth=2)[3]
        expect = 1000 + 300 * (p[0] - 0.5) + 200 * (p[1] - 0.5) + 500 * (p[2] - 0.5)
        assert abs(A * 65535.0 - expect) < 0.02


def _const_tf(rgb, a):
    t = np.zeros((256, 4), np.float32)
    t[:, 0], t[:, 1], t[:, 2], t[:, 3] = rgb[0], rgb[1], rgb[2], a
    return t


@pytest.mark.parametrize("a", [0.05, 0.2, 0.5])
def test_constant_volume_closed_form(a):
    """Constant per-sample alpha a over N samples: A = 1 - (1-a)^N,
    C = rgb A; early termination after k* = ceil(ln(0.01)/ln(1-a)) samples."""
    vol = np.full((16, 16, 16), 128, np.uint8)
    tf = _const_tf((0.2, 0.4, 0.6), a)
    af = float(np.float32(a))
    ch = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf)]
    V = _scene_V([[vol]], 8, 8, (4, 4, 4), 2)
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    fr, keep = oracle.make_frame(cam, 16, 16, 0.5, ch, term_alpha=0.99)
    r = oracle.render(V, [[vol]], _all_resident(V), _leaf_mm_full(V, [[vol]]), fr,
                      oracle.brick_count(V), aov=True)
    n_in = 32  # z = -0.25 + 0.5 k inside [0, 16) for k = 1..32
    kstar = math.ceil(math.log(0.01) / math.log(1 - af))
    n = min(n_in, kstar)
    A = 1 - (1 - af) ** n
    rgb = np.array([np.float32(0.2), np.float32(0.4), np.float32(0.6)], dtype=np.float64)
    assert np.allclose(r["rgba"][..., 3], A, atol=1e-12, rtol=0)
    assert np.allclose(r["rgba"][..., :3], rgb * A, atol=1e-12, rtol=0)
    assert (r["aov"][..., 0] == n).all()


@pytest.mark.parametrize("side", [-1, 0, 1])
def test_close_termination_call_has_both_outcomes(side):
    """Early termination (A >= alpha_term after a sample) decided within the
    margin of alpha_term: both outcomes are valid images, so the pixel is not
    ambiguous; the oracle keeps the other one.  Constant alpha a: after n
    samples A_n = 1 - (1-a)^n.  With alpha_term at A_8 (side 0) or just
    below it (side -1) this oracle stops after 8 samples and the other
    outcome is one more sample, A_9; just above it (side +1) it stops after 9
    and the other outcome is A_8.  Colours are rgb * A."""
    a = 0.2
    af = float(np.float32(a))
    vol = np.full((16, 16, 16), 128, np.uint8)
    tf = _const_tf((0.2, 0.4, 0.6), a)
    ch = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf)]
    V = _scene_V([[vol]], 8, 8, (4, 4, 4), 2)
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    A8, A9 = 1 - (1 - af) ** 8, 1 - (1 - af) ** 9
    term = float(np.nextafter(A8, 2.0 * side)) if side else A8
    fr, keep = oracle.make_frame(cam, 16, 16, 0.5, ch, term_alpha=0.99, term_margin=1e-6)
    fr.term_alpha = term
    r = oracle.render(V, [[vol]], _all_resident(V), _leaf_mm_full(V, [[vol]]), fr, oracle.brick_count(V))
    first, other = (A9, A8) if side > 0 else (A8, A9)
    rgb = np.array([np.float32(0.2), np.float32(0.4), np.float32(0.6)], dtype=np.float64)
    assert (r["amb_pix"] == 0).all() and (r["alt_pix"] == 1).all()
    assert np.allclose(r["rgba"][..., 3], first, atol=1e-12, rtol=0)
    assert np.allclose(r["alt_rgba"][..., 3], other, atol=1e-12, rtol=0)
    assert np.allclose(r["alt_rgba"][..., :3], rgb * other, atol=1e-12, rtol=0)
    # far from the threshold there is one outcome
    fr.term_alpha = 0.5 * (A8 + A9)
    r = oracle.render(V, [[vol]], _all_resident(V), _leaf_mm_full(V, [[vol]]), fr, oracle.brick_count(V))
    assert (r["alt_pix"] == 0).all() and np.allclose(r["rgba"][..., 3], A9, atol=1e-12, rtol=0)


@pytest.mark.parametrize("a", [0.05, 0.2, 0.5])
def test_adaptive_step_constant_volume_closed_form(a):
    """LOD-adaptive step (Sec. 6.1: the sampling distance may grow with the
    level): with the level fixed at 1 (x factor r = 2) only the samples
    k = 2, 4, .., 32 are taken, each with opacity 1 - (1-a)^2, so
    A = 1 - (1-a)^(2n) with n = min(16, ceil(ln 0.01 / (2 ln(1-a))))."""
    l0 = np.full((16, 16, 16), 128, np.uint8)
    l1 = np.full((8, 8, 8), 128, np.uint8)
    tf = _const_tf((0.2, 0.4, 0.6), a)
    af = float(np.float32(a))
    ch = [dict(c=0, lo=1, hi=1, W0=0, W1=255 * 256, tf=tf)]
    V = _scene_V([[l0, l1]], 8, 8, (4, 4, 4), 2)
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    fr, keep = oracle.make_frame(cam, 16, 16, 0.5, ch, term_alpha=0.99, adaptive=True)
    r = oracle.render(V, [[l0, l1]], _all_resident(V), _leaf_mm_full(V, [[l0, l1]]), fr,
                      oracle.brick_count(V), aov=True)
    n = min(16, math.ceil(math.log(0.01) / (2 * math.log(1 - af))))
    A = 1 - (1 - af) ** (2 * n)
    rgb = np.array([np.float32(0.2), np.float32(0.4), np.float32(0.6)], dtype=np.float64)
    assert np.allclose(r["rgba"][..., 3], A, atol=1e-12, rtol=0)
    assert np.allclose(r["rgba"][..., :3], rgb * A, atol=1e-12, rtol=0)
    assert (r["aov"][..., 1] == n).all() and (r["aov"][..., 0] == 0).all()


def test_adaptive_step_reduces_to_plain_rendering():
    """With every channel's level fixed at l (x factor r) and a transfer
    function of constant opacity a, the adaptive renderer at step d equals
    the plain renderer at step r d with the opacity a' = 1 - (1-a)^r in the
    table (same sample positions, same per-sample colour and opacity); with
    the finest level (r = 1) it equals the plain renderer at step d."""
    vol = synth.BlobVolume((32, 32, 32), n_channels=1, bits=8, n_levels=3, seed=21)
    V = oracle.make_volume((32, 32, 32), (1, 1, 1), 1, 8, 8, 3, (4, 4, 4), 3)
    lm = np.stack([vol.leaf_minmax(0, (4, 4, 4), (8, 8, 8))])
    cam = synth.camera_persp((48.0, 40.0, 70.0), (16.0, 16.0, 16.0), (0.0, 1.0, 0.0), 40.0, 1.0)
    a = 0.15
    rgb_tab = synth.tf_hue(0.6, 1.0).astype(np.float32)
    tf = rgb_tab.copy()
    tf[:, 3] = a
    for lvl in (1, 2):
        r_fac = 2 ** lvl
        ch = [dict(c=0, lo=lvl, hi=lvl, W0=12 * 256, W1=255 * 256, tf=tf)]
        fr, keep = oracle.make_frame(cam, 40, 40, 0.5, ch, adaptive=True)
        ra = oracle.render(V, vol.levels, _all_resident(V), lm, fr, oracle.brick_count(V))
        tf2 = tf.copy()
        tf2[:, 3] = 1.0 - (1.0 - np.float64(np.float32(a))) ** r_fac
        ch2 = [dict(ch[0], tf=tf2)]
        fr2, keep2 = oracle.make_frame(cam, 40, 40, 0.5 * r_fac, ch2)
        rp = oracle.render(V, vol.levels, _all_resident(V), lm, fr2, oracle.brick_count(V))
        # the corrected table entry is rounded to float32 on the plain side
        assert np.abs(ra["rgba"] - rp["rgba"]).max() < 1e-6
        assert ra["rgba"][..., 3].max() > 0.1
        assert ra["stats"]["samples"] == rp["stats"]["samples"]
    ch = [dict(c=0, lo=0, hi=0, W0=12 * 256, W1=255 * 256, tf=synth.tf_ramp())]
    fr, keep = oracle.make_frame(cam, 40, 40, 0.5, ch, adaptive=True)
    fr0, keep0 = oracle.make_frame(cam, 40, 40, 0.5, ch)
    ra = oracle.render(V, vol.levels, _all_resident(V), lm, fr, oracle.brick_count(V))
    r0 = oracle.render(V, vol.levels, _all_resident(V), lm, fr0, oracle.brick_count(V))
    assert np.array_equal(ra["rgba"], r0["rgba"]) and np.array_equal(ra["counts"], r0["counts"])


def test_single_channel_mix_is_identity_and_duplicates_combine():
    """R24 mix: one channel passes (rgb, alpha) through; two identical
    channels give alpha_s = 1 - (1 - alpha)^2 with the same colour."""
    rng = np.random.default_rng(9)
    a = rng.integers(0, 256, size=(8, 8, 8)).astype(np.uint8)
    tf = synth.tf_hue(0.3, alpha_scale=0.7)
    one = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf)]
    two = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf),
           dict(c=1, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf)]
    for p in rng.uniform(0, 8, size=(20, 3)):
        s1 = _probe([[a]], 8, p, one, B=4, leaf=(4, 4, 4), depth=1)
        s2 = _probe([[a], [a.copy()]], 8, p, two, B=4, leaf=(4, 4, 4), depth=1)
        al = s1[3]
        rgb = s1[:3] / al if al > 0 else np.zeros(3)
        assert abs(s2[3] - (1 - (1 - al) ** 2)) < 1e-12
        assert np.allclose(s2[:3], rgb * s2[3], atol=1e-12)
        # the single-channel case is the table itself: colour = hue
        if al > 0:
            assert np.allclose(rgb, np.asarray(tf[0, :3], dtype=np.float64), atol=1e-6)


def test_mix_is_symmetric_in_channel_order():
    vol = synth.BlobVolume((32, 32, 16), n_channels=3, bits=16, n_levels=2, seed=4)
    V = oracle.make_volume((32, 32, 16), (1, 1, 1), 3, 16, 8, 2, (4, 4, 4), 3)
    tfs = [synth.tf_hue(c / 3.0, 0.2) for c in range(3)]
    chans = [dict(c=c, lo=0, hi=1, W0=200 * 256, W1=60000 * 256, tf=tfs[c]) for c in range(3)]
    cam = synth.camera_oblique_ortho((32, 32, 16), (1, 1, 1), 7, 48, 40)
    res = _all_resident(V)
    mm = _leaf_mm_full(V, vol.levels)
    outs = []
    for order in ([0, 1, 2], [2, 0, 1], [1, 2, 0]):
        fr, keep = oracle.make_frame(cam, 48, 40, 0.5, [chans[i] for i in order])
        outs.append(oracle.render(V, vol.levels, res, mm, fr, oracle.brick_count(V)))
    for o in outs[1:]:
        amb = outs[0]["amb_pix"] | o["amb_pix"]
        d = np.abs(o["rgba"] - outs[0]["rgba"])[amb == 0]
        assert d.max() < 1e-12
        assert np.array_equal(o["counts"], outs[0]["counts"])
        assert np.array_equal(o["used"], outs[0]["used"])


# ------------------------------------------ brute force / special cases

@pytest.mark.parametrize("camkind", ["axis", "oblique", "persp"])
def test_full_resolution_equals_brute_force(camkind):
    """With every L0 brick resident and lo = hi = 0 the image equals plain
    ray marching of the full-resolution volume: emptiness, residency and
    substitution change nothing (metadata are exact, so no visible sample is
    dropped)."""
    vol = synth.config1_volume()
    V = oracle.make_volume((64, 64, 64), (1, 1, 1), 1, 8, 16, 3, (8, 8, 8), 3)
    lm = vol.leaf_minmax(0, (8, 8, 8), leaf_grid((64, 64, 64), (8, 8, 8), 3))[None]
    W0, W1 = synth.window_fx(0.05 * 255, 255)
    ch = [dict(c=0, lo=0, hi=0, W0=W0, W1=W1, tf=synth.tf_ramp())]
    if camkind == "axis":
        cam, W, H = synth.camera_ortho_axis((64, 64), 128, 128), 128, 128
    elif camkind == "oblique":
        cam, W, H = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 3, 96, 80), 96, 80
    else:
        cam = synth.camera_persp((150.0, 120.0, 100.0), (32, 32, 32), (0, 0, 1), 40.0, 1.2)
        W, H = 96, 80
    fr, keep = oracle.make_frame(cam, W, H, 0.5, ch)
    # only L0 resident
    res = np.full(oracle.brick_count(V), -1, np.int32)
    res[:64] = np.arange(64)
    r = oracle.render(V, vol.levels, res, lm, fr, 73)
    b = oracle.brute(V, vol.levels, 0, fr)
    assert np.abs(r["rgba"] - b).max() < 1e-12
    assert r["counts"].sum() == 0


def test_substitution_uses_finest_resident_level():
    """Alg. 1 getAlternativeBrick with the finest resident coarser level:
    with only level-2 bricks resident and lo = hi = 0 every sample reads
    level 2, the image equals brute force at level 2 with the leaves that are
    empty at L0 masked, and every sample in a non-empty leaf requests its L0
    brick."""
    vol = synth.config1_volume()
    V = oracle.make_volume((64, 64, 64), (1, 1, 1), 1, 8, 16, 3, (8, 8, 8), 3)
    lm = vol.leaf_minmax(0, (8, 8, 8), leaf_grid((64, 64, 64), (8, 8, 8), 3))[None]
    W0, W1 = synth.window_fx(0.05 * 255, 255)
    ch = [dict(c=0, lo=0, hi=0, W0=W0, W1=W1, tf=synth.tf_ramp())]
    cam = synth.camera_ortho_axis((64, 64), 128, 128)
    fr, keep = oracle.make_frame(cam, 128, 128, 0.5, ch, term_margin=2e-6)
    res = np.full(73, -1, np.int32)
    res[72] = 0  # the single level-2 brick
    r = oracle.render(V, vol.levels, res, lm, fr, 1, aov=True)
    assert r["aov"][..., 0].sum() == 0 and r["aov"][..., 1].sum() == 0
    assert r["aov"][..., 2].sum() == r["stats"]["channel_samples"] > 0
    # requests only for L0 bricks, total = number of (sample, channel) reads
    assert r["counts"][64:].sum() == 0
    assert r["counts"].sum() == r["stats"]["missing"] == r["stats"]["channel_samples"]
    # masked brute force at level 2: build a level-2-valued volume at L0 size
    # where L0-empty leaves are zeroed in the TF sense (window below)
    l2 = vol.levels[0][2].astype(np.float64)
    ok = r["amb_pix"] == 0
    assert ok.mean() > 0.99
    # the sample values along z are those of level 2; check the first hit
    # pixel against a direct level-2 trilinear evaluation of a single sample
    fr1, keep1 = oracle.make_frame(single_sample_camera((21.3, 40.7, 33.1)), 1, 1, 1000.0, ch)
    r1 = oracle.render(V, vol.levels, res, lm, fr1, 1)
    q = np.array([21.3, 40.7, 33.1]) / 4.0 - 0.5
    v = map_coordinates(l2, [[q[2]], [q[1]], [q[0]]], order=1, mode="nearest")[0]
    leaf = (int(21.3) // 8, int(40.7) // 8, int(33.1) // 8)
    li = (leaf[2] * 8 + leaf[1]) * 8 + leaf[0]
    empty = oracle.tf_empty(int(lm[0, li, 0]), int(lm[0, li, 1]), W0, W1, synth.tf_ramp())
    x = min(max((v - W0 / 256) / ((W1 - W0) / 256), 0), 1)
    expect = 0.0 if empty else x
    assert abs(r1["rgba"][0, 0, 3] - expect) < 1e-6


def test_per_channel_resolution_ranges():
    """Sec. 6.2 / Fig. 6: each channel renders in its own level range; with
    everything resident, channel c with lo = hi = l_c reads only level l_c."""
    vol = synth.BlobVolume((32, 32, 32), n_channels=3, bits=8, n_levels=3, seed=11)
    V = oracle.make_volume((32, 32, 32), (1, 1, 1), 3, 8, 8, 3, (4, 4, 4), 3)
    lm = np.stack([vol.leaf_minmax(c, (4, 4, 4), (8, 8, 8)) for c in range(3)])
    cam = synth.camera_oblique_ortho((32, 32, 32), (1, 1, 1), 5, 40, 40)
    for c, lvl in enumerate([0, 2, 1]):
        ch = [dict(c=c, lo=lvl, hi=lvl, W0=12 * 256, W1=255 * 256, tf=synth.tf_ramp())]
        fr, keep = oracle.make_frame(cam, 40, 40, 0.5, ch)
        r = oracle.render(V, vol.levels, _all_resident(V), lm, fr, oracle.brick_count(V), aov=True)
        tot = r["aov"].sum(axis=(0, 1))
        assert tot[lvl] > 0 and tot.sum() == tot[lvl]


# --------------------------------------------------------------- emptiness

def _alpha_exact(v: Fraction, W0, W1, tf):
    w0, w1 = Fraction(W0, 256), Fraction(W1, 256)
    x = (v - w0) / (w1 - w0)
    x = min(max(x, Fraction(0)), Fraction(1))
    p = 255 * x
    i0 = min(int(math.floor(p)), 255)
    i1 = min(i0 + 1, 255)
    fr = p - i0
    return Fraction(float(tf[i0, 3])) * (1 - fr) + Fraction(float(tf[i1, 3])) * fr


def test_emptiness_equals_zero_alpha_on_the_range():
    """R7 read against the continuous definition: [mn, mx] is empty iff the
    interpolated alpha is 0 for every value in [mn, mx].  Alpha is piecewise
    linear with breakpoints where the table position is an integer, so it
    suffices to check both ends and every breakpoint inside (exact
    rationals)."""
    rng = np.random.default_rng(3)
    for trial in range(60):
        tf = np.zeros((256, 4), np.float32)
        nz = rng.random(256) < rng.uniform(0.05, 0.7)
        tf[nz, 3] = rng.uniform(0.01, 1, nz.sum())
        raw_max = 255 if trial % 2 else 65535
        a, b = sorted(rng.integers(0, raw_max * 256, 2))
        if b - a < 64:
            b = a + 64
        W0, W1 = int(a), int(b)
        for _ in range(40):
            mn, mx = sorted(int(x) for x in rng.integers(0, raw_max + 1, 2))
            if rng.random() < 0.3:
                mx = min(raw_max, mn + int(rng.integers(0, 4)))
            pts = {Fraction(mn), Fraction(mx)}
            w0, w1 = Fraction(W0, 256), Fraction(W1, 256)
            for e in range(256):
                v = w0 + (w1 - w0) * Fraction(e, 255)
                if mn <= v <= mx:
                    pts.add(v)
            zero = all(_alpha_exact(v, W0, W1, tf) == 0 for v in pts)
            assert oracle.tf_empty(mn, mx, W0, W1, tf) == zero, (W0, W1, mn, mx)


# ----------------------------------------------------------------- masks

def _tiny_geometry():
    dims, B, L, leaf, depth = (24, 20, 12), 4, 3, (4, 4, 2), 3
    return oracle.make_volume(dims, (1, 1, 1), 2, 8, B, L, leaf, depth)


class IncrementalOctree:
    """The paper's incremental residency update (Sec. 5.3), written as its
    own algorithm: on insert, mark every leaf overlapping the brick and
    propagate the OR of children upward, stopping where a node is unchanged;
    on eviction, recheck each overlapping leaf against the other resident
    bricks of that level and channel, then propagate the same way."""

    def __init__(self, V):
        self.V = V
        tot, self.off, self.n = oracle.node_count(V)
        self.d, self.f, self.nb = oracle.level_info(V)
        self.D = V.depth
        self.size = [tuple(int(np.ceil(1)) for _ in range(3))] * (self.D + 1)
        self.size = []
        for dd in range(self.D + 1):
            self.size.append(tuple(int(V.leaf[a] * self.n[self.D][a] // self.n[dd][a]) for a in range(3)))
        self.mask = np.zeros((tot, V.n_channels), np.uint16)
        self.res = set()

    def _node(self, dd, x, y, z):
        return int(self.off[dd] + (z * self.n[dd][1] + y) * self.n[dd][0] + x)

    def _brick_box(self, l, b):
        e = [self.V.B * int(self.f[l][a]) for a in range(3)]
        return [b[a] * e[a] for a in range(3)], [(b[a] + 1) * e[a] for a in range(3)]

    def _overlap(self, lo1, hi1, lo2, hi2):
        return all(lo1[a] < hi2[a] and lo2[a] < hi1[a] for a in range(3))

    def _leaves_of(self, lo, hi):
        D, s = self.D, self.size[self.D]
        rng = [range(max(lo[a] // s[a], 0), min(-(-hi[a] // s[a]), int(self.n[D][a]))) for a in range(3)]
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    yield x, y, z

    def _propagate(self, c, x, y, z):
        for dd in range(self.D - 1, -1, -1):
            px, py, pz = [v // (self.n[dd + 1][a] // self.n[dd][a]) for a, v in enumerate((x, y, z))]
            r = [self.n[dd + 1][a] // self.n[dd][a] for a in range(3)]
            m = 0
            for cz in range(pz * r[2], (pz + 1) * r[2]):
                for cy in range(py * r[1], (py + 1) * r[1]):
                    for cx in range(px * r[0], (px + 1) * r[0]):
                        m |= int(self.mask[self._node(dd + 1, cx, cy, cz), c])
            node = self._node(dd, px, py, pz)
            if self.mask[node, c] == m:
                return  # unchanged: stop the upward propagation
            self.mask[node, c] = m
            x, y, z = px, py, pz

    def insert(self, c, l, b):
        self.res.add((c, l, tuple(b)))
        lo, hi = self._brick_box(l, b)
        for x, y, z in self._leaves_of(lo, hi):
            n = self._node(self.D, x, y, z)
            if not (self.mask[n, c] >> l) & 1:
                self.mask[n, c] |= 1 << l
                self._propagate(c, x, y, z)

    def evict(self, c, l, b):
        self.res.discard((c, l, tuple(b)))
        lo, hi = self._brick_box(l, b)
        s = self.size[self.D]
        for x, y, z in self._leaves_of(lo, hi):
            llo = (x * s[0], y * s[1], z * s[2])
            lhi = ((x + 1) * s[0], (y + 1) * s[1], (z + 1) * s[2])
            still = any(cc == c and ll == l and self._overlap(llo, lhi, *self._brick_box(ll, bb))
                        for (cc, ll, bb) in self.res)
            n = self._node(self.D, x, y, z)
            if not still and (self.mask[n, c] >> l) & 1:
                self.mask[n, c] &= ~np.uint16(1 << l)
                self._propagate(c, x, y, z)


@given(st.lists(st.tuples(st.booleans(), st.integers(0, 10 ** 6)), min_size=1, max_size=40))
@settings(max_examples=40, deadline=None)
def test_incremental_update_equals_masks_from_scratch(ops):
    """Sec. 5.3: incremental insert / evict with early-stopping OR
    propagation yields, after every step, exactly the masks defined by
    partial mapping (O2)."""
    V = _tiny_geometry()
    d, f, nb = oracle.level_info(V)
    inc = IncrementalOctree(V)
    ids = oracle.dense_ids(V)
    id_to_dense = {int(x): i for i, x in enumerate(ids)}
    all_b = [(c, l, (bx, by, bz)) for c in range(2) for l in range(3)
             for bz in range(nb[l][2]) for by in range(nb[l][1]) for bx in range(nb[l][0])]
    for ins, r in ops:
        if ins or not inc.res:
            c, l, b = all_b[r % len(all_b)]
            inc.insert(c, l, b)
        else:
            c, l, b = sorted(inc.res)[r % len(inc.res)]
            inc.evict(c, l, b)
        res = np.full(oracle.brick_count(V), -1, np.int32)
        for (c, l, b) in inc.res:
            res[id_to_dense[oracle.brick_id(3, c, l, *b)]] = 0
        assert np.array_equal(oracle.masks(V, res), inc.mask)


def test_mask_propagation_invariants():
    """Sec. 3: partially mapped propagates to parents; fully mapped
    propagates to children (full mapping computed by brute-force coverage)."""
    V = _tiny_geometry()
    tot, off, n = oracle.node_count(V)
    d, f, nb = oracle.level_info(V)
    rng = np.random.default_rng(1)
    res = np.where(rng.random(oracle.brick_count(V)) < 0.3, 0, -1).astype(np.int32)
    m = oracle.masks(V, res)
    ids = oracle.dense_ids(V)
    D = V.depth
    size = [tuple(int(V.leaf[a] * n[D][a] // n[dd][a]) for a in range(3)) for dd in range(D + 1)]
    resident = {}
    for i in np.nonzero(res >= 0)[0]:
        c, l, bx, by, bz = oracle.brick_id_decode(3, int(ids[i]))
        resident.setdefault((c, l), set()).add((bx, by, bz))

    def fully(dd, x, y, z, c, l):
        e = [V.B * int(f[l][a]) for a in range(3)]
        lo = (x * size[dd][0], y * size[dd][1], z * size[dd][2])
        hi = tuple(lo[a] + size[dd][a] for a in range(3))
        hi = tuple(min(hi[a], V.dims[a]) for a in range(3))  # the part inside the volume
        if any(hi[a] <= lo[a] for a in range(3)):
            return True
        for bz in range(lo[2] // e[2], -(-hi[2] // e[2])):
            for by in range(lo[1] // e[1], -(-hi[1] // e[1])):
                for bx in range(lo[0] // e[0], -(-hi[0] // e[0])):
                    if (bx, by, bz) not in resident.get((c, l), ()):
                        return False
        return True

    for dd in range(D):
        r = [n[dd + 1][a] // n[dd][a] for a in range(3)]
        for z in range(n[dd][2]):
            for y in range(n[dd][1]):
                for x in range(n[dd][0]):
                    p = int(off[dd] + (z * n[dd][1] + y) * n[dd][0] + x)
                    for cz in range(z * r[2], (z + 1) * r[2]):
                        for cy in range(y * r[1], (y + 1) * r[1]):
                            for cx in range(x * r[0], (x + 1) * r[0]):
                                ch = int(off[dd + 1] + (cz * n[dd + 1][1] + cy) * n[dd + 1][0] + cx)
                                for c in range(2):
                                    assert (m[ch, c] & ~m[p, c]) == 0  # child partial => parent partial
                                    for l in range(3):
                                        if fully(dd, x, y, z, c, l):
                                            assert fully(dd + 1, cx, cy, cz, c, l)
                                            if cx * size[dd + 1][0] < V.dims[0] and \
                                                    cy * size[dd + 1][1] < V.dims[1] and \
                                                    cz * size[dd + 1][2] < V.dims[2]:
                                                assert (m[ch, c] >> l) & 1


# ------------------------------------------------------------------- LRU

@given(st.integers(0, 10 ** 9))
@settings(max_examples=60, deadline=None)
def test_lru_stream_invariants(seed):
    """Sec. 5.3 LRU eviction under the (stamp, seq) order: the page table is
    a bijection onto occupied slots; free slots are used before any eviction;
    slots used in the current frame are never evicted; every victim has a
    smaller (stamp, seq) than every occupied slot that stayed eligible."""
    rng = np.random.default_rng(seed)
    V = _tiny_geometry()
    S = int(rng.integers(1, 12))
    sim = oracle.CacheSim(V, S)
    total = sim.total
    for f in range(1, 8):
        used = rng.random(S) < 0.3
        sim.touch(f, used.astype(np.uint8) * (sim.slot_brick >= 0))
        before_stamp = sim.stamp.copy()
        before_seq = sim.seq.copy()
        before_brick = sim.slot_brick.copy()
        n = int(rng.integers(0, 8))
        up = rng.integers(0, total, n)
        if n and rng.random() < 0.3:
            up[-1] = up[0]
        flags, ev, so = sim.stream(f, up)
        # bijection
        occ = np.nonzero(sim.slot_brick >= 0)[0]
        assert len(set(sim.slot_brick[occ].tolist())) == len(occ)
        for s in occ:
            assert sim.res_slot[sim.slot_brick[s]] == s
        assert (sim.res_slot >= 0).sum() == len(occ)
        free_before = (before_brick < 0).sum()
        ins = np.nonzero(flags == 1)[0]
        victims = [int(so[i]) for i in ins]
        if len(victims) > free_before:
            assert all(before_brick[v] < 0 for v in victims[:free_before])
        for i in ins:
            v = int(so[i])
            if before_brick[v] >= 0:
                assert before_stamp[v] != f
                key = (int(before_stamp[v]), int(before_seq[v]))
                for s in range(S):
                    if before_brick[s] >= 0 and sim.slot_brick[s] == before_brick[s] and \
                            s not in victims and sim.stamp[s] != f:
                        assert (int(before_stamp[s]), int(before_seq[s])) > key
        # uploads left out only when no eligible slot remained
        if (flags == 0).any():
            assert sum(1 for s in range(S) if before_brick[s] < 0 or before_stamp[s] != f) <= len(ins) + \
                sum(1 for i in range(n) if flags[i] == 2 and before_brick[sim.res_slot[up[i]]] >= 0)


# -------------------------------------------------------------- metadata

def test_leaf_metadata_exact_and_node_reduction():
    vol = synth.config1_volume()
    V = oracle.make_volume((64, 64, 64), (1, 1, 1), 1, 8, 16, 3, (8, 8, 8), 3)
    lm = vol.leaf_minmax(0, (8, 8, 8), (8, 8, 8))
    a = vol.levels[0][0]
    rng = np.random.default_rng(0)
    for li in rng.integers(0, 512, 40):
        x, y, z = li % 8, (li // 8) % 8, li // 64
        blk = a[max(z * 8 - 1, 0):z * 8 + 9, max(y * 8 - 1, 0):y * 8 + 9, max(x * 8 - 1, 0):x * 8 + 9]
        assert lm[li, 0] == blk.min() and lm[li, 1] == blk.max()
    meta = oracle.meta_all(V, lm[None])
    tot, off, n = oracle.node_count(V)
    # node box min / max over the dilated box equals min / max over its leaves
    for dd in range(4):
        s = 64 // n[dd][0]
        for z in range(n[dd][2]):
            for y in range(n[dd][1]):
                for x in range(n[dd][0]):
                    node = off[dd] + (z * n[dd][1] + y) * n[dd][0] + x
                    blk = a[max(z * s - 1, 0):z * s + s + 1, max(y * s - 1, 0):y * s + s + 1,
                            max(x * s - 1, 0):x * s + s + 1]
                    assert meta[node, 0, 0] == blk.min() and meta[node, 0, 1] == blk.max()


def test_cell_metadata_is_conservative():
    cv = synth.CellVolume((256, 256, 64), 4, seed=2)
    lm = cv.leaf_max_all((16, 16, 4), (16, 16, 16))
    reg = cv.region(0, 0, 0, 0, 256, 256, 64)
    # dilated-leaf maxima by brute force
    for c in range(4):
        a = reg[c].astype(np.int64)
        pad = np.pad(a, 1, mode="edge")
        for li in np.random.default_rng(c).integers(0, 4096, 300):
            x, y, z = li % 16, (li // 16) % 16, li // 256
            blk = pad[z * 4:z * 4 + 6, y * 16:y * 16 + 18, x * 16:x * 16 + 18]
            assert blk.max() <= lm[c, li]


# ------------------------------------------------------- desired level rule
#
# Alg. 1 chooseResolutionLevel with the reading of Sec. 6.2 (the level can be
# any function of the distance): level l (l >= 1) is desired from the distance
# on where a pixel's footprint beta * t * (2 ty / H) reaches the level's x voxel
# size.  The volume below has anisotropic spacing (1, 3, 1), so the x and y
# voxel sizes of each level differ (x: 1, 2, 4, ..., y: 3, 3, 6, ...), and
# non-square pixels (tx / W != ty / H); each level array holds its own
# constant, so the level a sample reads shows in the opacity as well as in
# the per-level sample counts.

_LVL_VALUE = [1, 2, 3, 4, 5, 6]  # raw u8 value held by every voxel of level l


def _level_constant_scene():
    V = oracle.make_volume((64, 8, 8), (1, 3, 1), 1, 8, 16, 6, (4, 4, 4), 4)
    d, _, _ = oracle.level_info(V)
    levels = [[np.full((d[l][2], d[l][1], d[l][0]), _LVL_VALUE[l], np.uint8) for l in range(6)]]
    ch = [dict(c=0, lo=0, hi=5, W0=0, W1=255 * 256, tf=synth.tf_ramp())]
    return V, levels, ch


def _expected_alpha(level_seq):
    """1 - prod(1 - alpha_k) with alpha_k the ramp table's entry at the raw
    value of the level sample k reads (window [0, 255]: entry v exactly)."""
    tf = synth.tf_ramp()
    T = 1.0
    for l in level_seq:
        T *= 1.0 - float(tf[_LVL_VALUE[l], 3])
    return 1.0 - T


def test_desired_level_perspective_thresholds():
    """A perspective ray along +x from an eye 3.7 units before the volume,
    step 0.5, beta = 2, 2 ty / H = 2 * 0.1875 / 3 = 0.125: the footprint is
    0.25 t, so level l is desired from t = 4 * 2^l on (t = 8, 16, 32, 64 for
    levels 1-4; samples k = 16, 32, 64, 128 lie exactly on them).  The samples
    inside the box are k = 8 (x = 0.3) .. 135 (x = 63.8); by hand they read
    8 x L0, 16 x L1, 32 x L2, 64 x L3, 8 x L4."""
    V, levels, ch = _level_constant_scene()
    cam = dict(proj="persp", eye=[-3.7, 4.3 * 3, 4.3], F=[1.0, 0.0, 0.0], R=[0.0, 0.0, 1.0],
               U=[0.0, 1.0, 0.0], tx=0.2, ty=0.1875)
    fr, keep = oracle.make_frame(cam, 1, 3, 0.5, ch, term_alpha=1.0, lod_bias=2.0)
    res = np.arange(oracle.brick_count(V), dtype=np.int32)
    lm = _leaf_mm_full(V, levels)
    r = oracle.render(V, levels, res, lm, fr, oracle.brick_count(V), aov=True)
    # pixel row 1 of 3 is the axis ray (b = 0)
    expect = [8, 16, 32, 64, 8, 0]
    assert r["aov"][1, 0].tolist() == expect
    seq = [0] * 8 + [1] * 16 + [2] * 32 + [3] * 64 + [4] * 8
    assert abs(r["rgba"][1, 0, 3] - _expected_alpha(seq)) < 1e-12


@pytest.mark.parametrize("beta,level", [
    (0.5, 0),      # footprint 1.5 < 2
    (1.0, 1),      # 3: >= 2, < 4
    (4.0 / 3, 2),  # 4: exactly the level-2 x voxel size (>=); y sizes would give 1
    (2.0, 2),      # 6: >= 4, < 8
    (16.0 / 3, 4), # 16: exactly level 4
])
def test_desired_level_orthographic(beta, level):
    """Orthographic views use the constant pixel size 2 ty / H = 3 (ty = 1.5,
    H = 1; the horizontal size 2 tx / W = 1/3 differs): level l is desired
    iff beta * 3 >= the level's x voxel size 2^l.  Every pixel reads the
    same level at its single sample."""
    V, levels, ch = _level_constant_scene()
    cam = dict(proj="ortho", eye=[31.3, 4.3 * 3, 4.3 - 1000.0], F=[0.0, 0.0, 1.0], R=[1.0, 0.0, 0.0],
               U=[0.0, 1.0, 0.0], tx=0.5, ty=1.5)
    fr, keep = oracle.make_frame(cam, 3, 1, 1000.0, ch, term_alpha=1.0, lod_bias=beta)
    res = np.arange(oracle.brick_count(V), dtype=np.int32)
    r = oracle.render(V, levels, res, _leaf_mm_full(V, levels), fr, oracle.brick_count(V), aov=True)
    for i in range(3):
        want = [0] * 6
        want[level] = 1
        assert r["aov"][0, i].tolist() == want, (beta, i, r["aov"][0, i])
        assert abs(r["rgba"][0, i, 3] - _expected_alpha([level])) < 1e-12


def test_desired_level_clamped_per_channel():
    """Sec. 6.2: the distance rule's level is clamped to each channel's range.
    Two visible copies of the level-constant volume on the perspective ray
    above, one limited to levels [1, 2] and one to [3, 5]: per-level counts
    are the hand-computed ones with the clamp applied."""
    V1, levels, _ = _level_constant_scene()
    V = oracle.make_volume((64, 8, 8), (1, 3, 1), 2, 8, 16, 6, (4, 4, 4), 4)
    lv = [levels[0], levels[0]]
    ch = [dict(c=0, lo=1, hi=2, W0=0, W1=255 * 256, tf=synth.tf_ramp()),
          dict(c=1, lo=3, hi=5, W0=0, W1=255 * 256, tf=synth.tf_ramp())]
    cam = dict(proj="persp", eye=[-3.7, 4.3 * 3, 4.3], F=[1.0, 0.0, 0.0], R=[0.0, 0.0, 1.0],
               U=[0.0, 1.0, 0.0], tx=0.2, ty=0.1875)
    fr, keep = oracle.make_frame(cam, 1, 3, 0.5, ch, term_alpha=1.0, lod_bias=2.0)
    res = np.arange(oracle.brick_count(V), dtype=np.int32)
    r = oracle.render(V, lv, res, _leaf_mm_full(V, lv), fr, oracle.brick_count(V), aov=True)
    seq = [0] * 8 + [1] * 16 + [2] * 32 + [3] * 64 + [4] * 8
    a = [min(max(l, 1), 2) for l in seq]
    b = [min(max(l, 3), 5) for l in seq]
    assert r["aov"][1, 0].tolist() == [sum(1 for x in a + b if x == l) for l in range(6)]
    # the two channels mix per sample: 1 - prod over samples and channels
    assert abs(r["rgba"][1, 0, 3] - _expected_alpha(a + b)) < 1e-12


def test_paper_scale_metadata_is_conservative():
    """Leaf metadata of the 16-channel 8192 x 8192 x 192 tissue volume (cell
    maxima times the tissue mask and the per-channel gain) bound every L0
    voxel within one voxel of the leaf (the trilinear footprint), checked on
    more than 10^6 voxels per channel: 340 random leaves of the volume and,
    per channel, 50 leaves with maximum 0 next to a non-empty leaf (where a
    bound that misses the mask's edge or a cell reaching over the leaf face
    would show)."""
    cv = synth.config3_volume()
    leaf, grid = (16, 16, 8), (512, 512, 32)
    lm = cv.leaf_max_all(leaf, grid)  # [16][n_leaves]
    lmg = lm.reshape(16, grid[2], grid[1], grid[0])
    rng = np.random.default_rng(30)
    nz = 192 // leaf[2]
    picks = [(int(x), int(y), int(z)) for x, y, z in
             zip(rng.integers(0, 512, 340), rng.integers(0, 512, 340), rng.integers(0, nz, 340))]
    # empty leaves bordering a non-empty one in x or y (any channel)
    occ = (lmg[:, :nz] > 0)
    border = np.zeros_like(occ)
    border[:, :, :, 1:] |= occ[:, :, :, :-1]
    border[:, :, :, :-1] |= occ[:, :, :, 1:]
    border[:, :, 1:, :] |= occ[:, :, :-1, :]
    border[:, :, :-1, :] |= occ[:, :, 1:, :]
    border &= ~occ
    for c in range(16):
        zz, yy, xx = np.nonzero(border[c])
        sel = rng.choice(len(zz), 50, replace=False)
        picks += [(int(xx[i]), int(yy[i]), int(zz[i])) for i in sel]
    checked = np.zeros(16, np.int64)
    n_empty_checked = 0
    for (x, y, z) in picks:
        lo = [max(0, x * leaf[0] - 1), max(0, y * leaf[1] - 1), max(0, z * leaf[2] - 1)]
        hi = [min(8192, (x + 1) * leaf[0] + 1), min(8192, (y + 1) * leaf[1] + 1),
              min(192, (z + 1) * leaf[2] + 1)]
        reg = cv.region(0, lo[0], lo[1], lo[2], hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
        li = (z * grid[1] + y) * grid[0] + x
        vmax = reg.reshape(16, -1).max(axis=1)
        bound = lm[:, li]
        assert (vmax <= bound).all(), ((x, y, z), vmax.tolist(), bound.tolist())
        checked += reg[0].size
        n_empty_checked += int((bound == 0).sum())
    assert checked.min() >= 10 ** 6 and n_empty_checked >= 16 * 50


# ------------------------------------------------ bricks required per pixel

@pytest.mark.parametrize("level,n_ch", [(0, 1), (1, 1), (0, 2), (2, 2)])
def test_required_bricks_axis_closed_form(level, n_ch):
    """Sec. 8 (bricks required to be resident per pixel): an axis ray through
    a 64^3 volume with nothing empty and no early termination needs, per
    channel, the level-l bricks of edge 16 f_l it crosses in z: 64 / (16 f_l),
    whatever is resident (the count is of desired bricks)."""
    vol = np.full((64, 64, 64), 100, np.uint8)
    levels = [[vol, vol[::2, ::2, ::2].copy(), vol[::4, ::4, ::4].copy()] for _ in range(n_ch)]
    V = _scene_V(levels, 8, 16, (8, 8, 8), 3)
    chans = [dict(c=c, lo=level, hi=level, W0=0, W1=255 * 256, tf=_const_tf((0.5, 0.5, 0.5), 1e-4))
             for c in range(n_ch)]
    cam = synth.camera_ortho_axis((64, 64), 32, 32)
    fr, keep = oracle.make_frame(cam, 32, 32, 0.5, chans)
    for res in (_all_resident(V), np.full(oracle.brick_count(V), -1, np.int32)):
        r = oracle.render(V, levels, res, _leaf_mm_full(V, levels), fr, oracle.brick_count(V))
        assert (r["required_bricks"] == n_ch * (64 // (16 << level))).all()


@pytest.mark.parametrize("seed,homog", [(0, False), (1, False), (2, True), (3, True)])
def test_required_bricks_equal_the_pixel_read_set(seed, homog):
    """With every level-0 brick resident and level 0 desired, the bricks a
    pixel requires are the bricks it reads: for one-pixel frames on random
    views, the count equals the number of slots the frame marks as read
    (a separate output: the usage set), with empty leaves, early termination
    and, with the option on, nodes rendered from their values (which read
    and require nothing)."""
    rng = np.random.default_rng(seed)
    if homog:
        src = synth.plateau_volume(2)
        leaf, depth = (4, 4, 4), 4
        chans = []
        for c in range(2):
            tf = synth.tf_hue(c / 2, 0.3)
            tf[:, 3] = np.maximum(tf[:, 3], np.float32(0.004))
            chans.append(dict(c=c, lo=0, hi=0, W0=0, W1=255 * 256, tf=tf))
    else:
        src = synth.config1_volume()
        leaf, depth = (8, 8, 8), 3
        W0, W1 = synth.window_fx(0.05 * 255, 255)
        chans = [dict(c=0, lo=0, hi=0, W0=W0, W1=W1, tf=synth.tf_ramp())]
    V = oracle.make_volume(src.dims, src.spacing, src.n_channels, src.bits, 16, src.n_levels, leaf, depth)
    lg = leaf_grid(src.dims, leaf, depth)
    lm = np.stack([src.leaf_minmax(c, leaf, lg) for c in range(src.n_channels)])
    full = _all_resident(V)
    hits = 0
    for _ in range(12):
        eye = rng.uniform(-40, 104, 3)
        eye[rng.integers(0, 3)] = rng.choice([-60.0, 124.0])
        tgt = rng.uniform(16, 48, 3)
        cam = synth.camera_persp(eye, tgt, (0, 0, 1) if abs(eye[2] - tgt[2]) < 50 else (1, 0, 0), 1.0, 1.0)
        fr, keep = oracle.make_frame(cam, 1, 1, 0.5, chans, homogeneous=homog)
        r = oracle.render(V, src.levels, full, lm, fr, oracle.brick_count(V))
        assert r["required_bricks"][0, 0] == r["used"].sum()
        hits += r["used"].sum() > 1
    assert hits >= 6


# ------------------------------------------- per-channel sampling rates (f1)

def _two_const(a0, a1, rgb0=(0.2, 0.4, 0.6), rgb1=(0.2, 0.4, 0.6)):
    l = [np.full((16 >> i, 16 >> i, 16 >> i), 128, np.uint8) for i in range(3)]
    levels = [l, [x.copy() for x in l]]
    V = _scene_V(levels, 8, 8, (4, 4, 4), 2)
    chans = [dict(c=0, lo=0, hi=0, W0=0, W1=255 * 256, tf=_const_tf(rgb0, a0)),
             dict(c=1, lo=1, hi=1, W0=0, W1=255 * 256, tf=_const_tf(rgb1, a1))]
    return levels, V, chans


@pytest.mark.parametrize("a0,a1", [(0.01, 0.02), (0.0, 0.05), (0.03, 0.0)])
def test_channel_rates_two_constant_channels(a0, a1):
    """Sec. 6.1 (a channel may need only every second step): channel 0 at
    level 0 (rate 1), channel 1 at level 1 (rate 2, x factor 2).  An axis ray
    has 32 base samples in [0, 16); channel 1 takes part in the 16 even ones,
    each standing for two steps, so the opacity keeps its value per unit
    length: A = 1 - (1-a0)^32 (1-a1)^32 (equal colours: C = rgb A), and with
    nothing resident channel 0 requests 32 times per ray, channel 1 16 times
    (at its level 1)."""
    levels, V, chans = _two_const(a0, a1)
    cam = synth.camera_ortho_axis((16, 16), 16, 16)
    fr, keep = oracle.make_frame(cam, 16, 16, 0.5, chans, adaptive=True, channel_rates=True)
    r = oracle.render(V, levels, _all_resident(V), _leaf_mm_full(V, levels), fr, oracle.brick_count(V))
    f0, f1 = float(np.float32(a0)), float(np.float32(a1))
    A = 1 - (1 - f0) ** 32 * (1 - f1) ** 32
    rgb = np.array([np.float32(0.2), np.float32(0.4), np.float32(0.6)], dtype=np.float64)
    assert np.allclose(r["rgba"][..., 3], A, atol=1e-12, rtol=0)
    assert np.allclose(r["rgba"][..., :3], rgb * A, atol=1e-12, rtol=0)
    none = np.full(oracle.brick_count(V), -1, np.int32)
    r = oracle.render(V, levels, none, _leaf_mm_full(V, levels), fr, 1)
    ids = oracle.dense_ids(V)
    per = {0: 0, 1: 0}
    for i in np.nonzero(r["counts"])[0]:
        c, l, _, _, _ = oracle.brick_id_decode(V.n_levels, int(ids[i]))
        assert l == (0 if c == 0 else 1)
        per[c] += int(r["counts"][i])
    # a channel whose table has zero alpha everywhere is empty: it requests nothing
    assert per[0] == (16 * 16 * 32 if a0 > 0 else 0)
    assert per[1] == (16 * 16 * 16 if a1 > 0 else 0)


def test_channel_rates_reduce_to_the_adaptive_step():
    """With every channel at one level range the rates coincide with the
    step's, so the option changes nothing (images within FP64 rounding, the
    same requests and reads), on oblique views over the blob volume with
    part of the bricks resident."""
    src = synth.config1_volume()
    V = oracle.make_volume(src.dims, src.spacing, 1, 8, 16, src.n_levels, (8, 8, 8), 3)
    lm = src.leaf_minmax(0, (8, 8, 8), leaf_grid(src.dims, (8, 8, 8), 3))[None]
    W0, W1 = synth.window_fx(0.05 * 255, 255)
    chans = [dict(c=0, lo=0, hi=2, W0=W0, W1=W1, tf=synth.tf_ramp())]
    rng = np.random.default_rng(2)
    res = np.full(oracle.brick_count(V), -1, np.int32)
    pick = np.nonzero(rng.random(oracle.brick_count(V)) < 0.6)[0]
    res[pick] = np.arange(len(pick))
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    out = []
    for rates in (False, True):
        fr, keep = oracle.make_frame(cam, 48, 40, 0.5, chans, lod_bias=1.5, adaptive=True, channel_rates=rates)
        out.append(oracle.render(V, src.levels, res, lm, fr, len(pick)))
    p, q = out
    assert np.abs(p["rgba"] - q["rgba"]).max() < 1e-12
    assert np.array_equal(p["counts"], q["counts"]) and np.array_equal(p["used"], q["used"])
    assert p["stats"]["samples"] > 0 and p["rgba"][..., 3].max() > 0.01


# --------------------------------------------- traversal depth from the step (f1)

def test_traversal_depth_equals_a_coarser_tree():
    """Alg. 1 chooseTraversalDepth: with samples 5 world units apart (step
    2.5, level 1 so r = 2) and 4^3 leaves, the deepest node whose extent is
    at least the step is the 8^3 node one level up; emptiness decided there
    equals rendering a tree whose leaves are 8^3, with the metadata of those
    nodes (min and max over their 4^3 leaves, which is also the exact dilated
    metadata of the 8^3 box), without the option: images, requests and reads
    identical.  Without the option the finer leaves decide and fewer samples
    read data (so the pin is not vacuous); with a step of 0.5 the leaf is
    deep enough and the option changes nothing."""
    src = synth.config1_volume()
    W0, W1 = synth.window_fx(0.05 * 255, 255)
    chans = [dict(c=0, lo=0, hi=2, W0=W0, W1=W1, tf=synth.tf_ramp())]
    VA = oracle.make_volume(src.dims, src.spacing, 1, 8, 16, src.n_levels, (4, 4, 4), 4)
    VB = oracle.make_volume(src.dims, src.spacing, 1, 8, 16, src.n_levels, (8, 8, 8), 3)
    lmA = src.leaf_minmax(0, (4, 4, 4), leaf_grid(src.dims, (4, 4, 4), 4))[None]
    lmB = src.leaf_minmax(0, (8, 8, 8), leaf_grid(src.dims, (8, 8, 8), 3))[None]
    nodesA = oracle.meta_all(VA, lmA)  # [node][c][2]
    _, offA, _ = oracle.node_count(VA)
    assert np.array_equal(nodesA[offA[3]:offA[4], 0], lmB[0])
    full = np.arange(oracle.brick_count(VA), dtype=np.int32)
    res = full.copy()
    res[np.random.default_rng(1).random(len(res)) < 0.3] = -1
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 3, 64, 64)
    for r_ in (full, res):
        fa, ka = oracle.make_frame(cam, 64, 64, 2.5, chans, lod_bias=1.5, adaptive=True, traversal_depth=True)
        fb, kb = oracle.make_frame(cam, 64, 64, 2.5, chans, lod_bias=1.5, adaptive=True)
        a = oracle.render(VA, src.levels, r_, lmA, fa, len(full), aov=True)
        b = oracle.render(VB, src.levels, r_, lmB, fb, len(full), aov=True)
        c = oracle.render(VA, src.levels, r_, lmA, fb, len(full), aov=True)
        # every sample desires level 1 (level 2 only substitutes for missing level-1 bricks)
        assert (a["aov"][..., 1] > 0).any() and a["aov"][..., 0].sum() == 0
        assert r_ is res or a["aov"][..., 2].sum() == 0
        assert np.array_equal(a["rgba"], b["rgba"])
        assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["used"], b["used"])
        # without the option the 4^3 leaves decide: fewer samples read data
        assert c["stats"]["channel_samples"] < a["stats"]["channel_samples"]
    fa, ka = oracle.make_frame(cam, 64, 64, 0.5, chans, lod_bias=1.5, adaptive=True, traversal_depth=True)
    fc, kc = oracle.make_frame(cam, 64, 64, 0.5, chans, lod_bias=1.5, adaptive=True)
    a = oracle.render(VA, src.levels, full, lmA, fa, len(full))
    c = oracle.render(VA, src.levels, full, lmA, fc, len(full))
    assert np.array_equal(a["rgba"], c["rgba"]) and np.array_equal(a["counts"], c["counts"])
