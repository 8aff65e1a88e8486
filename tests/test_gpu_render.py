"""GPU parity of the render path against the CPU oracle (through the C ABI).

Images: per RGBA channel <= 1e-3 max abs and <= 1e-5 mean abs over the
pixels that are not ambiguous.  Requests (multiset), usage (slot set), page
tables and masks: bit-exact outside the oracle's tolerated set."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import (aov_mask, compare_images, compare_requests, compare_usage, gpu_rgba, leaf_grid,
                           oracle_alt)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_04393_amd import resoct  # noqa: E402
from paper_2309_04393_amd.pipeline import GpuScene  # noqa: E402


def _report(name, **kw):
    print(f"[{name}] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


class Pair:
    """A GPU scene and the oracle's view of the same inputs."""

    def __init__(self, src, B, leaf, depth, n_slots, max_batch=1024, start_level=0):
        self.src = src
        self.gpu = GpuScene(src, B, leaf, depth, n_slots, max_batch=max_batch, start_level=start_level)
        self.V = oracle.make_volume(src.dims, src.spacing, src.n_channels, src.bits, B, src.n_levels, leaf,
                                    depth)
        self.sim = oracle.CacheSim(self.V, n_slots)
        self.ids = oracle.dense_ids(self.V)
        lg = leaf_grid(src.dims, leaf, depth)
        self.leaf_mm = np.stack([src.leaf_minmax(c, leaf, lg) for c in range(src.n_channels)])
        self.S = n_slots

    def upload(self, frame, ids):
        fg = self.gpu.upload(frame, ids)
        fo, ev, so = self.sim.stream(frame, self.sim.dense_of(ids))
        assert np.array_equal(fg, fo), "upload flags differ"
        pt_gpu = self.gpu.cache.page_table_host()
        dev_pt = self.gpu.cache.t["page_table"][:4 * len(pt_gpu)].view(torch.int32).cpu().numpy().view(np.uint32)
        assert np.array_equal(dev_pt, pt_gpu), "device page table differs from the host mirror"
        return fg

    def check_page_table(self):
        pt = self.gpu.cache.page_table_host()
        all_ids = self.gpu.all_ids()
        gmap = {int(i): int(s) for i, s in zip(all_ids, pt) if s != 0xFFFFFFFF}
        assert gmap == self.sim.page_table(), "page tables differ"

    def check_masks(self):
        self.gpu.tree.update_residency()
        torch.cuda.synchronize()
        m_gpu = self.gpu.tree.masks()
        m_or = oracle.masks(self.V, self.sim.res_slot)
        assert np.array_equal(m_gpu, m_or), f"masks differ at {np.argwhere(m_gpu != m_or)[:5]}"

    def frame(self, f, cam, W, H, step, chans, term_margin=1e-6, aov=False, bricks=False, **kw):
        r = self.gpu.render(f, cam, W, H, step, chans, aov=aov, bricks=bricks, **kw)
        torch.cuda.synchronize()
        ids, cnt, nu, tot = self.gpu.cache.read_requests(1 << 20)
        used, nused = self.gpu.cache.read_usage(f)
        fr, keep = oracle.make_frame(cam, W, H, step, chans, term_margin=term_margin,
                                     lod_bias=kw.get("lod_bias", 1.0),
                                     adaptive=bool(kw.get("flags", 0) & resoct.RENDER_ADAPTIVE_STEP),
                                     homogeneous=bool(kw.get("flags", 0) & resoct.RENDER_HOMOGENEOUS),
                                     channel_rates=bool(kw.get("flags", 0) & resoct.RENDER_CHANNEL_RATES),
                                     traversal_depth=bool(kw.get("flags", 0) & resoct.RENDER_TRAVERSAL_DEPTH))
        o = oracle.render(self.V, self.src.levels, self.sim.res_slot, self.leaf_mm, fr, self.S, aov=aov)
        self.sim.touch(f, o["used"])
        out = dict(gpu=gpu_rgba(r["rgba"], H, W), ref=o["rgba"], o=o, ids=ids, cnt=cnt, nu=nu, tot=tot,
                   used=used, r=r)
        if aov:
            out["aov"] = r["aov"].cpu().numpy().reshape(H, W, self.src.n_levels)
        if bricks:
            out["bricks"] = r["bricks"].cpu().numpy()
        return out

    def check_frame(self, res, name):
        st = compare_images(res["gpu"], res["ref"], res["o"]["amb_pix"], alt=oracle_alt(res["o"]))
        nreq = compare_requests(res["ids"], res["cnt"], res["o"]["counts"], res["o"]["amb_counts"], self.ids)
        compare_usage(res["used"], res["o"]["used"], res["o"]["amb_used"])
        _report(name, requests=nreq, total=res["tot"], used=len(res["used"]), **st,
                samples=res["o"]["stats"]["samples"])
        return st


def _cfg1_chans(lo=0, hi=2):
    W0, W1 = synth.window_fx(0.05 * 255, 255)
    return [dict(c=0, lo=lo, hi=hi, W0=W0, W1=W1, tf=synth.tf_ramp())]


@pytest.fixture(scope="module")
def cfg1():
    return synth.config1_volume()


def test_cfg1_full_resident_axis_view(cfg1):
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    ids = p.gpu.all_ids()
    assert (p.upload(0, ids) == 1).all()
    p.check_page_table()
    p.check_masks()
    cam = synth.camera_ortho_axis((64, 64), 128, 128)
    res = p.frame(1, cam, 128, 128, 0.5, _cfg1_chans(0, 0), term_margin=1e-6, aov=True)
    p.check_frame(res, "cfg1-axis")
    assert res["tot"] == 0
    ok = aov_mask(res["o"])
    assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])
    # brute force at full resolution (all L0 resident); its image equals the
    # oracle frame's, so the frame's alternate outcomes apply to it as well
    fr, keep = oracle.make_frame(cam, 128, 128, 0.5, _cfg1_chans(0, 0))
    b = oracle.brute(p.V, cfg1.levels, 0, fr)
    assert np.abs(b - res["ref"]).max() < 1e-12
    compare_images(res["gpu"], b, res["o"]["amb_pix"], alt=oracle_alt(res["o"]))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cfg1_partial_residency_oblique(cfg1, seed):
    rng = np.random.default_rng(seed)
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    ids = p.gpu.all_ids()
    pick = ids[rng.random(len(ids)) < 0.45]
    rng.shuffle(pick)
    p.upload(0, pick)
    p.check_page_table()
    p.check_masks()
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), seed, 96, 80)
    res = p.frame(1, cam, 96, 80, 0.5, _cfg1_chans(0, 2), aov=True)
    p.check_frame(res, f"cfg1-partial-{seed}")
    ok = aov_mask(res["o"])
    assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])


def test_cfg1_substitution_levels(cfg1):
    """Only level-2 bricks (and a few level-1) resident, desired level 0:
    every sample uses the finest resident coarser level."""
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=20)
    ids = p.gpu.all_ids(levels=[2]).tolist() + p.gpu.all_ids(levels=[1]).tolist()[:3]
    p.upload(0, ids)
    p.check_masks()
    cam = synth.camera_ortho_axis((64, 64), 128, 128)
    res = p.frame(1, cam, 128, 128, 0.5, _cfg1_chans(0, 0), term_margin=1e-6, aov=True)
    p.check_frame(res, "cfg1-substitution")
    assert res["aov"][..., 0].sum() == 0
    assert res["aov"][..., 1].sum() > 0 and res["aov"][..., 2].sum() > 0


def test_skip_and_start_level_change_nothing(cfg1):
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    rng = np.random.default_rng(7)
    ids = p.gpu.all_ids()
    p.upload(0, ids[rng.random(len(ids)) < 0.6])
    p.gpu.tree.update_residency()
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 11, 96, 96)
    outs = []
    from paper_2309_04393_amd import resoct
    for f, (flags, sl) in enumerate([(resoct.RENDER_NO_SKIP, -1), (0, 0), (0, 1), (0, 2), (0, 3)]):
        r = p.gpu.render(1 + f, cam, 96, 96, 0.5, _cfg1_chans(0, 2), flags=flags, start_level=sl)
        torch.cuda.synchronize()
        ids_, cnt, nu, tot = p.gpu.cache.read_requests(1 << 20)
        used, _ = p.gpu.cache.read_usage(1 + f)
        outs.append((r["rgba"].cpu().numpy().copy(), ids_.copy(), cnt.copy(), np.sort(used)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]), "image changed"
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2]), "requests changed"
        assert np.array_equal(o[3], outs[0][3]), "usage changed"


def test_cfg1_perspective(cfg1):
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    rng = np.random.default_rng(4)
    ids = p.gpu.all_ids()
    p.upload(0, ids[rng.random(len(ids)) < 0.7])
    p.check_masks()
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    res = p.frame(1, cam, 100, 80, 0.5, _cfg1_chans(0, 2), lod_bias=0.6, aov=True)
    p.check_frame(res, "cfg1-persp")
    assert (res["aov"].sum(axis=(0, 1)) > 0).sum() >= 2  # several levels in use


def test_multichannel_ragged_u16():
    src = synth.BlobVolume((40, 24, 20), n_channels=3, bits=16, n_levels=3, seed=21, spacing=(1, 1, 2))
    p = Pair(src, 8, (4, 4, 4), 4, n_slots=60, max_batch=64)
    rng = np.random.default_rng(2)
    ids = p.gpu.all_ids()
    rng.shuffle(ids)
    p.upload(0, ids[: len(ids) // 2])
    p.upload(1, ids[len(ids) // 2:])  # more than the cache holds: evictions
    p.check_page_table()
    p.check_masks()
    chans = [dict(c=c, lo=0, hi=2, W0=3000 * 256, W1=60000 * 256, tf=synth.tf_hue(c / 3.0, 0.3))
             for c in (2, 0, 1)]
    cam = synth.camera_persp((70.0, -30.0, 60.0), (20, 12, 20), (0, 0, 1), 45.0, 1.0)
    res = p.frame(2, cam, 64, 64, 0.5, chans, lod_bias=0.8, aov=True)
    p.check_frame(res, "ragged-3ch")


def test_cells_reduced_config2():
    src = synth.CellVolume((256, 256, 64), 4, spacing=(1, 1, 4), n_levels=5, seed=2)
    src.levels = [[src.level_array(c, l) for l in range(src.n_levels)] for c in range(4)]
    p = Pair(src, 32, (16, 16, 4), 4, n_slots=200, max_batch=512)
    ids = p.gpu.all_ids()
    rng = np.random.default_rng(3)
    rng.shuffle(ids)
    p.upload(0, ids[:150])
    p.check_page_table()
    p.check_masks()
    chans = [dict(c=c, lo=0, hi=4, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / 4.0, 0.1)) for c in range(4)]
    cams = synth.orbit_path(src.dims, src.spacing, 2)
    res = p.frame(1, cams[1], 128, 128, 0.5, chans, aov=True)
    p.check_frame(res, "cells-4ch")


def test_adaptive_step_cfg1_perspective(cfg1):
    """LOD-adaptive step (Sec. 6.1): a perspective view whose samples fall in
    level bands 1 and 2 (sampling distances 2 and 4 base steps), every brick
    resident and then about half: images, requests and usage against the
    oracle's adaptive definition, and fewer samples than the plain step."""
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    flags = resoct.RENDER_ADAPTIVE_STEP
    for frac, seed in ((1.0, 0), (0.5, 7)):
        p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
        ids = p.gpu.all_ids()
        p.upload(0, ids[np.random.default_rng(seed).random(len(ids)) < frac])
        p.check_masks()
        res = p.frame(1, cam, 100, 80, 0.5, _cfg1_chans(0, 2), lod_bias=3.0, aov=True, flags=flags)
        p.check_frame(res, f"cfg1-adaptive-{frac}")
        ok = aov_mask(res["o"])
        assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])
        plain = p.frame(2, cam, 100, 80, 0.5, _cfg1_chans(0, 2), lod_bias=3.0)
        assert res["o"]["stats"]["samples"] < 0.8 * plain["o"]["stats"]["samples"]
        assert res["gpu"][..., 3].max() > 0.1


def test_adaptive_step_cells_channel_ranges():
    """Adaptive step with per-channel level ranges (Sec. 6.2): the finest
    desired level over the channels sets the distance (min of the ranges),
    four u16 channels, partial residency with substitution."""
    src = synth.CellVolume((256, 256, 64), 4, spacing=(1, 1, 4), n_levels=5, seed=2)
    src.levels = [[src.level_array(c, l) for l in range(src.n_levels)] for c in range(4)]
    p = Pair(src, 32, (16, 16, 4), 4, n_slots=200, max_batch=512)
    ids = p.gpu.all_ids()
    rng = np.random.default_rng(5)
    rng.shuffle(ids)
    p.upload(0, ids[:160])
    p.check_masks()
    ranges = [(1, 4), (2, 4), (1, 3), (3, 4)]
    chans = [dict(c=c, lo=lo, hi=hi, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / 4.0, 0.1))
             for c, (lo, hi) in enumerate(ranges)]
    cam = synth.camera_persp((380.0, -120.0, 420.0), (128, 128, 128), (0, 0, 1), 45.0, 1.0)
    res = p.frame(1, cam, 128, 128, 0.5, chans, lod_bias=1.5, aov=True, flags=resoct.RENDER_ADAPTIVE_STEP)
    p.check_frame(res, "cells-adaptive")
    ok = aov_mask(res["o"])
    assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])


def test_adaptive_step_at_finest_level_changes_nothing(cfg1):
    """Where the finest desired level is 0 the adaptive frame is the plain
    frame, bit for bit (images, requests, usage)."""
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(3).random(len(ids)) < 0.6])
    p.check_masks()
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 2, 96, 80)
    outs = []
    for f, flags in ((1, 0), (2, resoct.RENDER_ADAPTIVE_STEP)):
        r = p.gpu.render(f, cam, 96, 80, 0.5, _cfg1_chans(0, 0), flags=flags)
        torch.cuda.synchronize()
        ids_, cnt, nu, tot = p.gpu.cache.read_requests(1 << 20)
        used, _ = p.gpu.cache.read_usage(f)
        outs.append((r["rgba"].cpu().numpy().copy(), ids_.copy(), cnt.copy(), np.sort(used)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("W,H", [(1, 1), (7, 3), (33, 65)])
def test_tiny_and_ragged_viewports(cfg1, W, H):
    """Viewports smaller than one 8x8 block and not multiples of the 32x32
    tile: the blocks' pixels outside the image are never written and the
    image, requests and usage match the oracle."""
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(W * 100 + H).random(len(ids)) < 0.6])
    p.check_masks()  # residency update (the renderer reads residency from the octree masks)
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 30.0, W / H)
    sentinel = torch.full((W * H * 4 + 64,), -7.0, dtype=torch.float32, device="cuda")
    res = p.frame(1, cam, W, H, 0.5, _cfg1_chans(0, 2), lod_bias=0.6, out=sentinel)
    p.check_frame(res, f"ragged-{W}x{H}")
    assert (sentinel[W * H * 4:].cpu().numpy() == -7.0).all(), "wrote past the image"


def test_render_argument_errors(cfg1):
    """Frame descriptors the ABI rejects before any launch (RO_E_ARG):
    unknown flag bits, an empty viewport, an inverted level range."""
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 1, 16, 16)
    for kw, chans, W in ((dict(flags=16), _cfg1_chans(0, 2), 16), ({}, _cfg1_chans(0, 2), 0),
                         ({}, _cfg1_chans(2, 1), 16)):
        with pytest.raises(resoct.ResoctError) as e:
            p.gpu.render(1, cam, W, 16, 0.5, chans, **kw)
        assert e.value.code == -1
    r = p.gpu.render(1, cam, 16, 16, 0.5, _cfg1_chans(0, 2))  # still usable
    torch.cuda.synchronize()
    assert np.isfinite(gpu_rgba(r["rgba"], 16, 16)).all()


# ------------------------------------- render-and-skip of homogeneous nodes (row f2)

def _plateau_chans(n=2, lo=0, hi=0):
    """Hue tables with a faint haze (value 0 is visible, so the zero
    background is homogeneous, not empty)."""
    out = []
    for c in range(n):
        tf = synth.tf_hue(c / n, 0.06)
        tf[:, 3] = np.maximum(tf[:, 3], np.float32(0.004))
        out.append(dict(c=c, lo=lo, hi=hi, W0=0, W1=255 * 256, tf=tf))
    return out


@pytest.fixture(scope="module")
def plateau():
    return synth.plateau_volume(2)


def test_render_and_skip_full_residency(plateau):
    """Alg. 1 renderAndSkipNode with every brick resident and level 0
    desired: images, requests and usage match the oracle, and the image
    equals the plain frame to rounding (the node's value goes through the
    same table arithmetic as an interpolation of equal voxels; a node's
    samples are composited at once, so the colour sums round differently)
    with fewer brick reads and the same samples."""
    p = Pair(plateau, 16, (4, 4, 4), 4, n_slots=146)
    assert (p.upload(0, p.gpu.all_ids()) == 1).all()
    p.check_masks()
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 40.0, 1.0)
    stats, imgs = [], []
    for f, flags in ((1, 0), (2, resoct.RENDER_HOMOGENEOUS)):
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        res = p.frame(f, cam, 96, 96, 0.5, _plateau_chans(), stats=st, flags=flags)
        p.check_frame(res, f"rskip-full-{flags}")
        stats.append(st.cpu().numpy())
        imgs.append(res["gpu"])
    assert np.abs(imgs[0] - imgs[1]).max() < 1e-6
    assert stats[1][1] < 0.7 * stats[0][1]  # brick reads
    assert stats[1][0] == stats[0][0] and stats[1][6] > 0 and stats[0][6] == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_render_and_skip_partial_residency(plateau, seed):
    """Part of the bricks resident, levels 0..2: render-and-skip nodes
    neither request nor read, whatever is resident; images, request
    multisets and usage match the oracle."""
    p = Pair(plateau, 16, (4, 4, 4), 4, n_slots=146)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(seed).random(len(ids)) < 0.5])
    p.check_masks()
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 2 + seed, 96, 80)
    res = p.frame(1, cam, 96, 80, 0.5, _plateau_chans(2, 0, 2), lod_bias=0.7, flags=resoct.RENDER_HOMOGENEOUS)
    p.check_frame(res, f"rskip-partial-{seed}")


def test_homogeneous_in_some_channels_changes_nothing():
    """Channel 0 constant (homogeneous in every leaf), channel 1 varying in
    every leaf: no node is homogeneous for all channels, so the option
    changes nothing on the GPU (bit-identical image, same requests and
    reads, channel 0 read from its bricks) and both frames match the
    oracle."""
    arr = [np.full((32, 32, 32), 150, np.uint8),
           np.random.default_rng(3).integers(40, 251, (32, 32, 32)).astype(np.uint8)]
    src = synth.ArrayVolume(arr, 8, (1, 1, 1), 3)
    p = Pair(src, 8, (4, 4, 4), 3, n_slots=80)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(4).random(len(ids)) < 0.5])
    p.check_masks()
    chans = [dict(ch, hi=2) for ch in _plateau_chans(2)]
    cam = synth.camera_persp((70.0, 55.0, 48.0), (16, 15, 17), (0, 0, 1), 45.0, 1.0)
    out = []
    for f, flags in ((1, 0), (2, resoct.RENDER_HOMOGENEOUS)):
        res = p.frame(f, cam, 48, 48, 0.5, chans, lod_bias=0.6, flags=flags)
        p.check_frame(res, f"rskip-some-{flags}")
        out.append(res)
    assert np.array_equal(out[0]["gpu"], out[1]["gpu"])
    assert np.array_equal(out[0]["ids"], out[1]["ids"]) and np.array_equal(out[0]["cnt"], out[1]["cnt"])
    assert np.array_equal(out[0]["used"], out[1]["used"])
    ch0 = set(int(x) for x in p.gpu.cache.page_table_host()[:len(ids) // 2] if x != 0xFFFFFFFF)
    assert ch0 & set(int(x) for x in out[1]["used"])


@pytest.mark.parametrize("adaptive", [False, True])
def test_render_and_skip_with_aov_and_adaptive_step(plateau, adaptive):
    """The option in the AOV kernel and together with the LOD-adaptive step
    (the generic-edge instantiation): levels 0..2, about 60 % resident;
    images, requests, usage and per-level brick-read counts (which leave
    render-and-skip samples out) against the oracle."""
    p = Pair(plateau, 16, (4, 4, 4), 4, n_slots=146)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(11).random(len(ids)) < 0.6])
    p.check_masks()
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    flags = resoct.RENDER_HOMOGENEOUS | (resoct.RENDER_ADAPTIVE_STEP if adaptive else 0)
    res = p.frame(1, cam, 100, 80, 0.5, _plateau_chans(2, 0, 2), lod_bias=3.0 if adaptive else 0.8, aov=True,
                  flags=flags)
    p.check_frame(res, f"rskip-aov-{adaptive}")
    ok = aov_mask(res["o"])
    assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])


# --------------------------------------------- bricks required per pixel (row f4)

@pytest.mark.parametrize("case", ["cfg1-partial", "cells-ranges", "plateau-homog"])
def test_required_bricks_per_pixel(cfg1, plateau, case):
    """Sec. 8 (bricks required to be resident per pixel): the per-pixel count
    of distinct desired bricks of the samples that need data, against the
    oracle's sets, pixel for pixel (outside pixels with a close call); the
    image, requests and usage of the same frame match as well."""
    if case == "cfg1-partial":
        p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
        ids = p.gpu.all_ids()
        p.upload(0, ids[np.random.default_rng(3).random(len(ids)) < 0.5])
        chans, kw = _cfg1_chans(0, 2), dict(lod_bias=0.7)
        cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    elif case == "cells-ranges":
        src = synth.CellVolume((256, 256, 64), 4, spacing=(1, 1, 4), n_levels=5, seed=2)
        src.levels = [[src.level_array(c, l) for l in range(src.n_levels)] for c in range(4)]
        p = Pair(src, 32, (16, 16, 4), 4, n_slots=200, max_batch=512)
        ids = p.gpu.all_ids()
        np.random.default_rng(5).shuffle(ids)
        p.upload(0, ids[:160])
        chans = [dict(c=c, lo=lo, hi=hi, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / 4.0, 0.1))
                 for c, (lo, hi) in enumerate([(0, 4), (1, 4), (0, 3), (2, 4)])]
        kw = dict(lod_bias=1.5)
        cam = synth.camera_persp((380.0, -120.0, 420.0), (128, 128, 128), (0, 0, 1), 45.0, 1.0)
    else:
        p = Pair(plateau, 16, (4, 4, 4), 4, n_slots=146)
        ids = p.gpu.all_ids()
        p.upload(0, ids[np.random.default_rng(11).random(len(ids)) < 0.6])
        chans, kw = _plateau_chans(2, 0, 2), dict(lod_bias=0.8, flags=resoct.RENDER_HOMOGENEOUS)
        cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    p.check_masks()
    res = p.frame(1, cam, 96, 80, 0.5, chans, bricks=True, **kw)
    p.check_frame(res, f"bricks-{case}")
    ok = aov_mask(res["o"])
    ref = res["o"]["required_bricks"]
    assert ok.mean() > 0.99 and ref[ok].max() > 1
    bad = np.argwhere(ok & (res["bricks"] != ref))
    assert len(bad) == 0, f"{len(bad)} pixels differ, first {bad[:4]}: {res['bricks'][tuple(bad[0])]} vs {ref[tuple(bad[0])]}"
    _report(f"bricks-{case}", mean=float(ref.mean()), max=int(ref.max()))


# ------------------------------------------- per-channel sampling rates (row f1)

@pytest.mark.parametrize("aov", [False, True])
def test_channel_rates_cells(aov):
    """Per-channel sampling rates with the adaptive step (Sec. 6.1): four u16
    channels with different level ranges (Sec. 6.2), partial residency with
    substitution; images, requests, usage (and per-level reads and required
    bricks in the diagnostic kernel) against the oracle; fewer brick reads
    than the adaptive step alone."""
    src = synth.CellVolume((256, 256, 64), 4, spacing=(1, 1, 4), n_levels=5, seed=2)
    src.levels = [[src.level_array(c, l) for l in range(src.n_levels)] for c in range(4)]
    p = Pair(src, 32, (16, 16, 4), 4, n_slots=200, max_batch=512)
    ids = p.gpu.all_ids()
    np.random.default_rng(5).shuffle(ids)
    p.upload(0, ids[:170])
    p.check_masks()
    chans = [dict(c=c, lo=lo, hi=hi, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / 4.0, 0.1))
             for c, (lo, hi) in enumerate([(0, 4), (2, 4), (1, 3), (3, 4)])]
    cam = synth.camera_persp((380.0, -120.0, 420.0), (128, 128, 128), (0, 0, 1), 45.0, 1.0)
    flags = resoct.RENDER_ADAPTIVE_STEP | resoct.RENDER_CHANNEL_RATES
    st = torch.zeros(8, dtype=torch.int64, device="cuda")
    res = p.frame(1, cam, 112, 112, 0.5, chans, lod_bias=0.8, aov=aov, bricks=aov, stats=st, flags=flags)
    p.check_frame(res, f"rates-{aov}")
    if aov:
        ok = aov_mask(res["o"])
        assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])
        assert np.array_equal(res["bricks"][ok], res["o"]["required_bricks"][ok])
    st0 = torch.zeros(8, dtype=torch.int64, device="cuda")
    p.frame(2, cam, 112, 112, 0.5, chans, lod_bias=0.8, stats=st0, flags=resoct.RENDER_ADAPTIVE_STEP)
    st, st0 = st.cpu().numpy(), st0.cpu().numpy()
    _report(f"rates-{aov}", reads=int(st[1]), reads_adaptive=int(st0[1]))
    assert st[1] < 0.9 * st0[1]


def test_channel_rates_one_range_is_the_adaptive_frame(cfg1):
    """One level range for every channel: the option changes nothing on the
    GPU (bit-identical image, same requests and reads)."""
    p = Pair(cfg1, 16, (8, 8, 8), 3, n_slots=73)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(4).random(len(ids)) < 0.7])
    p.check_masks()
    cam = synth.camera_persp((120.0, 95.0, 80.0), (32, 30, 34), (0, 0, 1), 50.0, 1.25)
    out = []
    for f, flags in ((1, resoct.RENDER_ADAPTIVE_STEP), (2, resoct.RENDER_ADAPTIVE_STEP | resoct.RENDER_CHANNEL_RATES)):
        res = p.frame(f, cam, 100, 80, 0.5, _cfg1_chans(0, 2), lod_bias=1.5, flags=flags)
        p.check_frame(res, f"rates-one-{flags}")
        out.append(res)
    assert np.abs(out[0]["gpu"] - out[1]["gpu"]).max() < 1e-6
    assert np.array_equal(out[0]["ids"], out[1]["ids"]) and np.array_equal(out[0]["cnt"], out[1]["cnt"])
    assert np.array_equal(out[0]["used"], out[1]["used"])


@pytest.mark.parametrize("step,frac", [(2.5, 1.0), (2.5, 0.7), (4.5, 0.7)])
def test_traversal_depth_from_step(cfg1, step, frac):
    """Alg. 1 chooseTraversalDepth with the adaptive step: 4^3 leaves, samples
    2 x 2.5 or 2 x 4.5 world units apart, so emptiness is decided one or two
    tree levels above the leaves; images, requests, usage and per-level reads
    against the oracle, with full and partial residency."""
    p = Pair(cfg1, 16, (4, 4, 4), 4, n_slots=73)
    ids = p.gpu.all_ids()
    p.upload(0, ids[np.random.default_rng(2).random(len(ids)) < frac])
    p.check_masks()
    cam = synth.camera_oblique_ortho((64, 64, 64), (1, 1, 1), 3, 64, 64)
    flags = resoct.RENDER_ADAPTIVE_STEP | resoct.RENDER_TRAVERSAL_DEPTH
    res = p.frame(1, cam, 64, 64, step, _cfg1_chans(0, 2), lod_bias=1.5, aov=True, flags=flags)
    p.check_frame(res, f"tdepth-{step}-{frac}")
    ok = aov_mask(res["o"])
    assert ok.mean() > 0.99 and np.array_equal(res["aov"][ok], res["o"]["aov"][ok])
