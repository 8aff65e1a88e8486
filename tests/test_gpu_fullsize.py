"""Parity at the full 16-channel 8192 x 8192 x 192 workload the bench times:
a 128 x 128 window of the mid-path fly-through frame (same rays as the
1920 x 1080 frame's window) rendered on the GPU against the oracle, with the
cache empty, then partially resident with coarser substitutes for part of
the missing bricks.  Images, request multisets and the set of bricks read
are compared."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import compare_images, compare_requests, gpu_rgba, oracle_alt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import bench  # noqa: E402
from paper_2309_04393_amd import resoct  # noqa: E402
from paper_2309_04393_amd.pipeline import GpuScene  # noqa: E402
from tests.test_gpu_render import _report  # noqa: E402

TILE = 128
# A pixel is ambiguous when a discrete decision of the oracle lies within its
# margin (positions within 1e-9 of a cell or level boundary) or when a ray
# makes two termination calls within 1e-6 of the threshold; a single close
# termination call is not ambiguous, the oracle gives both valid outcomes.
MAX_AMB = 1e-3


def test_cfg3_window_parity():
    """The timed frame (mid-path, every sample at level 0)."""
    _window_parity(bench.config("cfg3")["f0"], 0, 3, 0, "cfg3-window")


def test_cfg3_adaptive_window_parity():
    """A zoomed-out frame of the same path (its samples want level 2) with
    the LOD-adaptive step; level data materialised for levels 2 and 3."""
    _window_parity(40, resoct.RENDER_ADAPTIVE_STEP, 4, 2, "cfg3-adaptive-window")


def _window_parity(f, flags, need, first, name):
    cfg = bench.config("cfg3")
    vol = cfg["vol"]
    scene = GpuScene(vol, cfg["B"], cfg["leaf"], cfg["depth"], 60000, max_batch=4096,
                     start_level=cfg["start_level"], set_metadata=False)
    mm = bench.leaf_mm_all(cfg)
    for c in range(vol.n_channels):
        scene.set_metadata(c, mm[c])
    cams = synth.flythrough_path(vol.dims, vol.spacing, cfg["n_frames"], bench.tissue_target(vol, cfg["seed"]))
    chans = [dict(ch, hi=vol.n_levels - 1) for ch in bench.channels(vol.n_channels, cfg["seed"])]
    step = 0.5 * min(vol.spacing)
    W, H = cfg["W"], cfg["H"]
    x0, y0 = (W - TILE) // 2, (H - TILE) // 2
    cam = cams[f]
    sub = bench.sub_camera(cam, W, H, x0, y0, TILE)
    adaptive = bool(flags & resoct.RENDER_ADAPTIVE_STEP)
    V, levels, boxes, lm, fr = bench.oracle_window(cfg, cam, W, H, x0, y0, TILE, step, chans, need=need,
                                                   first=first, adaptive=adaptive)
    ids_all = oracle.dense_ids(V)
    dense_of = {int(i): k for k, i in enumerate(ids_all)}

    # 1. empty cache: nothing drawn, every desired brick requested
    r = scene.render(1, sub, TILE, TILE, step, chans, flags=flags)
    torch.cuda.synchronize()
    g_ids, g_cnt, nu, tot = scene.cache.read_requests(1 << 20)
    empty = np.full(len(ids_all), -1, np.int32)
    o = oracle.render(V, levels, empty, lm, fr, 1, boxes=boxes)
    assert not np.isnan(o["rgba"]).any()
    n_req = compare_requests(g_ids, g_cnt, o["counts"], o["amb_counts"], ids_all)
    compare_images(gpu_rgba(r["rgba"], TILE, TILE), o["rgba"], o["amb_pix"], max_amb_frac=MAX_AMB,
                   alt=oracle_alt(o))
    _report(f"{name}-empty", requests=n_req, missing=tot, samples=o["stats"]["samples"])

    # 2. three quarters of the requested bricks resident; for half of the
    # others the level above is resident instead (substitution)
    rng = np.random.default_rng(11)
    req = np.sort(g_ids)
    keep = rng.random(len(req)) < 0.75
    up = list(req[keep])
    for i in req[~keep][: len(req[~keep]) // 2]:
        c, l, b = scene.vol.decode(int(i))
        if l + 1 < vol.n_levels:
            _, lf, _ = scene.vol.levels()
            f0, f1 = lf[l], lf[l + 1]
            pb = tuple(int(b[a] * f0[a] // f1[a]) for a in range(3))
            up.append(scene.vol.encode(c, l + 1, pb))
    up = np.unique(np.array(up, np.uint32))
    assert len(up) < 60000
    scene.upload(2, up)
    scene.tree.update_residency()
    res = np.full(len(ids_all), -1, np.int32)
    for k, i in enumerate(up):
        res[dense_of[int(i)]] = k
    r = scene.render(3, sub, TILE, TILE, step, chans, flags=flags)
    torch.cuda.synchronize()
    g_ids, g_cnt, nu, tot = scene.cache.read_requests(1 << 20)
    used_slots, n_used = scene.cache.read_usage(3)
    o = oracle.render(V, levels, res, lm, fr, len(up), boxes=boxes)
    assert not np.isnan(o["rgba"]).any()
    st = compare_images(gpu_rgba(r["rgba"], TILE, TILE), o["rgba"], o["amb_pix"], max_amb_frac=MAX_AMB,
                   alt=oracle_alt(o))
    n_req = compare_requests(g_ids, g_cnt, o["counts"], o["amb_counts"], ids_all)
    # bricks read: GPU slots mapped through its page table (dense brick
    # order, as the ABI defines it), oracle slots are ranks in `up`
    pt = scene.cache.page_table_host()
    occ = np.nonzero(pt != 0xFFFFFFFF)[0]
    slot_to_id = dict(zip(pt[occ].tolist(), ids_all[occ].tolist()))
    g_read = {slot_to_id[int(s)] for s in used_slots}
    o_read = {int(up[s]) for s in np.nonzero(o["used"])[0]}
    o_amb = {int(up[s]) for s in np.nonzero(o["amb_used"])[0]}
    assert o_read <= g_read <= o_read | o_amb
    _report(f"{name}-partial", uploaded=len(up), requests=n_req, missing=tot, read=len(o_read), **st)
