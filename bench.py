#!/usr/bin/env python3
"""Benchmark of the residency-octree hot path on one MI355X.

One step = one frame of the whole path: ray casting over the residency
octree (traversal, empty-space skipping, desired level, page-table lookup,
substitution, trilinear sampling, per-channel transfer functions, channel
mix, front-to-back compositing, request and usage recording), request
compaction and readback, the plain request-driven upload policy, the LRU
streaming batch (slot choice, page-table update, brick scatter) and the
residency-octree update.

Workload (default): 16 channels of uint16, 8192 x 8192 x 192 voxels
(z spacing 3), Poisson-placed cells under a low-frequency tissue mask,
32^3 bricks with a one-voxel halo, 9 levels, 16 GiB brick cache, a
1920 x 1080 perspective fly-through (300 frames) from the whole slide down
to single cells; the timed frames sit mid-path at about one voxel per pixel.

Inputs are resident in HBM when the timed region starts: the cache is warmed
along the path with bricks from the host generator (the data server), then
the K timed frames are run once untimed from a device-side checkpoint to
collect the bricks they will upload, the checkpoint is restored, and the same
K frames are timed with those bricks already in device memory.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples/s & ms/frame @1080p 16ch; HBM GB/s; frames-to-converge; p99 latency"
HBM_PEAK_GBS = 8000.0


def profiled_traffic(workload):
    """HBM bytes per k_render launch from the committed rocprofv3 summary of
    this workload (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known
    size), or None when the summary is missing or the kernel's sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_render-{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    if "<!-- roofline" not in txt:
        return None
    block = txt.split("<!-- roofline", 1)[1].split("-->", 1)[0]
    kv = dict(line.split(": ", 1) for line in block.strip().splitlines() if ": " in line)
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256() or kv.get("workload") != workload:
        return None
    return float(kv["traffic_bytes_per_launch"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("render_core.h", "render.hip"):
        h.update(open(os.path.join(ROOT, "paper_2309_04393_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def profile_summary(trace_dir, fetch_dir, write_dir, last, workload, kernel="k_render<16, 2, false, 34, 0>"):
    """Markdown summary of rocprofv3 runs of the headline frame loop: mean
    duration of the last `last` dispatches of the headline kernel (the timed
    pass; the untimed pass A and the warm-up frames come before it) from the
    kernel trace, and FETCH_SIZE / WRITE_SIZE of the same dispatches, scaled by
    what the counters read for the 1 GiB device copy (--copy-calibration)."""
    tr = [r for r in _csv_rows(trace_dir, "kernel_trace.csv") if kernel in r["Kernel_Name"]]
    tr.sort(key=lambda r: int(r["Dispatch_Id"]))
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in tr]
    sel = dur[-last:]

    def counter(d, name):
        rows = _csv_rows(d, "counter_collection.csv")
        k = sorted((r for r in rows if kernel in r["Kernel_Name"] and r["Counter_Name"].startswith(name)),
                   key=lambda r: int(r["Dispatch_Id"]))
        # the calibration copies are the largest copies after the last frame
        # (earlier copies are set-up and uploads of other sizes)
        end = int(k[-1]["Dispatch_Id"]) if k else -1
        cp = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
              and r["Counter_Name"].startswith(name) and int(r["Dispatch_Id"]) > end]
        return [float(r["Counter_Value"]) for r in k][-last:], (max(cp) if cp else None)

    fetch, fcopy = counter(fetch_dir, "FETCH_SIZE")
    write, wcopy = counter(write_dir, "WRITE_SIZE")
    gib_kib = (1 << 30) / 1024.0
    fs = gib_kib / fcopy if fcopy else 1.0
    ws = gib_kib / wcopy if wcopy else 1.0
    traffic = (np.mean(fetch) * fs + np.mean(write) * ws) * 1024.0
    mean_ms = float(np.mean(sel))
    lines = [f"* `{kernel}`: {len(tr)} dispatches; the last {len(sel)} (the timed pass): mean {mean_ms:.3f} ms, "
             f"min {min(sel):.3f}, max {max(sel):.3f}.",
             f"* Copy calibration: FETCH_SIZE {fcopy} KiB and WRITE_SIZE {wcopy} KiB for a 1 GiB copy; factors "
             f"{fs:.4f} and {ws:.4f}.",
             f"* Per timed launch: FETCH_SIZE {np.mean(fetch):.4g} KiB, WRITE_SIZE {np.mean(write):.4g} KiB -> "
             f"{traffic / 1e9:.2f} GB = {traffic / 1e9 / (mean_ms / 1e3):.0f} GB/s of fabric traffic.",
             "", "<!-- roofline", f"workload: {workload}", f"kernel_sources_sha256: {kernel_sources_sha256()}",
             f"mean_ms_timed_launches: {mean_ms:.4f}", f"traffic_bytes_per_launch: {traffic:.0f}", "-->"]
    return "\n".join(lines)


def config(name):
    import synth
    if name == "cfg3":
        vol = synth.config3_volume()
        return dict(name="16ch-8192x8192x192-u16-1080p", vol=vol, B=32, leaf=(16, 16, 8), depth=9,
                    n_slots=218551, U=2048, W=1920, H=1080, n_frames=300, f0=150, start_level=2,
                    path="fly", seed=3)
    if name == "cfg2":
        vol = synth.config2_volume()
        return dict(name="4ch-2048x2048x64-u16-1024p", vol=vol, B=32, leaf=(16, 16, 4), depth=7,
                    n_slots=27318, U=512, W=1024, H=1024, n_frames=120, f0=60, start_level=2,
                    path="orbit", seed=2)
    raise SystemExit(f"unknown config {name}")


def channels(n, seed):
    import synth
    rng = np.random.default_rng(seed + 100)
    out = []
    for c in range(n):
        j = rng.uniform(0.8, 1.2, 2)
        W0, W1 = synth.window_fx(300 * j[0], 8000 * j[1])
        out.append(dict(c=c, lo=0, W0=W0, W1=W1, tf=synth.tf_hue(c / n, 0.1)))
    return out


def tissue_target(vol, seed):
    import synth
    rng = np.random.default_rng(seed + 7)
    L = synth.lib()
    for _ in range(10000):
        x, y = rng.uniform(0.25, 0.75, 2) * np.array(vol.dims[:2])
        if L.synth_tissue(vol._ctx, float(x), float(y)) > 0.95:
            return (x * vol.spacing[0], y * vol.spacing[1], vol.dims[2] * vol.spacing[2] / 2)
    return tuple(np.array(vol.dims) * np.array(vol.spacing) / 2)


class Frames:
    """Frame loop over the GPU scene (plain request-driven streaming)."""

    def __init__(self, scene, cams, chans, W, H, U, step):
        import torch
        self.torch = torch
        self.s = scene
        self.cams = cams
        self.chans = chans
        self.W, self.H, self.U, self.step = W, H, U, step
        self.tf = scene.tf_tensor(chans)
        self.out = torch.empty(W * H * 4, dtype=torch.float32, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.int64, device="cuda")

    def render(self, f, cam_index=None):
        return self.s.render(f, self.cams[f if cam_index is None else cam_index], self.W, self.H,
                             self.step, self.chans, tf_dev=self.tf, out=self.out,
                             stats=self.stats)

    def plan(self, cap=1 << 20):
        ids, cnt, nu, tot = self.s.cache.read_requests(cap)
        order = np.lexsort((ids, -cnt.astype(np.int64)))  # count desc, id asc
        return ids[order][: self.U], tot, nu

    def step_frame(self, f, staged=None):
        """One full step; returns (upload ids, staged tensor, missing)."""
        self.render(f)
        ids, tot, nu = self.plan()
        self.last_nu = nu
        if staged is None:
            staged = self.s.stage(ids) if len(ids) else None
        if len(ids):
            self.s.cache.stream_bricks(f, ids, staged)
        self.s.tree.update_residency()
        return ids, staged, tot


def snapshot(scene):
    import torch
    dev = {("c", k): v.clone() for k, v in scene.cache.t.items() if k != "scratch"}
    dev.update({("t", k): v.clone() for k, v in scene.tree.t.items() if k != "scratch"})
    torch.cuda.synchronize()
    return dev, scene.cache.save_state()


def restore(scene, snap):
    import torch
    dev, host = snap
    for (kind, k), v in dev.items():
        (scene.cache.t if kind == "c" else scene.tree.t)[k].copy_(v)
    torch.cuda.synchronize()
    scene.cache.load_state(host)


def oracle_window(cfg, cam, W, H, x0, y0, tile, step, chans, need=2, first=0, adaptive=False):
    """Oracle inputs for the tile x tile pixel window at (x0, y0) of a W x H
    frame: the volume description, level data materialised (levels first ..
    need - 1) over the bounding box of the window's rays, the boxes, leaf
    metadata and the oracle frame of the window's sub-camera."""
    import oracle
    vol = cfg["vol"]
    V = oracle.make_volume(vol.dims, vol.spacing, vol.n_channels, 16, cfg["B"], vol.n_levels, cfg["leaf"],
                           cfg["depth"])
    eye = np.array(cam["eye"]) / np.array(vol.spacing)
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    edge = [(i, y0) for i in range(x0, x0 + tile)] + [(i, y0 + tile - 1) for i in range(x0, x0 + tile)] + \
           [(x0, j) for j in range(y0, y0 + tile)] + [(x0 + tile - 1, j) for j in range(y0, y0 + tile)]
    dims = np.array(vol.dims, dtype=np.float64)
    for (i, j) in edge:
        a = (2 * i + 1 - W) / W
        b = (H - 2 * j - 1) / H
        d = np.array(cam["F"]) + a * cam["tx"] * np.array(cam["R"]) + b * cam["ty"] * np.array(cam["U"])
        d = d / np.linalg.norm(d) / np.array(vol.spacing)
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = np.where(d != 0, (0 - eye) / d, -np.inf)
            t1 = np.where(d != 0, (dims - eye) / d, np.inf)
        ta, tb = np.max(np.minimum(t0, t1)), np.min(np.maximum(t0, t1))
        if ta > tb:
            continue
        for t in (ta, tb):
            p = eye + t * d
            lo = np.minimum(lo, p)
            hi = np.maximum(hi, p)
    lo = np.clip(np.floor(lo) - 2, 0, dims - 1).astype(int)
    hi = np.clip(np.ceil(hi) + 2, 1, dims).astype(int)
    ldims, lf, _ = oracle.level_info(V)
    if need is None:
        # levels the window's samples desire (every brick resident): from the
        # distance range of a grid of its rays through the volume
        assert cam["proj"] == "persp"
        ts = []
        for i in np.linspace(x0, x0 + tile - 1, 17):
            for j in np.linspace(y0, y0 + tile - 1, 17):
                a = (2 * i + 1 - W) / W
                b = (H - 2 * j - 1) / H
                d = np.array(cam["F"]) + a * cam["tx"] * np.array(cam["R"]) + b * cam["ty"] * np.array(cam["U"])
                d = d / np.linalg.norm(d) / np.array(vol.spacing)
                with np.errstate(divide="ignore", invalid="ignore"):
                    t0 = np.where(d != 0, (0 - eye) / d, -np.inf)
                    t1 = np.where(d != 0, (dims - eye) / d, np.inf)
                ta, tb = np.max(np.minimum(t0, t1)), np.min(np.maximum(t0, t1))
                if ta <= tb:
                    ts += [max(ta, 0.0), tb]
        pix = 2.0 * cam["ty"] / H
        D = [float(lf[l][0]) * vol.spacing[0] / pix for l in range(1, vol.n_levels)]
        lev = lambda t: sum(1 for x in D if t >= x)
        first = lev(min(ts) * (1 - 1e-3)) if ts else 0
        need = lev(max(ts) * (1 + 1e-3)) + 1 if ts else 1
    levels, boxes = [], np.zeros((vol.n_channels, vol.n_levels, 6), np.int32)
    per_level = []
    for l in range(vol.n_levels):
        if l >= need or l < first:
            per_level.append(None)
            continue
        a = lo // lf[l]
        b = np.minimum(-(-hi // lf[l]) + 1, ldims[l])
        reg = vol.region(l, int(a[0]), int(a[1]), int(a[2]), int(b[0] - a[0]), int(b[1] - a[1]),
                         int(b[2] - a[2]))
        per_level.append((reg, a, b - a))
    for c in range(vol.n_channels):
        row = []
        for l in range(vol.n_levels):
            if per_level[l] is None:
                row.append(np.zeros((1, 1, 1), np.uint16))
                boxes[c, l] = [0, 0, 0, 1, 1, 1]
            else:
                reg, a, n = per_level[l]
                row.append(np.ascontiguousarray(reg[c]))
                boxes[c, l] = [a[0], a[1], a[2], n[0], n[1], n[2]]
        levels.append(row)
    lm = leaf_mm_all(cfg)
    fr, keep = oracle.make_frame(sub_camera(cam, W, H, x0, y0, tile), tile, tile, step,
                                 [dict(ch, hi=vol.n_levels - 1) for ch in chans], term_margin=1e-6,
                                 adaptive=adaptive)
    return V, levels, boxes, lm, fr


def cpu_baseline(cfg, cams, chans, f, step, tile):
    """The oracle on a tile x tile pixel window at the centre of frame f,
    every brick resident (samples read their desired level), level data
    materialised for the window's rays from the generator."""
    import oracle
    W, H = cfg["W"], cfg["H"]
    x0, y0 = (W - tile) // 2, (H - tile) // 2
    V, levels, boxes, lm, fr = oracle_window(cfg, cams[f], W, H, x0, y0, tile, step, chans, need=None)
    res = np.arange(oracle.brick_count(V), dtype=np.int32)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t = time.perf_counter()
    r = oracle.render(V, levels, res, lm, fr, 1, n_threads=threads, boxes=boxes)
    dt = time.perf_counter() - t
    assert not np.isnan(r["rgba"]).any(), "oracle sampled outside the materialised window"
    s = r["stats"]["samples"]
    # one host thread on a quarter-edge window at the same centre
    t1 = max(tile // 4, 8)
    x1, y1 = (W - t1) // 2, (H - t1) // 2
    V1, lv1, bx1, lm1, fr1 = oracle_window(cfg, cams[f], W, H, x1, y1, t1, step, chans, need=None)
    t = time.perf_counter()
    r1 = oracle.render(V1, lv1, res, lm1, fr1, 1, n_threads=1, boxes=bx1)
    dt1 = time.perf_counter() - t
    s1 = r1["stats"]["samples"]
    return dict(value=s / dt, unit="samples/s", cores=threads, kind="oracle",
                sample=f"{tile}x{tile}-pixel window at the centre of timed frame {f}, all bricks resident, "
                       f"{s} ray samples x {len(chans)} channels in {dt:.1f} s",
                single_core_value=s1 / dt1,
                single_core_sample=f"{t1}x{t1}-pixel window at the same centre, one thread, {s1} ray samples "
                                   f"in {dt1:.1f} s"), r, (x0, y0)


def sub_camera(cam, W, H, x0, y0, n):
    """Camera whose n x n image is the window [x0, x0+n) x [y0, y0+n) of the
    W x H image of `cam` (same rays: perspective only)."""
    assert cam["proj"] == "persp"
    # pixel i of the window = pixel x0 + i of the full image:
    # a_full = (2 (x0+i) + 1 - W) / W = ((2i + 1 - n) / n) * (n / W) + (2 x0 + n - W) / W
    F = np.array(cam["F"]) + ((2 * x0 + n - W) / W) * cam["tx"] * np.array(cam["R"]) + \
        ((H - 2 * y0 - n) / H) * cam["ty"] * np.array(cam["U"])
    return dict(proj="persp", eye=cam["eye"], F=list(F), R=cam["R"], U=cam["U"], tx=cam["tx"] * n / W,
                ty=cam["ty"] * n / H)


_LM = {}


def leaf_grid(dims, leaf, depth):
    n = []
    for a in range(3):
        nl = -(-dims[a] // leaf[a])
        s = 0
        while (1 << s) < nl:
            s += 1
        n.append(1 << s)
    return tuple(n)


def leaf_mm_all(cfg):
    key = cfg["name"]
    if key not in _LM:
        vol = cfg["vol"]
        lg = leaf_grid(vol.dims, cfg["leaf"], cfg["depth"])
        mx = vol.leaf_max_all(cfg["leaf"], lg)
        mm = np.zeros((vol.n_channels, mx.shape[1], 2), np.uint16)
        mm[:, :, 1] = mx
        _LM[key] = mm
    return _LM[key]


def streaming_bench(scene, fl, cams, f_req, f_up, U, mm0):
    """Timing of the streaming steps on the paper-scale scene (after the
    timed frames): request compaction (readback of the dense counters after
    rendering the zoomed-out frame f_req, which misses many bricks), the
    upload of the U most requested bricks (slot choice, LRU eviction,
    scatter, page tables), the residency update of those bricks, the
    from-scratch residency rebuild and the metadata reduction of one
    channel.  GPU time from HIP events on the library's stream (torch's
    current stream); algorithmic bytes per call as stated per entry."""
    import torch

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        r = fn()
        b.record()
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    def entry(ms, nbytes, **kw):
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
        return dict(ms=ms, alg_bytes=int(nbytes), achieved_GBs=gbs,
                    frac_hbm_peak=gbs / HBM_PEAK_GBS if gbs is not None else None, **kw)

    c = scene.cache
    out = {"workload": "16ch-8192x8192x192-u16, 218551 slots, state after the timed frames",
           "request_frame": f_req, "upload_frame": f_up}
    fl.render(f_req)
    (ids, cnt, nu, tot), ms = timed(lambda: c.read_requests(1 << 22))
    out["a8_request_compaction"] = entry(ms, 4 * c.n_bricks + 12 * nu, bricks_scanned=c.n_bricks,
                                         distinct_requested=nu, missing_samples=tot,
                                         note="4 B per counter read + (ID, count) out + counter cleared per "
                                              "requested brick; includes the host readback")
    order = np.lexsort((ids, -cnt.astype(np.int64)))
    up = ids[order][:U]
    staged = scene.stage(up)
    flags, ms = timed(lambda: c.stream_bricks(f_up, up, staged))
    n_in = int((flags == 1).sum())
    out["a9_upload"] = entry(ms, 2 * len(up) * c.slot_stride + 8 * c.n_slots, bricks=len(up), inserted=n_in,
                             note="staging read + slot write per brick, (stamp, sequence) of every slot "
                                  "once; includes the LRU selection and the host flags readback")
    _, ms = timed(lambda: scene.tree.update_residency())
    out["a10_residency_update"] = dict(ms=ms, dirty_bricks=2 * n_in)
    _, ms = timed(lambda: scene.tree.rebuild_residency())
    m = scene.vol.n_channels
    out["a10_residency_rebuild"] = entry(ms, 2 * scene.tree.n_nodes * m + 4 * c.n_bricks,
                                         note="every node mask written once, every page-table entry read once")
    t = torch.from_numpy(np.ascontiguousarray(mm0, dtype=np.uint16).reshape(-1).view(np.int16)).to("cuda") \
        .view(torch.uint16)
    _, ms = timed(lambda: scene.tree.set_leaf_metadata(0, t))
    out["a11_metadata_one_channel"] = entry(ms, 4 * scene.tree.n_leaves + 4 * scene.tree.n_nodes,
                                            note="leaf (min, max) read + one metadata word written per node")
    # metadata computed from the voxels of the uploaded channel-0 bricks;
    # then the server's metadata of channel 0 is restored
    L = scene.vol.n_levels
    c0 = up[(up >> 24) // L == 0]
    if len(c0):
        n_up = scene.tree.n_nodes - scene.tree.n_leaves
        lg = scene.tree.leaf_grid
        leaves = 0
        for i in c0:  # leaves of the padded grid inside each brick
            _, l, b = scene.vol.decode(int(i))
            n = 1
            for a in range(3):
                per = scene.B * int(scene.lf[l][a]) // scene.leaf[a]
                n *= max(min((b[a] + 1) * per, lg[a]) - b[a] * per, 0)
            leaves += n
        _, ms = timed(lambda: scene.tree.leaf_metadata_from_bricks(c0))
        out["f3_metadata_from_bricks"] = entry(
            ms, len(c0) * c.slot_stride + 4 * leaves + 36 * n_up, bricks=len(c0), leaves=leaves,
            note="each brick's slot read once + one metadata word per leaf inside the bricks + the inner "
                 "nodes of the channel reduced again (8 children read, 1 written); includes the host "
                 "work-list copy")
        scene.tree.set_leaf_metadata(0, t)
        torch.cuda.synchronize()
    return out


def adaptive_bench(scene, fl, frames, reps=3):
    """The LOD-adaptive step (RO_RENDER_ADAPTIVE_STEP) on zoomed-out frames of
    the fly-through, where samples fall in coarse level bands: each frame's
    working set is made resident (bulk uploads of its requests), then the
    frame is rendered with the plain and with the adaptive step; mean kernel
    time from HIP events and the ray samples evaluated."""
    import torch
    from paper_2309_04393_amd import resoct
    out = {}
    for f in frames:
        for it in range(3):
            fl.render(f)
            ids, cnt, nu, tot = scene.cache.read_requests(1 << 22)
            log(f"adaptive step, frame {f}: warm-up {it}: {nu} bricks requested")
            if nu == 0:
                break
            order = np.lexsort((ids, -cnt.astype(np.int64)))
            ids = ids[order][: scene.cache.n_slots]
            t = time.perf_counter()
            scene.upload(f, ids)
            scene.tree.update_residency()
            torch.cuda.synchronize()
            log(f"  uploaded {len(ids)} bricks in {time.perf_counter() - t:.1f} s")
        row = {}
        for name, flags in (("plain", 0), ("adaptive", resoct.RENDER_ADAPTIVE_STEP)):
            ms = []
            for _ in range(reps):
                fl.stats.zero_()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record()
                scene.render(f, fl.cams[f], fl.W, fl.H, fl.step, fl.chans, tf_dev=fl.tf, out=fl.out,
                             stats=fl.stats, flags=flags)
                b.record()
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b))
            st = fl.stats.cpu().numpy()
            _, _, nu2, tot2 = scene.cache.read_requests(1 << 22)
            row[name] = dict(ms=float(np.mean(ms)), samples=int(st[0]), channel_samples=int(st[1]),
                             missing_samples=int(tot2), leaf_visits=int(st[3]),
                             lane_busy=float(st[0]) / max(float(st[5]), 1.0))
        row["speedup"] = row["plain"]["ms"] / row["adaptive"]["ms"]
        # per-channel sampling rates (Sec. 6.1) with mixed per-channel level
        # ranges (Sec. 6.2, Fig. 6): channel c at levels >= 2 (c mod 4), a
        # quarter of the channels at full resolution and the others two,
        # four and six levels coarser; the mixed frame's working set is made
        # resident first
        mixed = [dict(ch, lo=min(2 * (c % 4), ch["hi"])) for c, ch in enumerate(fl.chans)]
        for it in range(3):
            scene.render(f, fl.cams[f], fl.W, fl.H, fl.step, mixed, tf_dev=fl.tf, out=fl.out,
                         flags=resoct.RENDER_ADAPTIVE_STEP)
            ids, cnt, nu, tot = scene.cache.read_requests(1 << 22)
            if nu == 0:
                break
            order = np.lexsort((ids, -cnt.astype(np.int64)))
            scene.upload(f, ids[order][: scene.cache.n_slots])
            scene.tree.update_residency()
            torch.cuda.synchronize()
        for name, flags in (("mixed_ranges", resoct.RENDER_ADAPTIVE_STEP),
                            ("mixed_ranges_channel_rates", resoct.RENDER_ADAPTIVE_STEP | resoct.RENDER_CHANNEL_RATES)):
            ms = []
            for _ in range(reps):
                fl.stats.zero_()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record()
                scene.render(f, fl.cams[f], fl.W, fl.H, fl.step, mixed, tf_dev=fl.tf, out=fl.out,
                             stats=fl.stats, flags=flags)
                b.record()
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b))
            st = fl.stats.cpu().numpy()
            _, _, nu2, tot2 = scene.cache.read_requests(1 << 22)
            row[name] = dict(ms=float(np.mean(ms)), samples=int(st[0]), channel_samples=int(st[1]),
                             missing_samples=int(tot2), lane_busy=float(st[0]) / max(float(st[5]), 1.0))
        row["channel_rates_speedup"] = row["mixed_ranges"]["ms"] / row["mixed_ranges_channel_rates"]["ms"]
        row["channel_rates_read_ratio"] = (row["mixed_ranges_channel_rates"]["channel_samples"]
                                           / max(row["mixed_ranges"]["channel_samples"], 1))
        out[str(f)] = row
        log(f"adaptive step, frame {f}: {row}")
    return out


def homogeneous_bench(frames=(0, 12), reps=7, W=1920, H=1080, haze=0.05):
    """Render-and-skip of nodes homogeneous for all channels
    (RO_RENDER_HOMOGENEOUS) on two fully resident 4-channel 1024x1024x64
    u16 volumes whose leaf metadata are computed on the GPU from the level-0
    bricks (exact, so a constant region has min == max): the cell volume
    (cells on an empty background) and constant boxes on an empty
    background.  Channels 0 and 2 show a faint haze at the low values (value
    0 is visible), 1 and 3 are empty there, so background nodes are
    homogeneous or empty in every channel; box interiors are homogeneous.
    Each orbit frame is rendered plain and with the option, once untimed and
    then `reps` times: median kernel time from HIP events, samples, brick
    reads, distinct bricks read, samples rendered from homogeneous nodes,
    wave iterations, and the largest image difference (zero where level 0 is
    read; a coarse level's interpolation may differ from the node's
    value)."""
    import torch
    import synth
    from paper_2309_04393_amd import resoct
    from paper_2309_04393_amd.pipeline import GpuScene
    out = {"image": [W, H], "workloads": {}}
    for wname, make, wins in (
            ("4ch-1024x1024x64-u16 cells", lambda: synth.CellVolume((1024, 1024, 64), 4, spacing=(1, 1, 4),
                                                                   n_levels=6, seed=2), (100, 2000)),
            ("4ch-1024x1024x64-u16 constant boxes", lambda: synth.box_plateau_volume(), (50 * 256, 255 * 256))):
        vol = make()
        t = time.perf_counter()
        n_all = resoct.Volume(vol.dims, vol.spacing, 4, 2, 32, vol.n_levels).brick_count()
        scene = GpuScene(vol, 32, (16, 16, 4), 6, n_all, max_batch=4096, set_metadata=False)
        for c in range(4):
            scene.set_unknown(c)
        ids = scene.all_ids()
        scene.upload(0, ids)
        scene.tree.update_residency()
        torch.cuda.synchronize()
        log(f"homogeneous leaves ({wname}): {len(ids)} bricks resident ({time.perf_counter() - t:.1f} s)")
        l0 = scene.all_ids(levels=[0])
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        scene.tree.leaf_metadata_from_bricks(l0)
        b.record()
        torch.cuda.synchronize()
        res = {"metadata_from_bricks_ms": a.elapsed_time(b), "level0_bricks": len(l0)}
        chans = []
        for c in range(4):
            tf = synth.tf_hue(c / 4.0, 0.1)
            if c % 2 == 0:
                tf[:9] = tf[8]
                tf[:9, 3] = haze
            chans.append(dict(c=c, lo=0, hi=vol.n_levels - 1, W0=wins[0] * 256, W1=wins[1] * 256, tf=tf))
        cams = synth.orbit_path(vol.dims, vol.spacing, 24)
        for cam in cams:
            if cam["proj"] == "persp":
                cam["tx"] = cam["ty"] * W / H
        tf_dev = scene.tf_tensor(chans)
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        img = [torch.empty(W * H * 4, dtype=torch.float32, device="cuda") for _ in range(2)]
        fno = 1
        for f in frames:
            row = {}
            for k, (name, flags) in enumerate((("plain", 0), ("homogeneous", resoct.RENDER_HOMOGENEOUS))):
                ms = []
                for it in range(reps + 1):
                    stats.zero_()
                    fno += 1
                    a.record()
                    scene.render(fno, cams[f], W, H, 0.5, chans, tf_dev=tf_dev, out=img[k], stats=stats,
                                 flags=flags)
                    b.record()
                    torch.cuda.synchronize()
                    if it:  # the first render of each mode is untimed
                        ms.append(a.elapsed_time(b))
                st = stats.cpu().numpy()
                _, nused = scene.cache.read_usage(fno)
                scene.cache.read_requests(1 << 22)
                row[name] = dict(ms=float(np.median(ms)), samples=int(st[0]), brick_reads=int(st[1]),
                                 bricks_read=int(nused), leaf_visits=int(st[3]), wave_iterations=int(st[5]),
                                 homogeneous_samples=int(st[6]))
            row["speedup"] = row["plain"]["ms"] / row["homogeneous"]["ms"]
            row["image_max_abs_diff"] = float((img[0] - img[1]).abs().max().item())
            res[str(f)] = row
            log(f"homogeneous leaves ({wname}), frame {f}: {row}")
        out["workloads"][wname] = res
        del scene
        torch.cuda.empty_cache()
    return out


def serve_bench(rate=400.0, seconds=10.0, n_sat=160, graph=True, max_batch=64):
    """Serving on the 16-channel 2048 x 2048 x 64 cell volume, every brick
    resident in a 24 GiB cache: 64 clients, Poisson arrivals at `rate`
    requests/s, viewports {256^2, 512^2, 1024^2, 1920x1080}, 3-16 channels
    per request, per-client transfer functions and camera paths.  Measures
    the throughput of n_sat such requests batched (all queued at once) and
    one request at a time through the frame kernel, then p50/p99 latency over
    `seconds` of arrivals at `rate` and at 70% of the batched capacity (a
    request still unfinished 5 s after the arrivals stop counts as
    infinitely late).  The same measurements with continuous admission
    (requests admitted one at a time while others render) go under
    "continuous", with the 70%-load trace shared with the batched loop."""
    import torch

    import synth
    from paper_2309_04393_amd.pipeline import GpuScene
    from paper_2309_04393_amd.serving import ServingLoop, latency_summary, make_trace, reset_trace
    vol = synth.config2_volume(n_channels=16)
    t = time.perf_counter()
    stride = 78848
    n_slots = (24 << 30) // stride
    scene = GpuScene(vol, 32, (16, 16, 4), 7, n_slots, max_batch=4096, start_level=2, set_metadata=False)
    lg = leaf_grid(vol.dims, (16, 16, 4), 7)
    mx = vol.leaf_max_all((16, 16, 4), lg)
    for c in range(vol.n_channels):
        mm = np.zeros((mx.shape[1], 2), np.uint16)
        mm[:, 1] = mx[c]
        scene.set_metadata(c, mm)
    ids = scene.all_ids()
    scene.upload(0, ids)
    scene.tree.update_residency()
    torch.cuda.synchronize()
    log(f"serving scene: {len(ids)} bricks resident in {n_slots} slots ({time.perf_counter() - t:.1f} s)")
    loop = ServingLoop(scene, out_budget=4 << 30, max_requests=max_batch, max_tiles=1 << 17, graph=graph)
    from paper_2309_04393_amd import resoct
    # saturated throughput: the same requests batched vs one at a time
    sub = make_trace(scene, rate, n_sat / rate, arrival_seed=3001)
    for r in sub:
        r.arrival = 0.0
    loop.run(sub[:16])  # graph capture, first-touch
    reset_trace(sub)
    loop.stats.zero_()
    wb = loop.run(sub)
    sb = float(loop.stats.cpu().numpy()[0])
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    img = torch.empty(4 * 1920 * 1080, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in sub:
        fd = resoct.frame_desc(r.frame, r.cam, r.W, r.H, loop.step, r.chans, r.tf, scene.vol.n_levels,
                               stats=stats)
        scene.tree.render(fd, img)
    torch.cuda.synchronize()
    ws = time.perf_counter() - t
    ss = float(stats.cpu().numpy()[0])
    out = {"workload": "16ch-2048x2048x64-u16 cells, all 173392 bricks resident, 24 GiB cache",
           "clients": 64, "graph": graph, "max_batch_requests": max_batch,
           "saturated": {"requests": len(sub), "batched_samples_per_s": sb / wb, "batched_req_per_s": len(sub) / wb,
                         "one_at_a_time_samples_per_s": ss / ws, "one_at_a_time_req_per_s": len(sub) / ws,
                         "speedup": (sb / wb) / (ss / ws), "same_samples": sb == ss}}
    cap = len(sub) / wb

    # load shedding: batches of at most 1024 work items (about 3 full-HD
    # requests' worth of 8x8 blocks, ~0.1 s of device time), requests queued
    # longer than 0.1 s dropped
    shed_loop = ServingLoop(scene, out_budget=4 << 30, max_requests=max_batch, max_tiles=1024, graph=graph)
    shed_loop.run(sub[:4])  # graph capture
    reset_trace(sub)

    def at_rate(lam, seed, max_wait=None, lp=None):
        if lp is None:
            lp = loop if max_wait is None else shed_loop
        trace = make_trace(scene, lam, seconds, arrival_seed=seed)
        lp.stats.zero_()
        nb0 = lp.n_batches
        na0 = len(lp.in_flight_at_admission)
        wall = lp.run(trace, deadline=seconds + 5.0, max_wait=max_wait)
        st = lp.stats.cpu().numpy()
        lat = latency_summary(trace)
        sizes = lp.batch_sizes[nb0:]
        done = sum(1 for r in trace if np.isfinite(r.done))
        shed = sum(1 for r in trace if r.shed)
        res = {"rate_req_per_s": lam, "seconds": seconds, "requests": len(trace), "completed": done,
               "latency_ms": {k: v for k, v in lat.items() if k not in ("n", "completed")},
               "wall_s": wall, "served_req_per_s": done / wall, "samples_per_s": float(st[0]) / wall}
        if lp.continuous:
            fl = lp.in_flight_at_admission[na0:]
            res["mean_unfinished_at_admission"] = float(np.mean(fl)) if fl else 0.0
        else:
            res["batches"] = len(sizes)
            res["mean_batch"] = float(np.mean(sizes)) if sizes else 0.0
        if max_wait is not None:
            res["max_queue_wait_s"] = max_wait
            res["max_work_items_in_flight" if lp.continuous else "max_batch_work_items"] = lp.max_tiles
            res["shed"] = shed
        log(f"serving at {lam:.1f} requests/s (max wait {max_wait}, continuous {lp.continuous}): "
            f"{done} of {len(trace)} done, {shed} shed")
        return res

    out["stated_load"] = at_rate(rate, 3000)
    # the same arrivals with load shedding, so the served requests keep a
    # bounded latency
    out["stated_load_shedding"] = at_rate(rate, 3000, max_wait=0.1)
    out["load_70pct_capacity"] = at_rate(0.7 * cap, 3002)

    # continuous admission: the saturated throughput, then the same traces
    cloop = ServingLoop(scene, out_budget=4 << 30, max_requests=max_batch, max_tiles=1 << 17, continuous=True)
    cloop.run(sub[:8])  # first-touch
    reset_trace(sub)
    cloop.stats.zero_()
    wc = cloop.run(sub)
    sc = float(cloop.stats.cpu().numpy()[0])
    reset_trace(sub)
    cshed = ServingLoop(scene, out_budget=4 << 30, max_requests=max_batch, max_tiles=1024, continuous=True)
    out["continuous"] = {
        "saturated": {"requests": len(sub), "samples_per_s": sc / wc, "req_per_s": len(sub) / wc,
                      "vs_batched": (sc / wc) / (sb / wb), "same_samples": sc == sb},
        "stated_load_shedding": at_rate(rate, 3000, max_wait=0.1, lp=cshed),
        "load_70pct_capacity": at_rate(0.7 * cap, 3002, lp=cloop)}
    log(f"serving: {json.dumps(out)}")
    del loop, shed_loop, cloop, cshed, scene
    torch.cuda.empty_cache()
    return out


def incremental_bench(n_frames=16, W=768, H=768, U=512):
    """Incremental metadata (Alg. 1 reportNodeRequest, Sec. 5.3 without
    server metadata) on the 4-channel 2048x2048x64 cell volume, orbit path
    from a cold cache: the request-driven loop (render, plain policy, upload,
    residency update) with every leaf unknown and refined from the inserted
    bricks ("refined"), with every leaf unknown and never refined ("never":
    no empty space is ever skipped), and with the server's metadata
    ("server").  Per frame: kernel time from HIP events, ray samples
    evaluated, missing samples, uploads and the share of leaves with
    metadata; and the largest difference of the last frame's image from the
    server run's (metadata from coarse bricks are estimates, R32)."""
    import torch
    import synth
    from paper_2309_04393_amd.pipeline import GpuScene
    vol = synth.config2_volume()
    cams = synth.orbit_path(vol.dims, vol.spacing, n_frames)
    chans = [dict(ch, hi=vol.n_levels - 1) for ch in channels(vol.n_channels, 2)]
    out = {"workload": "4ch-2048x2048x64-u16 orbit, cold 27318-slot cache", "image": [W, H],
           "upload_budget": U, "frames": n_frames}
    last = {}
    for mode in ("refined", "never", "server"):
        scene = GpuScene(vol, 32, (16, 16, 4), 7, 27318, max_batch=U, start_level=2,
                         set_metadata=(mode == "server"))
        if mode != "server":
            for c in range(vol.n_channels):
                scene.set_unknown(c)
        tf = scene.tf_tensor(chans)
        img = torch.empty(W * H * 4, dtype=torch.float32, device="cuda")
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        rows = []
        for f in range(n_frames):
            stats.zero_()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            scene.render(f + 1, cams[f], W, H, 0.5, chans, tf_dev=tf, out=img, stats=stats)
            b.record()
            torch.cuda.synchronize()
            ids, cnt, nu, tot = scene.cache.read_requests(1 << 22)
            order = np.lexsort((ids, -cnt.astype(np.int64)))
            up = ids[order][:U]
            if len(up):
                flags = scene.upload(f + 1, up)
                if mode == "refined":
                    scene.tree.leaf_metadata_from_bricks(up[flags == 1])
            scene.tree.update_residency()
            torch.cuda.synchronize()
            st = stats.cpu().numpy()
            row = dict(ms=a.elapsed_time(b), samples=int(st[0]), missing=int(tot), uploads=int(len(up)))
            if mode != "server":
                lv = scene.tree.leaf_levels()
                row["known_leaves"] = float((lv < 255).mean())
                row["level0_leaves"] = float((lv == 0).mean())
            rows.append(row)
        out[mode] = rows
        last[mode] = img.cpu().numpy()
        log(f"incremental metadata ({mode}): " + ", ".join(f"{r['ms']:.2f}" for r in rows) + " ms")
        del scene
        torch.cuda.empty_cache()
    for mode in ("refined", "never"):
        out[f"{mode}_last_frame_max_abs_diff_from_server"] = float(np.abs(last[mode] - last["server"]).max())
    return out


def prefetch_bench(train_seeds=tuple(range(1000, 1010)), eval_seeds=tuple(range(1010, 1015)), n_frames=120,
                   U=512, lr=3e-3, train_steps=4, threshold=0.5, gate=0.5):
    """Learned prefetcher against plain request-driven streaming on the
    4-channel 2048 x 2048 x 64 cell volume (2 GiB cache, 1024 x 1024
    perspective views, upload budget U bricks per frame): the network trains
    online along the training paths, then both policies run each held-out
    path from an empty cache."""
    import torch

    import synth
    from paper_2309_04393_amd import resoct
    from paper_2309_04393_amd.pipeline import GpuScene
    from paper_2309_04393_amd.prefetch import BrickStore, run_path, save_state
    vol = synth.config2_volume()
    t = time.perf_counter()
    scene = GpuScene(vol, 32, (16, 16, 4), 7, 27318, max_batch=U, start_level=2, set_metadata=False)
    lg = leaf_grid(vol.dims, (16, 16, 4), 7)
    mx = vol.leaf_max_all((16, 16, 4), lg)
    for c in range(vol.n_channels):
        mm = np.zeros((mx.shape[1], 2), np.uint16)
        mm[:, 1] = mx[c]
        scene.set_metadata(c, mm)
    store = BrickStore(scene)
    empty = save_state(scene)
    log(f"prefetch scene: {len(store.index)} bricks in the device store ({time.perf_counter() - t:.1f} s)")
    chans = [dict(ch, hi=vol.n_levels - 1) for ch in channels(vol.n_channels, 2)]
    W = H = 1024
    step = 0.5 * min(vol.spacing)
    net = resoct.Mlp()
    net.set_weights(synth.mlp_init(7))
    path = lambda s: synth.random_path(vol.dims, vol.spacing, s, n_frames)
    t = time.perf_counter()
    train = []
    for s in train_seeds:
        _, sm = run_path(scene, store, path(s), chans, W, H, U, step, "learned", net, empty, lr=lr,
                         train_steps=train_steps, threshold=threshold, gate=gate)
        sm.pop("missing_curve")
        train.append(sm)
        log(f"train path {s}: {sm}")
    t_train = time.perf_counter() - t
    ev = []
    for s in eval_seeds:
        cams = path(s)
        _, sp = run_path(scene, store, cams, chans, W, H, U, step, "plain", None, empty)
        _, sl = run_path(scene, store, cams, chans, W, H, U, step, "learned", net, empty, lr=lr,
                         train_steps=train_steps, threshold=threshold, gate=gate)
        ev.append({"seed": s, "plain": sp, "learned": sl})
        brief = lambda d: {k: v for k, v in d.items() if k != "missing_curve"}
        log(f"eval path {s}: plain {brief(sp)}")
        log(f"eval path {s}: learned {brief(sl)}")

    def agg(key, pol):
        v = [e[pol][key] for e in ev]
        return None if any(x is None for x in v) else float(np.mean(v))

    out = {"workload": "4ch-2048x2048x64-u16 cells, 2 GiB cache, 1024x1024 perspective, random paths",
           "frames_per_path": n_frames, "upload_budget": U, "train_paths": list(train_seeds),
           "policy": {"lr": lr, "train_steps": train_steps, "threshold": threshold, "precision_gate": gate},
           "eval_paths": list(eval_seeds), "train_s": t_train,
           "summary": {pol: {k: agg(k, pol) for k in ("frames_to_converge", "first_below_1pct", "mean_missing",
                                                       "bytes_streamed")} for pol in ("plain", "learned")},
           "per_path": [{"seed": e["seed"], **{pol: {k: e[pol][k] for k in
                         ("frames_to_converge", "first_below_1pct", "mean_missing", "bytes_streamed", "extra",
                          "precision")} for pol in ("plain", "learned")}} for e in ev],
           "paths": ev}
    del store, scene
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=384,
                    help="edge of the centre window the oracle renders for the CPU baseline and the parity check")
    ap.add_argument("--serve", type=float, default=10.0, metavar="SECONDS",
                    help="seconds of the serving measurement after the frame measurement (0: skip)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement")
    ap.add_argument("--rate", type=float, default=400.0, help="serving arrival rate, requests/s")
    ap.add_argument("--serve-max-batch", type=int, default=64, help="requests per serving batch at most")
    ap.add_argument("--no-prefetch", action="store_true", help="skip the learned-prefetcher evaluation")
    ap.add_argument("--no-streaming", action="store_true", help="skip the timing of the streaming steps")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the LOD-adaptive step measurement on zoomed-out frames")
    ap.add_argument("--adaptive-frames", default="0,20",
                    help="fly-through frames of the adaptive-step measurement (each is made resident first; "
                         "the coarse bricks of zoomed-out frames take the host generator a while)")
    ap.add_argument("--no-homogeneous", action="store_true",
                    help="skip the homogeneous-leaves measurement (its own 4-channel scene)")
    ap.add_argument("--no-incremental", action="store_true",
                    help="skip the loop that starts from unknown leaf metadata")
    ap.add_argument("--prefetch-only", action="store_true",
                    help="only the learned-prefetcher evaluation (10 training, 5 held-out paths)")
    ap.add_argument("--pf-lr", type=float, default=3e-3)
    ap.add_argument("--pf-steps", type=int, default=4, help="Adam steps per frame")
    ap.add_argument("--pf-threshold", type=float, default=0.5, help="candidate probability threshold")
    ap.add_argument("--pf-gate", type=float, default=0.5, help="precision below which the plain policy is used")
    ap.add_argument("--profile-summary", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="print the summary of rocprofv3 output directories of the headline loop (no GPU work)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the measurement, copy a 1 GiB buffer three times (a plain copy kernel of "
                         "known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.profile_summary:
        print(profile_summary(*args.profile_summary, last=args.steps, workload=config(args.config)["name"]))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_2309_04393_amd.pipeline import GpuScene
    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.prefetch_only:
        print(json.dumps({"prefetch": prefetch_bench(lr=args.pf_lr, train_steps=args.pf_steps,
                                                     threshold=args.pf_threshold, gate=args.pf_gate)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serve_bench(args.rate, args.serve, max_batch=args.serve_max_batch)}), flush=True)
        return
    cfg = config(args.config)
    vol = cfg["vol"]
    t_setup = time.perf_counter()
    scene = GpuScene(vol, cfg["B"], cfg["leaf"], cfg["depth"], cfg["n_slots"], max_batch=cfg["U"],
                     start_level=cfg["start_level"], set_metadata=False)
    mm = leaf_mm_all(cfg)
    for c in range(vol.n_channels):
        scene.set_metadata(c, mm[c])
    log(f"scene ready: {scene.cache.n_bricks} bricks, {scene.tree.n_nodes} nodes, "
        f"{cfg['n_slots']} slots x {scene.cache.slot_stride} B ({time.perf_counter() - t_setup:.1f} s)")
    if cfg["path"] == "fly":
        cams = synth.flythrough_path(vol.dims, vol.spacing, cfg["n_frames"], tissue_target(vol, cfg["seed"]))
    else:
        cams = synth.orbit_path(vol.dims, vol.spacing, cfg["n_frames"])
    chans = [dict(ch, hi=vol.n_levels - 1) for ch in channels(vol.n_channels, cfg["seed"])]
    step = 0.5 * min(vol.spacing)
    K, Wm = args.steps, args.warmup
    f0 = cfg["f0"]
    fl = Frames(scene, cams, chans, cfg["W"], cfg["H"], cfg["U"], step)
    # bulk warm-up on the first warm-up frame: the visible working set resident
    fw = f0 - Wm
    for it in range(4):
        fl.render(fw)
        ids, cnt, nu, tot = scene.cache.read_requests(1 << 22)
        log(f"bulk warm {it}: {nu} bricks requested, {tot} missing samples")
        if nu == 0:
            break
        t = time.perf_counter()
        scene.upload(fw, ids)
        scene.tree.update_residency()
        torch.cuda.synchronize()
        log(f"  uploaded {len(ids)} bricks in {time.perf_counter() - t:.1f} s")
    for f in range(fw, f0):
        ids, _, tot = fl.step_frame(f)
        log(f"warm-up frame {f}: {tot} missing samples, {len(ids)} uploads")
    torch.cuda.synchronize()
    snap = snapshot(scene)
    # pass A: collect the uploads of the timed frames (untimed)
    plans, store, usage, stats_a, tree_reads, req_px, missed = [], [], [], [], [], [], []
    nodes_t = torch.zeros(scene.tree.n_nodes, dtype=torch.uint8, device="cuda")
    for f in range(f0, f0 + K):
        # diagnostic render of the frame (untimed, its own kernel): the nodes
        # whose metadata the frame reads and the bricks each pixel requires;
        # its miss counts are discarded and its stamps are the frame's own
        nodes_t.zero_()
        d = scene.render(f, fl.cams[f], fl.W, fl.H, fl.step, fl.chans, tf_dev=fl.tf, bricks=True, nodes=nodes_t)
        torch.cuda.synchronize()
        scene.cache.read_requests(1 << 22)
        marked = nodes_t.cpu().numpy()
        n_leaf = int(marked[scene.tree.n_nodes - scene.tree.n_leaves:].sum())
        tree_reads.append((int(marked.sum()) - n_leaf, n_leaf))
        req_px.append(d["bricks"].cpu().numpy().ravel())
        del d
        fl.stats.zero_()
        ids, staged, tot = fl.step_frame(f)
        missed.append(fl.last_nu)
        plans.append(ids.copy())
        store.append(staged)
        _, nused = scene.cache.read_usage(f)
        usage.append(nused)
        stats_a.append(fl.stats.cpu().numpy().copy())
        log(f"pass A frame {f}: {tot} missing samples, {len(ids)} uploads, {nused} slots read, "
            f"stats {stats_a[-1].tolist()}")
    restore(scene, snap)
    del snap
    # pass B: timed
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    fl.stats.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, f in enumerate(range(f0, f0 + K)):
        ev[i][0].record()
        fl.render(f)
        ev[i][1].record()
        ids, tot, nu = fl.plan()
        if not np.array_equal(ids, plans[i]):
            raise SystemExit(f"frame {f}: the timed pass planned other uploads than the collection pass")
        if len(ids):
            scene.cache.stream_bricks(f, ids, store[i])
        scene.tree.update_residency()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = fl.stats.cpu().numpy()
    render_ms = [a.elapsed_time(b) for a, b in ev]
    ms_step = (t1 - t0) * 1000.0 / K
    samples = int(st[0])
    ch_samples = int(st[1])
    # algorithmic bytes of a launch: every brick read once (its voxels with the
    # halo, its page-table entry, its stamp), the metadata (4 B per channel)
    # of the inner nodes and the metadata and masks (6 B per channel) of the
    # leaves the descents read, the image, and a read and write of the miss
    # counter of each missed brick
    slot_bytes = (cfg["B"] + 2) ** 3 * 2
    m = vol.n_channels
    alg_parts = [dict(bricks=u * (slot_bytes + 8), tree=ni * m * 4 + nl * m * 6, image=cfg["W"] * cfg["H"] * 16,
                      counters=8 * nm) for u, (ni, nl), nm in zip(usage, tree_reads, missed)]
    alg_bytes = [sum(p.values()) for p in alg_parts]
    mean_render_s = np.mean(render_ms) / 1000.0
    achieved = np.mean(alg_bytes) / mean_render_s / 1e9
    out = {
        "metric": METRIC,
        "value": samples / (t1 - t0),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "frames": f"{f0}..{f0 + K - 1} of {cfg['n_frames']}",
                   "image": [cfg["W"], cfg["H"]], "channels": vol.n_channels, "cache_slots": cfg["n_slots"],
                   "upload_budget": cfg["U"], "parallelism": "1 GPU"},
        "render_ms": float(np.mean(render_ms)),
        "channel_samples_per_s": ch_samples / (t1 - t0),
        "render_samples_per_s": samples / (np.sum(render_ms) / 1000.0),
        "uploads_per_frame": float(np.mean([len(p) for p in plans])),
        # bricks the frames read (every sample at its desired level, nothing missing in steady
        # state): the GPU memory the method needs per frame under these viewing conditions
        "bricks_read_per_frame": float(np.mean(usage)),
        "memory_read_per_frame_GB": float(np.mean(usage)) * scene.cache.slot_stride / 1e9,
        "lane_busy": float(st[0]) / max(float(st[5]), 1.0),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(cfg["name"]),
                     "kernel": "k_render", "alg_bytes_per_launch": float(np.mean(alg_bytes)),
                     "alg_bytes_parts": {k: float(np.mean([p[k] for p in alg_parts])) for k in alg_parts[0]}},
    }
    # bricks each pixel requires (Sec. 8, Fig. 8), over the timed frames
    rp = np.concatenate(req_px)
    out["required_bricks_per_pixel"] = {"mean": float(rp.mean()), "p50": float(np.percentile(rp, 50)),
                                        "p99": float(np.percentile(rp, 99)), "max": int(rp.max()),
                                        "tree_nodes_read_per_frame": float(np.mean([a + b for a, b in tree_reads])),
                                        "leaves_read_per_frame": float(np.mean([b for _, b in tree_reads]))}
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30
    log(f"timed frames: {out['render_ms']:.2f} ms per frame")
    if not args.no_cpu_baseline:
        log("oracle window (CPU baseline and parity)")
        # the oracle's window of the last timed frame, which read every sample
        # from its desired level (no missing samples), against the GPU image
        fl_last = f0 + K - 1
        img = fl.out[: cfg["W"] * cfg["H"] * 4].view(cfg["H"], cfg["W"], 4).cpu().numpy().astype(np.float64)
        try:
            cb, r, (x0, y0) = cpu_baseline(cfg, cams, chans, fl_last, step, args.tile)
            out["cpu_baseline"] = cb
            win = img[y0:y0 + args.tile, x0:x0 + args.tile]
            ok = r["amb_pix"] == 0
            # a pixel with one close termination call has two valid values:
            # compared with the nearer one
            d = np.abs(win - r["rgba"])
            da = np.abs(win - r["alt_rgba"])
            use = (r["alt_pix"] != 0) & (da.max(axis=-1) < d.max(axis=-1))
            d = np.where(use[..., None], da, d)[ok]
            out["parity"] = {"window": [x0, y0, args.tile, args.tile], "frame": fl_last,
                             "missing_samples_in_frame": int(stats_a[-1][2]),
                             "max_abs": d.max(axis=0).tolist(), "mean_abs": d.mean(axis=0).tolist(),
                             "ambiguous_frac": float(1.0 - ok.mean()),
                             "close_termination_frac": float((r["alt_pix"] != 0).mean())}
        except Exception as e:  # reported, not fatal
            out["cpu_baseline"] = {"error": repr(e)}
    # after the parity window, which reads the last timed frame's image
    if not args.no_streaming:
        log("streaming steps")
        out["streaming"] = streaming_bench(scene, fl, cams, f_req=max(f0 - 60, 0), f_up=f0 + K, U=cfg["U"],
                                           mm0=mm[0])
    if not args.no_adaptive:
        log("LOD-adaptive step on zoomed-out frames")
        out["adaptive_step"] = adaptive_bench(scene, fl, tuple(int(x) for x in args.adaptive_frames.split(",")))
    if args.serve > 0 or not args.no_prefetch or not args.no_homogeneous or not args.no_incremental:
        del fl, store, scene
        torch.cuda.empty_cache()
    if not args.no_homogeneous:
        log("homogeneous leaves")
        out["homogeneous_leaves"] = homogeneous_bench()
    if not args.no_incremental:
        log("incremental metadata")
        out["incremental_metadata"] = incremental_bench()
    if args.serve > 0:
        out["serving"] = serve_bench(args.rate, args.serve, max_batch=args.serve_max_batch)
    if not args.no_prefetch:
        pf = prefetch_bench(lr=args.pf_lr, train_steps=args.pf_steps, threshold=args.pf_threshold, gate=args.pf_gate)
        out["prefetch"] = {k: v for k, v in pf.items() if k != "paths"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
