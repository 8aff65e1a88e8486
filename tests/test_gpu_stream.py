"""GPU parity of the streaming side: multi-frame request-driven loop, LRU
batches, page tables, residency masks, metadata reduction, capped readback,
host-forced corruption + rebuild, checkpoint / restore determinism."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import compare_images, compare_requests, compare_usage, gpu_rgba, leaf_grid, oracle_alt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from tests.test_gpu_render import Pair, _report  # noqa: E402
from paper_2309_04393_amd import resoct  # noqa: E402


def _cells(dims=(512, 512, 64), n_ch=4, n_levels=6, seed=2):
    src = synth.CellVolume(dims, n_ch, spacing=(1, 1, 4), n_levels=n_levels, seed=seed)
    src.levels = [[src.level_array(c, l) for l in range(n_levels)] for c in range(n_ch)]
    return src


def _chans(n, lo=0, hi=5):
    return [dict(c=c, lo=lo, hi=hi, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / n, 0.1)) for c in range(n)]


def _plain(ids, cnt, U):
    order = np.lexsort((ids, -cnt.astype(np.int64)))
    return ids[order][:U]


@pytest.fixture(scope="module")
def cells():
    return _cells()


def test_streaming_loop_matches_oracle(cells):
    """Six frames of an orbit from a cold, too-small cache: every frame's
    image, request multiset and usage set, the plain policy's upload list,
    the LRU batch (flags, page table) and the residency masks agree."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=300, max_batch=128)
    cams = synth.orbit_path(cells.dims, cells.spacing, 8, az_step_deg=9.0)
    chans = _chans(4)
    for f in range(1, 7):
        res = p.frame(f, cams[f], 96, 96, 0.5, chans, lod_bias=0.7)
        p.check_frame(res, f"loop-{f}")
        g_up = _plain(res["ids"], res["cnt"], 128)
        o_up = p.sim.plain_policy(res["o"]["counts"], 128)
        assert np.array_equal(g_up, p.ids[o_up]), "plain policy differs"
        p.upload(f, g_up)
        p.check_page_table()
        p.check_masks()


def test_metadata_reduction_matches_oracle(cells):
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=8)
    torch.cuda.synchronize()
    assert np.array_equal(p.gpu.tree.meta(), oracle.meta_all(p.V, p.leaf_mm))


def test_capped_readback(cells):
    """Sec. 4 global limit: the first `cap` pairs in ascending ID, with the
    full distinct count and total, then the counters are clear."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=8)
    cam = synth.orbit_path(cells.dims, cells.spacing, 2)[1]
    chans = _chans(4)
    p.gpu.render(1, cam, 64, 64, 0.5, chans)
    torch.cuda.synchronize()
    ids, cnt, nu, tot = p.gpu.cache.read_requests(5)
    fr, keep = oracle.make_frame(cam, 64, 64, 0.5, chans, term_margin=1e-6)
    o = oracle.render(p.V, cells.levels, p.sim.res_slot, p.leaf_mm, fr, p.S)
    nz = np.nonzero(o["counts"])[0]
    o_ids = np.sort(p.ids[nz])
    assert o["amb_counts"].sum() == 0
    assert nu == len(nz) and tot == int(o["counts"].sum())
    assert np.array_equal(ids, o_ids[:5])
    ids2, cnt2, nu2, tot2 = p.gpu.cache.read_requests(5)
    assert nu2 == 0 and tot2 == 0 and len(ids2) == 0


def test_rebuild_after_corrupted_masks(cells):
    """Host-forced fault: garbage written into the node masks is repaired by
    the from-scratch rebuild, which equals the oracle's masks."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=120, max_batch=128)
    rng = np.random.default_rng(5)
    ids = p.gpu.all_ids()
    rng.shuffle(ids)
    p.upload(0, ids[:100])
    p.check_masks()
    m = p.gpu.tree.t["node_mask"]
    m.copy_(torch.randint(0, 255, m.shape, dtype=torch.uint8, device=m.device))
    p.gpu.tree.rebuild_residency()
    torch.cuda.synchronize()
    assert np.array_equal(p.gpu.tree.masks(), oracle.masks(p.V, p.sim.res_slot))


def test_invalid_ids_leave_state_unchanged(cells):
    from paper_2309_04393_amd import resoct
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=16, max_batch=32)
    ids = p.gpu.all_ids()[:4]
    p.upload(0, ids)
    before = p.gpu.cache.page_table_host().copy()
    bad = np.array([ids[0], 0x00FF0000], np.uint32)  # bz = 255 does not exist
    with pytest.raises(resoct.ResoctError) as e:
        p.gpu.cache.stream_bricks(1, bad, p.gpu.stage(ids[:2]))
    assert e.value.code == -1
    assert np.array_equal(p.gpu.cache.page_table_host(), before)
    many = p.gpu.all_ids()[:40]
    with pytest.raises(resoct.ResoctError) as e:
        p.gpu.cache.stream_bricks(1, many, p.gpu.cache.staging(len(many)))  # more than max_batch
    assert e.value.code == -1 and "max_batch" in str(e.value)
    assert np.array_equal(p.gpu.cache.page_table_host(), before)


def test_checkpoint_restore_replays_identically(cells):
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=200, max_batch=128)
    cams = synth.orbit_path(cells.dims, cells.spacing, 6, az_step_deg=12.0)
    chans = _chans(4)
    g = p.gpu

    def run(frames):
        outs = []
        for f in frames:
            r = g.render(f, cams[f], 64, 64, 0.5, chans)
            torch.cuda.synchronize()
            ids, cnt, nu, tot = g.cache.read_requests(1 << 16)
            up = _plain(ids, cnt, 128)
            fl = g.upload(f, up)
            g.tree.update_residency()
            outs.append((r["rgba"].cpu().numpy().copy(), ids.copy(), cnt.copy(), fl.copy()))
        return outs

    run([1, 2])
    dev = {("c", k): v.clone() for k, v in g.cache.t.items()}
    dev.update({("t", k): v.clone() for k, v in g.tree.t.items()})
    host = g.cache.save_state()
    a = run([3, 4, 5])
    for (kind, k), v in dev.items():
        (g.cache.t if kind == "c" else g.tree.t)[k].copy_(v)
    torch.cuda.synchronize()
    g.cache.load_state(host)
    b = run([3, 4, 5])
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_snapshot_restore_replays_identically(cells):
    """ro_snapshot / ro_restore: a snapshot with slots taken after frame 2,
    three more frames of the streaming loop (renders, readbacks, uploads
    that evict and overwrite slots, residency updates), a restore, and the
    same three frames again: images, requests and upload flags identical,
    and the final page table and masks too.  A snapshot without slots
    restores over frames that upload nothing; blobs of another shape or size
    are rejected without changing anything."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=200, max_batch=128)
    cams = synth.orbit_path(cells.dims, cells.spacing, 6, az_step_deg=12.0)
    chans = _chans(4)
    g = p.gpu

    def run(frames, upload=True):
        outs = []
        for f in frames:
            r = g.render(f, cams[f], 64, 64, 0.5, chans)
            torch.cuda.synchronize()
            ids, cnt, nu, tot = g.cache.read_requests(1 << 16)
            fl = np.zeros(0, np.uint8)
            if upload:
                fl = g.upload(f, _plain(ids, cnt, 128))
                g.tree.update_residency()
            outs.append((r["rgba"].cpu().numpy().copy(), ids.copy(), cnt.copy(), fl.copy()))
        return outs

    run([1, 2])
    blob = g.tree.snapshot(slots=True)
    a = run([3, 4, 5])
    pt_a, masks_a = g.cache.page_table_host(), g.tree.masks()
    g.tree.restore(blob)
    b = run([3, 4, 5])
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    assert np.array_equal(pt_a, g.cache.page_table_host()) and np.array_equal(masks_a, g.tree.masks())
    # without slots: valid while the slots are untouched (no uploads)
    small = g.tree.snapshot(slots=False)
    assert small.size < blob.size
    c = run([4, 5], upload=False)
    g.tree.restore(small)
    d = run([4, 5], upload=False)
    for x, y in zip(c, d):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    # a truncated blob and one from another cache are rejected; state unchanged
    with pytest.raises(resoct.ResoctError):
        g.tree.restore(small[:-4])
    other = Pair(cells, 32, (16, 16, 4), 5, n_slots=100, max_batch=128)
    with pytest.raises(resoct.ResoctError):
        g.tree.restore(other.gpu.tree.snapshot())
    e = run([4], upload=False)
    assert np.array_equal(e[0][0], d[0][0])


def test_run_is_deterministic(cells):
    """Determinism is the race test: the same frame twice gives identical
    counters, stamps, masks and page tables."""
    outs = []
    for _ in range(2):
        p = Pair(cells, 32, (16, 16, 4), 5, n_slots=150, max_batch=128)
        ids = p.gpu.all_ids()
        np.random.default_rng(1).shuffle(ids)
        p.upload(0, ids[:140])
        p.gpu.tree.update_residency()
        cam = synth.orbit_path(cells.dims, cells.spacing, 3)[2]
        r = p.gpu.render(1, cam, 80, 80, 0.5, _chans(4))
        torch.cuda.synchronize()
        rq = p.gpu.cache.read_requests(1 << 16)
        outs.append((r["rgba"].cpu().numpy(), rq[0], rq[1], p.gpu.cache.t["stamps"].cpu().numpy(),
                     p.gpu.tree.masks(), p.gpu.cache.page_table_host()))
    for u, v in zip(*outs):
        assert np.array_equal(u, v)


def test_render_between_upload_and_residency_update(cells):
    """Uploads that evict bricks change the page tables at once while the
    octree masks wait for the residency update: a frame rendered in between
    reads no evicted slot (the stale levels contribute nothing, stamps only
    on live slots), and after the update the frame matches the oracle."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=120, max_batch=128)
    ids = p.gpu.all_ids()
    rng = np.random.default_rng(12)
    rng.shuffle(ids)
    p.upload(0, ids[:110])
    p.check_masks()
    cams = synth.orbit_path(cells.dims, cells.spacing, 4, az_step_deg=15.0)
    chans = _chans(4)
    p.upload(1, ids[110:220])  # evicts most of the first batch; masks not updated
    r = p.gpu.render(2, cams[1], 64, 64, 0.5, chans)
    torch.cuda.synchronize()
    img = gpu_rgba(r["rgba"], 64, 64)
    assert np.isfinite(img).all() and img.min() >= 0.0 and img[..., 3].max() <= 1.0
    used, n = p.gpu.cache.read_usage(2)
    pt = p.gpu.cache.page_table_host()
    live = set(pt[pt != 0xFFFFFFFF].tolist())
    assert set(used.tolist()) <= live
    p.gpu.cache.read_requests(1 << 20)  # clear the in-between frame's counters
    p.check_masks()  # the residency update
    res = p.frame(3, cams[1], 64, 64, 0.5, chans)
    p.check_frame(res, "after-update")


def test_leaf_metadata_from_bricks(cells):
    """Sec. 5.3, metadata computed on the client from brick voxels: with
    every leaf first unknown ([0, 65535]), metadata derived from resident
    bricks of level 0 (part of two channels) and level 2 (every channel)
    equal the oracle's node metadata bit for bit; a frame rendered with them
    matches the oracle; bad calls change nothing."""
    from paper_2309_04393_amd import resoct
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=700, max_batch=256)
    n_leaves = p.leaf_mm.shape[1]
    unknown = np.zeros((cells.n_channels, n_leaves, 2), np.uint16)
    unknown[..., 1] = 65535
    for c in range(cells.n_channels):
        p.gpu.set_unknown(c)
    _, _, nb = oracle.level_info(p.V)
    l0 = [oracle.brick_id(p.V.n_levels, c, 0, x, y, 0) for c in (0, 2) for y in range(nb[0][1])
          for x in range(min(8, nb[0][0]))]
    l2 = [int(i) for i in p.gpu.all_ids(levels=[2])]
    ids = np.array(l2[::-1] + l0, np.uint32)
    assert len(ids) <= 700
    p.upload(0, ids)
    p.check_masks()
    before = p.gpu.tree.meta()
    missing = [i for i in p.gpu.all_ids(levels=[1])][:1]
    with pytest.raises(resoct.ResoctError) as e:
        p.gpu.tree.leaf_metadata_from_bricks(np.array(list(ids[:3]) + missing, np.uint32))
    assert e.value.code == -5
    with pytest.raises(resoct.ResoctError) as e:
        p.gpu.tree.leaf_metadata_from_bricks(np.array([ids[0], 0x00FF0000], np.uint32))
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert np.array_equal(p.gpu.tree.meta(), before)
    p.gpu.tree.leaf_metadata_from_bricks(ids)
    torch.cuda.synchronize()
    ref = oracle.leaf_meta_from_bricks(p.V, cells.levels, unknown, ids)
    got = p.gpu.tree.meta()
    want = oracle.meta_all(p.V, ref)
    assert np.array_equal(got, want), f"metadata differ at {np.argwhere(got != want)[:5]}"
    p.leaf_mm = ref
    cam = synth.orbit_path(cells.dims, cells.spacing, 3)[1]
    res = p.frame(1, cam, 80, 80, 0.5, _chans(4))
    p.check_frame(res, "meta-from-bricks")


def test_channel_exchange():
    """Sec. 5.2 run-time channel exchange with a cache that references 3 of
    a source's 5 channels: cache channel 1 changes from source channel 1 to
    4.  Its bricks leave (page tables equal the oracle's, freed slots are
    taken first by the next uploads), the masks follow, and frames before and
    after the new bricks arrive match the oracle on the new channel's data."""
    from paper_2309_04393_amd.pipeline import GpuScene
    src = _cells(dims=(256, 256, 32), n_ch=5, n_levels=5, seed=7)
    B, leaf, depth, S = 32, (16, 16, 4), 4, 260
    g = GpuScene(src, B, leaf, depth, S, max_batch=256, cache_channels=3)
    V = oracle.make_volume(src.dims, src.spacing, 3, src.bits, B, src.n_levels, leaf, depth)
    sim = oracle.CacheSim(V, S)
    dense = oracle.dense_ids(V)
    lg = leaf_grid(src.dims, leaf, depth)
    chans = _chans(3, hi=4)
    cam = synth.orbit_path(src.dims, src.spacing, 3)[1]

    def upload(f, ids):
        fg = g.upload(f, ids)
        fo, _, _ = sim.stream(f, sim.dense_of(ids))
        assert np.array_equal(fg, fo), "upload flags differ"
        pt = g.cache.page_table_host()
        assert {int(i): int(s) for i, s in zip(dense, pt) if s != 0xFFFFFFFF} == sim.page_table()

    def frame(f, name):
        r = g.render(f, cam, 72, 72, 0.5, chans)
        torch.cuda.synchronize()
        ids, cnt, nu, tot = g.cache.read_requests(1 << 20)
        used, _ = g.cache.read_usage(f)
        fr, _ = oracle.make_frame(cam, 72, 72, 0.5, chans, term_margin=1e-6)
        levels = [src.levels[s] for s in g.channel_map]
        mm = np.stack([src.leaf_minmax(s, leaf, lg) for s in g.channel_map])
        o = oracle.render(V, levels, sim.res_slot, mm, fr, S)
        sim.touch(f, o["used"])
        st = compare_images(gpu_rgba(r["rgba"], 72, 72), o["rgba"], o["amb_pix"], alt=oracle_alt(o))
        compare_requests(ids, cnt, o["counts"], o["amb_counts"], dense)
        compare_usage(used, o["used"], o["amb_used"])
        _report(name, requests=nu, **st)
        return ids, cnt

    ids = g.all_ids(levels=[1, 2, 3, 4])
    upload(0, ids[:S - 20])
    g.tree.update_residency()
    frame(1, "exchange-before")
    old = {int(i): int(s) for i, s in zip(dense, g.cache.page_table_host()) if s != 0xFFFFFFFF}
    g.exchange_channel(1, 4)
    sim.evict_channel(1)
    torch.cuda.synchronize()
    pt = g.cache.page_table_host()
    now = {int(i): int(s) for i, s in zip(dense, pt) if s != 0xFFFFFFFF}
    assert now == sim.page_table()
    assert len(now) < len(old) and all(old[i] == s for i, s in now.items())
    assert np.array_equal(g.tree.masks(), oracle.masks(V, sim.res_slot))
    ids, cnt = frame(2, "exchange-no-bricks")  # channel 1 contributes nothing yet and requests its bricks
    assert np.any((ids >> 24) // src.n_levels == 1)
    # the library's channel map names the data behind the requested IDs
    assert g.channel_map == [0, 4, 2]
    sb = g.cache.source_bricks(ids)
    for i, r in zip(ids, sb):
        c, l, b = g.vol.decode(int(i))
        assert tuple(int(x) for x in r) == ([0, 4, 2][c], l, *b)
    with pytest.raises(resoct.ResoctError):
        g.cache.set_channel_map(3, 0)
    with pytest.raises(resoct.ResoctError):
        g.cache.source_bricks(np.array([0xFFFFFFFF], np.uint32))
    order = np.lexsort((ids, -cnt.astype(np.int64)))
    upload(3, ids[order][:200])
    g.tree.update_residency()
    assert np.array_equal(g.tree.masks(), oracle.masks(V, sim.res_slot))
    frame(4, "exchange-after")
    # the map is part of a snapshot
    blob = g.tree.snapshot(slots=False)
    g.cache.set_channel_map(1, 1)
    assert g.channel_map == [0, 1, 2]
    g.tree.restore(blob)
    assert g.channel_map == [0, 4, 2]


def test_leaf_metadata_from_u8_bricks():
    """The u8 path of the metadata-from-bricks kernel: from every level-0
    brick of the 64^3 blob volume the derived metadata equal the oracle's and
    the data server's exact leaf metadata (L0 values within one voxel of the
    leaf); then level-1 bricks alone give the oracle's coarse estimate; level
    0 then level 1 again: the level-1 call leaves the exact metadata (finer
    data are never replaced by coarser)."""
    src = synth.config1_volume()
    p = Pair(src, 16, (8, 8, 8), 3, n_slots=73)
    n_leaves = p.leaf_mm.shape[1]
    unknown = np.zeros((1, n_leaves, 2), np.uint16)
    unknown[..., 1] = 255
    p.gpu.set_unknown(0)
    ids = p.gpu.all_ids()
    p.upload(0, ids)
    l0 = [int(i) for i in p.gpu.all_ids(levels=[0])]
    p.gpu.tree.leaf_metadata_from_bricks(np.array(l0, np.uint32))
    torch.cuda.synchronize()
    ref = oracle.leaf_meta_from_bricks(p.V, src.levels, unknown, l0)
    assert np.array_equal(ref, p.leaf_mm)  # the server's exact metadata
    assert np.array_equal(p.gpu.tree.meta(), oracle.meta_all(p.V, ref))
    p.gpu.set_unknown(0)
    l1 = [int(i) for i in p.gpu.all_ids(levels=[1])]
    p.gpu.tree.leaf_metadata_from_bricks(np.array(l1, np.uint32))
    torch.cuda.synchronize()
    ref1 = oracle.leaf_meta_from_bricks(p.V, src.levels, unknown, l1)
    assert np.array_equal(p.gpu.tree.meta(), oracle.meta_all(p.V, ref1))
    assert (p.gpu.tree.leaf_levels() == 1).all()
    for ids_ in (l0, l1):
        p.gpu.tree.leaf_metadata_from_bricks(np.array(ids_, np.uint32))
    torch.cuda.synchronize()
    assert np.array_equal(p.gpu.tree.meta(), oracle.meta_all(p.V, ref))
    assert (p.gpu.tree.leaf_levels() == 0).all()


def test_incremental_metadata_loop(cells):
    """Alg. 1 reportNodeRequest / Sec. 5.3 without server metadata: every
    leaf starts unknown; each frame renders, the plain policy uploads the
    requested bricks, and the inserted bricks give their leaves metadata
    (finer data refine, coarser never replace).  Every frame's image,
    requests and usage, the node metadata, the leaves' metadata levels and
    the masks match an oracle running the same loop; the same view rendered
    again at the end evaluates fewer samples (skipping has switched on where
    the data showed empty space)."""
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=600, max_batch=256)
    g = p.gpu
    n_leaves = p.leaf_mm.shape[1]
    for c in range(cells.n_channels):
        g.set_unknown(c)
    mm = np.zeros((cells.n_channels, n_leaves, 2), np.uint16)
    mm[..., 1] = 65535
    lvl = np.full((cells.n_channels, n_leaves), 255, np.uint8)
    p.leaf_mm = mm
    assert np.array_equal(g.tree.meta(), oracle.meta_all(p.V, mm))
    cams = synth.orbit_path(cells.dims, cells.spacing, 8, az_step_deg=10.0)
    chans = _chans(4)
    st0 = torch.zeros(8, dtype=torch.int64, device="cuda")
    first = None
    for f in range(1, 7):
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        res = p.frame(f, cams[f], 80, 80, 0.5, chans, lod_bias=0.8, stats=st)
        p.check_frame(res, f"incremental-{f}")
        if f == 1:
            first = int(st[0].item())
        up = _plain(res["ids"], res["cnt"], 256)
        flags = p.upload(f, up)
        got = up[flags == 1]
        g.tree.leaf_metadata_from_bricks(got)
        p.leaf_mm, lvl = oracle.leaf_meta_from_bricks(p.V, cells.levels, p.leaf_mm, got, lvl)
        torch.cuda.synchronize()
        want = oracle.meta_all(p.V, p.leaf_mm)
        have = g.tree.meta()
        assert np.array_equal(have, want), f"frame {f}: metadata differ at {np.argwhere(have != want)[:5]}"
        assert np.array_equal(g.tree.leaf_levels().T, lvl), f"frame {f}: metadata levels differ"
        p.check_masks()
    known = (lvl < 255).mean()
    res = p.frame(7, cams[1], 80, 80, 0.5, chans, lod_bias=0.8, stats=st0)
    p.check_frame(res, "incremental-again")
    _report("incremental", known_leaf_fraction=float(known), samples_first=first, samples_again=int(st0[0].item()))
    assert known > 0.1 and int(st0[0].item()) < first
