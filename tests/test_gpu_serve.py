"""Batched serving: a request's image is the same alone, in a mixed batch,
through graph replays and in the real-time serving loop, and equals the
frame kernel's image (which the render tests pin to the oracle)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import compare_images, gpu_rgba, oracle_alt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_04393_amd import resoct  # noqa: E402
from paper_2309_04393_amd.pipeline import GpuScene  # noqa: E402
from paper_2309_04393_amd.serving import Arena, ServingLoop, latency_summary, make_trace  # noqa: E402
from tests.test_gpu_render import _report  # noqa: E402

N_CH = 6


@pytest.fixture(scope="module")
def scene():
    src = synth.CellVolume((512, 512, 64), N_CH, spacing=(1, 1, 4), n_levels=6, seed=4)
    src.levels = [[src.level_array(c, l) for l in range(6)] for c in range(N_CH)]
    n_bricks = resoct.Volume(src.dims, src.spacing, N_CH, 2, 32, 6).brick_count()
    s = GpuScene(src, 32, (16, 16, 4), 5, n_slots=n_bricks, max_batch=2048)
    s.upload(0, s.all_ids())
    s.tree.update_residency()
    torch.cuda.synchronize()
    return s


def _chans(sub, seed):
    rng = np.random.default_rng(seed)
    out = []
    for c in sub:
        j = rng.uniform(0.8, 1.2, 2)
        W0, W1 = synth.window_fx(300 * j[0], 8000 * j[1])
        out.append(dict(c=int(c), lo=0, hi=5, W0=W0, W1=W1,
                        tf=synth.tf_hue(rng.uniform(), 0.1 * rng.uniform(0.7, 1.3))))
    return out


def _requests(src, seed, n=6):
    """Uneven viewports (ragged tiles, a single pixel), channel subsets in
    any order, perspective and orthographic cameras; every third request
    with the LOD-adaptive step."""
    rng = np.random.default_rng(seed)
    sizes = [(64, 48), (100, 70), (33, 17), (128, 128), (1, 1), (200, 90), (40, 160), (96, 33)]
    cams = synth.orbit_path(src.dims, src.spacing, 16, az_step_deg=23.0, az0_deg=float(seed))
    reqs = []
    for k in range(n):
        W, H = sizes[(k + seed) % len(sizes)]
        nv = int(rng.integers(1, N_CH + 1))
        sub = rng.permutation(N_CH)[:nv]
        if k == 3:
            cam = synth.camera_oblique_ortho(src.dims, src.spacing, seed + k, W, H)
        else:
            cam = dict(cams[k])
            cam["tx"] = cam["ty"] * W / H
        reqs.append(dict(W=W, H=H, cam=cam, chans=_chans(sub, seed * 31 + k), frame=2 + k,
                         flags=resoct.RENDER_ADAPTIVE_STEP if k % 3 == 2 else 0))
    return reqs


class Rig:
    def __init__(self, scene, reqs):
        self.s, self.reqs = scene, reqs
        self.tf = [scene.tf_tensor(r["chans"]) for r in reqs]
        self.stats = torch.zeros((len(reqs), 8), dtype=torch.int64, device="cuda")

    def fd(self, k, stats=True):
        r = self.reqs[k]
        return resoct.frame_desc(r["frame"], r["cam"], r["W"], r["H"], 0.5, r["chans"], self.tf[k],
                                 self.s.vol.n_levels, stats=self.stats[k] if stats else None,
                                 flags=r.get("flags", 0))

    def out(self, k, fill=np.nan):
        r = self.reqs[k]
        return torch.full((r["H"] * r["W"] * 4,), fill, dtype=torch.float32, device="cuda")

    def image(self, k, t):
        r = self.reqs[k]
        return gpu_rgba(t, r["H"], r["W"])

    def frame_kernel(self):
        imgs = []
        self.stats.zero_()
        for k in range(len(self.reqs)):
            o = self.out(k)
            self.s.tree.render(self.fd(k), o)
            imgs.append(o)
        torch.cuda.synchronize()
        st = self.stats.cpu().numpy().copy()
        return [self.image(k, o) for k, o in enumerate(imgs)], st


def _same(a, b, name):
    exact = np.array_equal(a, b)
    if not exact:
        compare_images(a, b, np.zeros(a.shape[:2], np.int32))
    return exact


def test_alone_equals_mix_equals_frame_kernel(scene):
    rig = Rig(scene, _requests(scene.src, 1))
    ref, st_ref = rig.frame_kernel()
    srv = resoct.Server(scene.tree, max_requests=16, max_tiles=4096)
    exact = 0
    # alone: one request per batch, kernel chosen by its channel count
    for k in range(len(rig.reqs)):
        o = rig.out(k)
        torch.cuda.synchronize()
        srv.wait(srv.launch([rig.fd(k, stats=False)], [o]))
        exact += _same(rig.image(k, o), ref[k], f"alone-{k}")
    # the mix, eager and as graphs (16-channel kernel)
    for graph in (False, True):
        rig.stats.zero_()
        outs = [rig.out(k) for k in range(len(rig.reqs))]
        torch.cuda.synchronize()
        t = srv.launch([rig.fd(k) for k in range(len(rig.reqs))], outs, graph=graph)
        srv.wait(t)
        assert all(srv.request_done(t, k) for k in range(len(rig.reqs))), "completion flags not posted"
        st = rig.stats.cpu().numpy()
        for k in range(len(rig.reqs)):
            exact += _same(rig.image(k, outs[k]), ref[k], f"mix-{k}")
        assert np.array_equal(st[:, :5], st_ref[:, :5]), "per-request sample statistics differ"
    _report("serve-alone-mix", requests=len(rig.reqs), bit_exact=f"{exact}/{3 * len(rig.reqs)}",
            samples=int(st_ref[:, 0].sum()))


def test_graph_replays_with_new_contents(scene):
    """Each half's graph is captured once and replayed with other batches
    (other requests, counts and sizes), with eager work in between; every
    replay equals the frame kernel."""
    srv = resoct.Server(scene.tree, max_requests=16, max_tiles=4096)
    rigs = [Rig(scene, _requests(scene.src, 10 + i, n=3 + i % 4)) for i in range(6)]
    refs = [rig.frame_kernel()[0] for rig in rigs]
    pending = []
    for i, rig in enumerate(rigs):
        outs = [rig.out(k) for k in range(len(rig.reqs))]
        torch.cuda.synchronize()
        t = srv.launch([rig.fd(k, stats=False) for k in range(len(rig.reqs))], outs, graph=True)
        pending.append((t, i, outs))
        if i % 2 == 1:
            # eager work of the program between replays
            x = torch.randn(1 << 20, device="cuda")
            (x * 2 + 1).sum().item()
            for t_, j, o_ in pending:
                srv.wait(t_)
                for k in range(len(rigs[j].reqs)):
                    _same(rigs[j].image(k, o_[k]), refs[j][k], f"replay-{j}-{k}")
            pending = []


def test_served_request_matches_oracle(scene):
    src = scene.src
    reqs = _requests(src, 3, n=4)
    r = reqs[2]
    rig = Rig(scene, [r])
    srv = resoct.Server(scene.tree, max_requests=4, max_tiles=256)
    o = rig.out(0)
    torch.cuda.synchronize()
    srv.wait(srv.launch([rig.fd(0, stats=False)], [o]))
    V = oracle.make_volume(src.dims, src.spacing, src.n_channels, src.bits, 32, src.n_levels, (16, 16, 4), 5)
    ids = oracle.dense_ids(V)
    res_slot = np.arange(len(ids), dtype=np.uint32)
    from tests.helpers import leaf_grid
    lg = leaf_grid(src.dims, (16, 16, 4), 5)
    leaf_mm = np.stack([src.leaf_minmax(c, (16, 16, 4), lg) for c in range(src.n_channels)])
    assert r["flags"] & resoct.RENDER_ADAPTIVE_STEP
    fr, keep = oracle.make_frame(r["cam"], r["W"], r["H"], 0.5, r["chans"], term_margin=1e-6, adaptive=True)
    ref = oracle.render(V, src.levels, res_slot, leaf_mm, fr, len(ids))
    st = compare_images(rig.image(0, o), ref["rgba"], ref["amb_pix"], alt=oracle_alt(ref))
    _report("serve-oracle", W=r["W"], H=r["H"], channels=len(r["chans"]), **st)


def test_server_errors(scene):
    rig = Rig(scene, _requests(scene.src, 5, n=3))
    srv = resoct.Server(scene.tree, max_requests=2, max_tiles=8)
    outs = [rig.out(k) for k in range(3)]
    with pytest.raises(resoct.ResoctError) as e:
        srv.prepare([rig.fd(k) for k in range(3)], outs)  # 3 > max_requests
    assert e.value.code == -2
    with pytest.raises(resoct.ResoctError) as e:
        srv.submit()  # nothing prepared
    assert e.value.code == -5
    big = dict(rig.reqs[0], W=400, H=300)
    rig2 = Rig(scene, [big])
    with pytest.raises(resoct.ResoctError) as e:
        srv.prepare([rig2.fd(0)], [rig2.out(0)])  # 22 work items > 8
    assert e.value.code == -2
    with pytest.raises(resoct.ResoctError):
        srv.poll(12345)
    # a valid batch still works after the errors
    small = dict(rig.reqs[0], W=8, H=8)
    rig3 = Rig(scene, [small])
    o = rig3.out(0)
    ref, _ = rig3.frame_kernel()
    srv.wait(srv.launch([rig3.fd(0, stats=False)], [o]))
    assert np.array_equal(rig3.image(0, o), ref[0])


def test_arena_first_fit():
    a = Arena.__new__(Arena)
    a.size, a.free_off, a.free_len, a.used, a.peak = 4096, [0], [4096], 0, 0
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert x == (0, 1024) and y == (1024, 1024) and z == (2048, 1024)
    assert a.alloc(2000) is None
    a.free(*y)
    assert a.alloc(1500) is None
    a.free(*x)
    assert a.alloc(1500) == (0, 1536)
    a.free(0, 1536)
    a.free(*z)
    assert a.free_off == [0] and a.free_len == [4096] and a.used == 0


def test_serving_loop_real_time(scene):
    """A Poisson trace served in real time under a small output budget:
    every request completes, the budget holds, and every image equals the
    frame kernel's image of that request."""
    trace = make_trace(scene, rate=300.0, duration=0.25, n_clients=8)
    assert len(trace) > 20
    budget = 3 * 16 * 1920 * 1080
    loop = ServingLoop(scene, out_budget=budget, max_requests=8, max_tiles=1 << 14, graph=True)
    got = {}
    loop.run(trace, on_done=lambda r, img: got.__setitem__(r.rid, img.cpu().numpy().copy()))
    assert len(got) == len(trace)
    assert loop.arena.used == 0 and loop.arena.peak <= loop.arena.size
    lat = latency_summary(trace)
    assert lat["n"] == len(trace) and np.isfinite(lat["p99_ms"])
    out = torch.empty(4 * 1920 * 1080, dtype=torch.float32, device="cuda")
    n_exact = 0
    for r in trace:
        fd = resoct.frame_desc(r.frame, r.cam, r.W, r.H, 0.5, r.chans, r.tf, scene.vol.n_levels)
        scene.tree.render(fd, out)
        ref = gpu_rgba(out, r.H, r.W)
        img = got[r.rid][: r.H * r.W * 4].reshape(r.H, r.W, 4).astype(np.float64)
        n_exact += _same(img, ref, f"loop-{r.rid}")
    _report("serve-loop", requests=len(trace), batches=loop.n_batches, mean_batch=np.mean(loop.batch_sizes),
            bit_exact=f"{n_exact}/{len(trace)}", peak_mb=loop.arena.peak / 2**20, **lat)


def test_load_shedding_bounds_queue_wait(scene):
    """Arrivals above capacity with a queue-wait limit: every request is
    either served or shed, none waits in the queue longer than the limit
    (plus one loop pass), and the served ones finish."""
    trace = make_trace(scene, rate=600.0, duration=0.5, n_clients=16)
    loop = ServingLoop(scene, out_budget=4 * 16 * 1920 * 1080, max_requests=16, max_tiles=1 << 15, graph=True)
    max_wait = 0.05
    loop.run(trace, max_wait=max_wait)
    served = [r for r in trace if not r.shed]
    shed = [r for r in trace if r.shed]
    assert shed and served
    assert all(np.isfinite(r.done) for r in served)
    assert all(not np.isfinite(r.done) and not np.isfinite(r.admitted) for r in shed)
    assert max(r.admitted - r.arrival for r in served) <= max_wait + 0.02
    lat = latency_summary(trace)
    assert lat["n"] == len(served) and np.isfinite(lat["p99_ms"])
    _report("serve-shedding", requests=len(trace), served=len(served), shed=len(shed), **lat)


def _wait_done(srv, tickets, limit_s=60.0):
    import time
    t0 = time.perf_counter()
    while not all(srv.done(t) for t in tickets):
        assert time.perf_counter() - t0 < limit_s, "continuous requests did not finish"
        time.sleep(1e-4)


def test_continuous_admission_equals_frame_kernel(scene):
    """Requests admitted one at a time into a small ring (4 slots, 32 work
    items, so admissions wait for completions and the ring wraps), some
    while others render, a large one among them: every image and every
    request's sample statistics equal the frame kernel's."""
    import time
    reqs = []
    for i in range(5):
        reqs += _requests(scene.src, 40 + i, n=6)
    big = _requests(scene.src, 44, n=1)[0]
    big.update(W=400, H=300, cam=dict(big["cam"], tx=big["cam"]["ty"] * 400 / 300))
    reqs.insert(2, big)
    rig = Rig(scene, reqs)
    ref, st_ref = rig.frame_kernel()
    srv = resoct.Server(scene.tree, max_requests=4, max_tiles=32)
    items = sum(resoct.serve_work_items(r["W"], r["H"]) for r in reqs)
    assert items > 2 * 32 and resoct.serve_work_items(400, 300) <= 32
    rig.stats.zero_()
    outs = [rig.out(k) for k in range(len(reqs))]
    torch.cuda.synchronize()
    tickets, waits = [], 0
    t0 = time.perf_counter()
    for k in range(len(reqs)):
        while True:
            t = srv.enqueue(rig.fd(k), outs[k])
            if t is not None:
                break
            waits += 1  # every slot busy or the ring full: wait for completions
            assert time.perf_counter() - t0 < 60.0, "admission never succeeded"
            time.sleep(1e-4)
        tickets.append(t)
    _wait_done(srv, tickets)
    srv.drain()
    assert tickets == list(range(tickets[0], tickets[0] + len(reqs)))
    st = rig.stats.cpu().numpy()
    exact = sum(_same(rig.image(k, outs[k]), ref[k], f"cont-{k}") for k in range(len(reqs)))
    assert np.array_equal(st[:, :5], st_ref[:, :5]), "per-request sample statistics differ"
    with pytest.raises(resoct.ResoctError):
        srv.done(tickets[-1] + 1)
    _report("serve-continuous", requests=len(reqs), work_items=items, admission_waits=waits,
            bit_exact=f"{exact}/{len(reqs)}")


def test_continuous_mixed_with_batches(scene):
    """Batches and continuous admission on one server, interleaved: both
    queues' images equal the frame kernel's."""
    rig = Rig(scene, _requests(scene.src, 50, n=6))
    ref, _ = rig.frame_kernel()
    srv = resoct.Server(scene.tree, max_requests=8, max_tiles=256)
    outs = [rig.out(k) for k in range(6)]
    torch.cuda.synchronize()
    tc = [srv.enqueue(rig.fd(k, stats=False), outs[k]) for k in (0, 1)]
    tb = srv.launch([rig.fd(k, stats=False) for k in (2, 3)], [outs[2], outs[3]])
    tc += [srv.enqueue(rig.fd(k, stats=False), outs[k]) for k in (4, 5)]
    assert None not in tc
    _wait_done(srv, tc)
    srv.wait(tb)
    srv.drain()
    exact = sum(_same(rig.image(k, outs[k]), ref[k], f"mixed-{k}") for k in range(6))
    _report("serve-continuous-mixed", requests=6, bit_exact=f"{exact}/6")


def test_serving_loop_continuous(scene):
    """The real-time loop with continuous admission under a small output
    budget: every request completes, the budget holds, requests are admitted
    while others are unfinished, and every image equals the frame kernel's."""
    trace = make_trace(scene, rate=300.0, duration=0.25, n_clients=8, arrival_seed=3004)
    assert len(trace) > 20
    budget = 3 * 16 * 1920 * 1080
    loop = ServingLoop(scene, out_budget=budget, max_requests=8, max_tiles=1 << 14, continuous=True)
    got = {}
    loop.run(trace, on_done=lambda r, img: got.__setitem__(r.rid, img.cpu().numpy().copy()))
    assert len(got) == len(trace)
    assert loop.arena.used == 0 and loop.arena.peak <= loop.arena.size
    assert max(loop.in_flight_at_admission) >= 1, "no request was admitted while another was unfinished"
    lat = latency_summary(trace)
    assert lat["n"] == len(trace) and np.isfinite(lat["p99_ms"])
    out = torch.empty(4 * 1920 * 1080, dtype=torch.float32, device="cuda")
    n_exact = 0
    for r in trace:
        fd = resoct.frame_desc(r.frame, r.cam, r.W, r.H, 0.5, r.chans, r.tf, scene.vol.n_levels)
        scene.tree.render(fd, out)
        ref = gpu_rgba(out, r.H, r.W)
        img = got[r.rid][: r.H * r.W * 4].reshape(r.H, r.W, 4).astype(np.float64)
        n_exact += _same(img, ref, f"cloop-{r.rid}")
    _report("serve-loop-continuous", requests=len(trace), mean_in_flight=np.mean(loop.in_flight_at_admission),
            bit_exact=f"{n_exact}/{len(trace)}", peak_mb=loop.arena.peak / 2**20, **lat)


def test_slot_pool_address_above_2gib_in_low_word(scene):
    """The slot pool at an address whose low 32-bit half has bit 31 set (the
    kernels rebuild the pool address from its two halves as scalar values):
    the frame kernel gives the images of the scene whose pool lies elsewhere,
    and batches and continuous admission give the frame kernel's images."""
    src = scene.src
    n_bricks = scene.cache.n_slots
    need = int(scene.cache.sizes.slots)
    pad = torch.empty(need + (1 << 31) + 512, dtype=torch.uint8, device="cuda")
    base = pad.data_ptr()
    lo = base & 0xFFFFFFFF
    off = 0 if lo >= 0x80000000 and lo + need < (1 << 32) else ((0x80000000 - lo) % (1 << 32) + 255) // 256 * 256
    pool = pad[off:off + need]
    addr = pool.data_ptr()
    assert addr % 256 == 0 and (addr & 0xFFFFFFFF) >= 0x80000000
    print(f"[pool] address {addr:#x} (low half {addr & 0xFFFFFFFF:#010x})", flush=True)
    s2 = GpuScene(src, 32, (16, 16, 4), 5, n_slots=n_bricks, max_batch=2048, slots=pool)
    s2.upload(0, s2.all_ids())
    s2.tree.update_residency()
    torch.cuda.synchronize()
    reqs = _requests(src, 60, n=6)
    ref, _ = Rig(scene, reqs).frame_kernel()
    rig = Rig(s2, reqs)
    img, _ = rig.frame_kernel()
    for k in range(len(reqs)):
        assert np.isfinite(img[k]).all()
        assert np.array_equal(img[k], ref[k]), f"frame kernel image {k} differs with the pool at {addr:#x}"
    srv = resoct.Server(s2.tree, max_requests=8, max_tiles=256)
    outs = [rig.out(k) for k in range(len(reqs))]
    torch.cuda.synchronize()
    srv.wait(srv.launch([rig.fd(k, stats=False) for k in range(len(reqs))], outs))
    exact = sum(_same(rig.image(k, outs[k]), img[k], f"pool-batch-{k}") for k in range(len(reqs)))
    outs2 = [rig.out(k) for k in range(len(reqs))]
    torch.cuda.synchronize()
    tickets = [srv.enqueue(rig.fd(k, stats=False), outs2[k]) for k in range(len(reqs))]
    assert None not in tickets
    _wait_done(srv, tickets)
    srv.drain()
    exact += sum(_same(rig.image(k, outs2[k]), img[k], f"pool-cont-{k}") for k in range(len(reqs)))
    _report("serve-pool-address", address=hex(addr), bit_exact=f"{exact}/{2 * len(reqs)}")
