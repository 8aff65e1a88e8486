"""Continuous-batching serving loop over the batched renderer.

Render requests (a camera, a viewport, a subset of the channels with their
transfer functions) arrive over time.  The loop admits queued requests, in
arrival order, into the next batch while the batch has descriptor slots and
tiles left and the output arena (a fixed HBM budget for result images) can
hold the request's image; a request that does not fit waits until a running
batch finishes and frees memory.  Batches alternate between the server's two
halves, so the next batch is prepared and queued while the previous one
renders and the tail of one overlaps the head of the next on the device.
With graph submission each half's device work (descriptor copy, queue reset,
persistent kernel) is a captured graph replayed with new contents.

With continuous admission (continuous=True) there are no batches: each
queued request is admitted on its own as soon as a request slot, room in
the server's work-item ring and output memory are free, also while others
render; the workgroups of the running serving kernels take its work items
as they free up (and the launch made for it fills emptied compute units),
so a request arriving mid-batch does not wait for a batch to retire.

Latency of a request = its completion on the device (the kernel posts each
request's completion to mapped host memory when its last pixels are
written; the loop polls) - its arrival.  Within a batch the smallest
requests come first.  The cache and octree are static while serving
(every brick resident); streaming would be ordered between batches.
"""
from __future__ import annotations

import bisect
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import resoct


class Arena:
    """First-fit allocator over one device buffer (offsets aligned to 256
    bytes); admission asks it for each request's image."""

    def __init__(self, nbytes: int, device="cuda"):
        self.size = int(nbytes) // 256 * 256
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free_off = [0]
        self.free_len = [self.size]
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = (int(n) + 255) // 256 * 256
        for k, (o, ln) in enumerate(zip(self.free_off, self.free_len)):
            if ln >= n:
                if ln == n:
                    del self.free_off[k], self.free_len[k]
                else:
                    self.free_off[k] += n
                    self.free_len[k] -= n
                self.used += n
                self.peak = max(self.peak, self.used)
                return o, n
        return None

    def free(self, o: int, n: int):
        k = bisect.bisect_left(self.free_off, o)
        self.free_off.insert(k, o)
        self.free_len.insert(k, n)
        self.used -= n
        # merge with the neighbours
        if k + 1 < len(self.free_off) and self.free_off[k] + self.free_len[k] == self.free_off[k + 1]:
            self.free_len[k] += self.free_len[k + 1]
            del self.free_off[k + 1], self.free_len[k + 1]
        if k > 0 and self.free_off[k - 1] + self.free_len[k - 1] == self.free_off[k]:
            self.free_len[k - 1] += self.free_len[k]
            del self.free_off[k], self.free_len[k]

    def view(self, o: int, n_floats: int) -> torch.Tensor:
        return self.buf[o:o + 4 * n_floats].view(torch.float32)


@dataclass
class Request:
    rid: int
    client: int
    arrival: float
    W: int
    H: int
    cam: dict
    chans: list          # [{c, lo, hi, W0, W1}] in visible-slot order
    tf: torch.Tensor     # [n_vis][256][4] float32 on the device
    frame: int = 1
    admitted: float = math.nan
    done: float = math.nan
    shed: bool = False
    mem: tuple = None
    ticket: int = 0
    fd: object = field(default=None, repr=False)

    @property
    def tiles(self):
        return resoct.serve_work_items(self.W, self.H)

    @property
    def image_bytes(self):
        return 16 * self.W * self.H


@dataclass
class Batch:
    ticket: int
    reqs: list
    submitted: float


class ServingLoop:
    def __init__(self, scene, out_budget: int = 2 << 30, max_requests: int = 64, max_tiles: int = 1 << 16,
                 step: float = 0.5, graph: bool = True, lod_bias: float = 1.0, term_alpha: float = 0.99,
                 continuous: bool = False):
        self.s = scene
        self.server = resoct.Server(scene.tree, max_requests, max_tiles)
        self.arena = Arena(out_budget)
        self.max_requests, self.max_tiles = max_requests, max_tiles
        self.step, self.graph, self.lod_bias, self.term_alpha = step, graph, lod_bias, term_alpha
        self.continuous = continuous
        self.ring_items = 1 << max(0, (max_tiles - 1).bit_length())  # the server's ring (a power of two)
        self.stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        self.n_batches = 0
        self.batch_sizes = []
        self.in_flight_at_admission = []  # continuous: requests unfinished when each one was admitted

    def frame_desc(self, r: Request, out: torch.Tensor):
        return resoct.frame_desc(r.frame, r.cam, r.W, r.H, self.step, r.chans, r.tf, self.s.vol.n_levels,
                                 term_alpha=self.term_alpha, lod_bias=self.lod_bias, stats=self.stats)

    def _admit(self, queue, now):
        batch, tiles = [], 0
        while queue and len(batch) < self.max_requests:
            r = queue[0]
            if r.tiles > self.max_tiles or r.image_bytes > self.arena.size:
                raise ValueError(f"request {r.rid} ({r.W}x{r.H}) can never be admitted")
            if tiles + r.tiles > self.max_tiles:
                break
            mem = self.arena.alloc(r.image_bytes)
            if mem is None:
                break
            queue.pop(0)
            r.mem, r.admitted = mem, now
            tiles += r.tiles
            batch.append(r)
        return batch

    def _submit(self, batch, now):
        # smallest requests first: each request completes (and is reported)
        # as soon as its own work items are done
        batch = sorted(batch, key=lambda r: r.tiles)
        outs = [self.arena.view(r.mem[0], 4 * r.W * r.H) for r in batch]
        fds = [self.frame_desc(r, o) for r, o in zip(batch, outs)]
        for r, fd in zip(batch, fds):
            r.fd = fd
        self.server.prepare(fds, outs, full_channels=self.graph)
        t = self.server.submit(self.graph)
        self.n_batches += 1
        self.batch_sizes.append(len(batch))
        return Batch(t, batch, now)

    def run(self, trace, on_done=None, idle_sleep=20e-6, deadline=None, max_wait=None):
        """Serve `trace` (requests sorted by arrival, times in seconds from
        the start) in real time; returns the wall time of the run.
        on_done(request, image) is called for each finished request before
        its image memory is released.  After `deadline` seconds nothing more
        is admitted: batches in flight finish, requests still queued or not
        yet arrived stay unfinished (done = nan).  With max_wait (seconds), a
        queued request that has waited longer is shed (r.shed = True, never
        rendered): load shedding keeps the latency of the served requests
        bounded when arrivals exceed the capacity."""
        if self.continuous:
            return self._run_continuous(trace, on_done, idle_sleep, deadline, max_wait)
        # the server's streams do not wait for work queued on torch's streams
        torch.cuda.synchronize()
        clock = time.perf_counter
        t0 = clock()
        i, n = 0, len(trace)
        queue, inflight = [], []
        while i < n or queue or inflight:
            now = clock() - t0
            if deadline is not None and now >= deadline:
                i = n
                queue = []
                if not inflight:
                    break
            progressed = False
            while i < n and trace[i].arrival <= now:
                queue.append(trace[i])
                i += 1
                progressed = True
            for b in list(inflight):
                # requests complete one by one (flags posted by the kernel);
                # the batch leaves the device when its kernel has ended
                for idx, r in enumerate(b.reqs):
                    if r.mem is not None and self.server.request_done(b.ticket, idx):
                        r.done = clock() - t0
                        if on_done is not None:
                            on_done(r, self.arena.view(r.mem[0], 4 * r.W * r.H))
                        self.arena.free(*r.mem)
                        r.mem = None
                        progressed = True
                if all(r.mem is None for r in b.reqs) and self.server.poll(b.ticket):
                    inflight.remove(b)
                    progressed = True
            if max_wait is not None and queue and now - queue[0].arrival > max_wait:
                keep = []
                for r in queue:
                    if now - r.arrival > max_wait:
                        r.shed = True
                    else:
                        keep.append(r)
                queue[:] = keep
                progressed = True
            if len(inflight) < 2 and queue:
                batch = self._admit(queue, now)
                if batch:
                    inflight.append(self._submit(batch, now))
                    progressed = True
            if not progressed:
                if inflight or i < n:
                    time.sleep(idle_sleep)
        return clock() - t0


    def _run_continuous(self, trace, on_done, idle_sleep, deadline, max_wait):
        torch.cuda.synchronize()
        clock = time.perf_counter
        t0 = clock()
        i, n = 0, len(trace)
        queue, inflight = [], []
        while i < n or queue or inflight:
            now = clock() - t0
            if deadline is not None and now >= deadline:
                i = n
                queue = []
                if not inflight:
                    break
            progressed = False
            while i < n and trace[i].arrival <= now:
                queue.append(trace[i])
                i += 1
                progressed = True
            for r in list(inflight):
                if self.server.done(r.ticket):
                    r.done = clock() - t0
                    if on_done is not None:
                        on_done(r, self.arena.view(r.mem[0], 4 * r.W * r.H))
                    self.arena.free(*r.mem)
                    r.mem = None
                    inflight.remove(r)
                    progressed = True
            if max_wait is not None and queue and now - queue[0].arrival > max_wait:
                keep = []
                for r in queue:
                    if now - r.arrival > max_wait:
                        r.shed = True
                    else:
                        keep.append(r)
                queue[:] = keep
                progressed = True
            # admit in arrival order while a slot, ring room and output memory are free
            while queue:
                r = queue[0]
                if r.tiles > self.ring_items or r.image_bytes > self.arena.size:
                    raise ValueError(f"request {r.rid} ({r.W}x{r.H}) can never be admitted")
                mem = self.arena.alloc(r.image_bytes)
                if mem is None:
                    break
                out = self.arena.view(mem[0], 4 * r.W * r.H)
                fd = self.frame_desc(r, out)
                t = self.server.enqueue(fd, out)
                if t is None:
                    self.arena.free(*mem)
                    break
                queue.pop(0)
                r.mem, r.admitted, r.ticket = mem, now, t
                self.in_flight_at_admission.append(len(inflight))
                inflight.append(r)
                progressed = True
            if not progressed:
                if inflight or i < n:
                    time.sleep(idle_sleep)
        self.server.drain()
        return clock() - t0


def latency_summary(trace, t_from=0.0):
    """Latency percentiles over the requests arriving from t_from on that
    were not shed; an unfinished request counts as infinitely late (p50_ms /
    p99_ms are None when that percentile is unbounded).  The *_completed_ms
    figures are over the finished requests only."""
    lat = np.array([r.done - r.arrival for r in trace if r.arrival >= t_from and not r.shed])
    if not len(lat):
        return dict(n=0)
    fin = np.isfinite(lat)
    lat = np.where(fin, lat, np.inf)

    def pct(q):
        with np.errstate(invalid="ignore"):  # interpolation next to infinite entries
            v = np.percentile(lat, q)
        return float(v * 1e3) if np.isfinite(v) else None
    done = lat[fin]
    return dict(n=int(len(lat)), completed=int(fin.sum()), p50_ms=pct(50), p99_ms=pct(99),
                mean_ms=float(done.mean() * 1e3) if fin.any() else None,
                max_ms=float(done.max() * 1e3) if fin.any() else None,
                p50_completed_ms=float(np.percentile(done, 50) * 1e3) if fin.any() else None,
                p99_completed_ms=float(np.percentile(done, 99) * 1e3) if fin.any() else None)


VIEWPORTS = ((256, 256), (512, 512), (1024, 1024), (1920, 1080))


def make_trace(scene, rate: float, duration: float, n_clients: int = 64, client_seed0: int = 2000,
               arrival_seed: int = 3000, n_channels: int = None, min_channels: int = 3, device="cuda"):
    """Poisson arrivals at `rate` requests/s over `duration` s from
    n_clients clients chosen uniformly; each client walks its own seeded
    camera path (one path frame per request) with its own transfer
    functions (hue offset, opacity scale, window jitter per channel); each
    request draws its viewport uniformly from VIEWPORTS and a channel subset
    of uniform size min_channels..n_channels.  All transfer-function tables
    are built up front in one device tensor."""
    import synth
    src = scene.src
    m = src.n_channels if n_channels is None else n_channels
    rng = np.random.default_rng(arrival_seed)
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    clients = rng.integers(0, n_clients, len(times))
    per_client = np.bincount(clients, minlength=n_clients)
    paths, ctf, cwin = [], [], []
    for k in range(n_clients):
        crng = np.random.default_rng(client_seed0 + k)
        nf = max(int(per_client[k]), 2)
        paths.append(synth.random_path(src.dims, src.spacing, client_seed0 + k, nf))
        h0 = crng.uniform(0, 1)
        tabs, wins = [], []
        for c in range(m):
            tabs.append(synth.tf_hue((h0 + c / m) % 1.0, 0.1 * crng.uniform(0.7, 1.3)))
            j = crng.uniform(0.8, 1.2, 2)
            wins.append(synth.window_fx(300 * j[0], 8000 * j[1]))
        ctf.append(tabs)
        cwin.append(wins)
    reqs, tfs, offs = [], [], []
    seen = np.zeros(n_clients, np.int64)
    off = 0
    for rid, (ta, k) in enumerate(zip(times, clients)):
        W, H = VIEWPORTS[rng.integers(0, len(VIEWPORTS))]
        nv = int(rng.integers(min_channels, m + 1))
        sub = np.sort(rng.choice(m, nv, replace=False))
        cam = dict(paths[k][seen[k]])
        seen[k] += 1
        if cam["proj"] == "persp":
            cam["tx"] = cam["ty"] * W / H
        chans = [dict(c=int(c), lo=0, hi=src.n_levels - 1, W0=cwin[k][c][0], W1=cwin[k][c][1]) for c in sub]
        tfs.extend(ctf[k][c] for c in sub)
        offs.append((off, nv))
        off += nv
        reqs.append(Request(rid, int(k), float(ta), W, H, cam, chans, None))
    tf_all = torch.from_numpy(np.stack(tfs).astype(np.float32)).to(device) if tfs else None
    for r, (o, nv) in zip(reqs, offs):
        r.tf = tf_all[o:o + nv]
    return reqs


def reset_trace(trace):
    for r in trace:
        r.admitted = r.done = math.nan
        r.shed = False
        r.mem = None
        r.fd = None
        r.ticket = 0
