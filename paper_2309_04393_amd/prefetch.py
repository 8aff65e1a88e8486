"""Request-driven streaming with an optional learned prefetcher.

The plain policy streams the frame's requested bricks by (count desc,
ID asc), at most U per frame.  The learned policy streams the same list and
fills the rest of the budget with bricks the predictor (24-64-64-9 network,
MFMA kernels in the library) expects to be requested or read within the next
four frames, by probability; it falls back to the plain policy while its
online precision (share of its extra bricks that were needed within four
frames) is below one half.  The network trains online every frame on the
rows of four frames earlier, labelled from the brick history.  The policy
only changes which bricks are streamed; a frame rendered from a given cache
state is the same either way.  Below the precision gate a probe of at most
`probe` predicted bricks per frame is still streamed, so a model that
improves is noticed.
"""
from __future__ import annotations

import numpy as np
import torch

from . import resoct


class BrickStore:
    """Every brick of a volume source held in device memory (the data
    server's content when it fits in HBM), addressed by brick ID."""

    def __init__(self, scene, device="cuda"):
        ids = scene.all_ids()
        self.index = {int(i): k for k, i in enumerate(ids)}
        stride = scene.cache.slot_stride
        self.data = torch.empty((len(ids), stride), dtype=torch.uint8, device=device)
        for s in range(0, len(ids), 4096):
            part = ids[s:s + 4096]
            st = scene.stage(part)
            self.data[s:s + len(part)].copy_(st.view(-1, stride)[:len(part)])
        torch.cuda.synchronize()

    def gather(self, ids) -> torch.Tensor:
        idx = torch.tensor([self.index[int(i)] for i in ids], dtype=torch.int64, device=self.data.device)
        return self.data.index_select(0, idx).reshape(-1)


class StreamingLoop:
    def __init__(self, scene, store: BrickStore, chans, W, H, U, step, policy="plain", net=None, lr=3e-3,
                 threshold=0.5, lod_bias=1.0, train=True, train_steps=4, gate=0.5, probe=32):
        self.s, self.store = scene, store
        self.chans, self.W, self.H, self.U, self.step = chans, W, H, U, step
        self.policy, self.net, self.lr, self.thr, self.lod_bias, self.train = policy, net, lr, threshold, lod_bias, train
        self.train_steps, self.gate, self.probe = train_steps, gate, probe
        self.tf = scene.tf_tensor(chans)
        self.out = torch.empty(W * H * 4, dtype=torch.float32, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        self.pf = resoct.PrefetchRows(scene.tree)
        R = self.pf.rows
        self.ring = [torch.zeros((R, 32), dtype=torch.float16, device="cuda") for _ in range(5)]
        self.y = torch.zeros((R, 16), dtype=torch.uint8, device="cuda")
        self.m = torch.zeros((R, 16), dtype=torch.uint8, device="cuda")
        self.z = torch.zeros((R, 16), dtype=torch.float32, device="cuda")
        self.extra = {}  # frame -> extra (predicted) bricks streamed
        self.hits, self.tries = [], []
        self.log = []

    def precision(self):
        n = sum(self.tries[-8:])
        return (sum(self.hits[-8:]) / n) if n else 1.0

    def frame(self, f, cam):
        s = self.s
        self.stats.zero_()
        r = s.render(f, cam, self.W, self.H, self.step, self.chans, tf_dev=self.tf, out=self.out, stats=self.stats,
                     lod_bias=self.lod_bias)
        fd = r["fd"]
        self.pf.record(f)
        ids, cnt, nu, tot = s.cache.read_requests(1 << 20)
        plain = ids[np.lexsort((ids, -cnt.astype(np.int64)))][: self.U]
        up = plain
        learned_used = False
        if self.policy == "learned":
            x = self.ring[f % 5]
            self.pf.features(fd, x)
            if f >= 4 and self.train:
                self.pf.labels(self.y, self.m)
                for _ in range(self.train_steps):
                    self.net.train_step(self.ring[(f - 4) % 5], self.y, self.m, self.lr)
            # precision of the extra bricks streamed four frames ago
            if (f - 4) in self.extra:
                old = self.extra.pop(f - 4)
                if len(old):
                    h = self.pf.hist.cpu().numpy()
                    dense = self._dense(old)
                    self.hits.append(int((h[dense] != 0).sum()))
                    self.tries.append(len(old))
            room = self.U - len(plain)
            # below the precision gate only a small probe of predictions is
            # streamed, which keeps measuring the precision
            if self.precision() < self.gate:
                room = min(room, self.probe)
            if room > 0:
                self.net.forward(x, self.z)
                cid, cpr = self.pf.candidates(self.z, self.thr)
                if len(cid):
                    order = np.lexsort((cid, -cpr))
                    pset = set(int(i) for i in plain)
                    extra = [int(cid[i]) for i in order if int(cid[i]) not in pset][:room]
                    if extra:
                        up = np.concatenate([plain, np.array(extra, np.uint32)])
                        self.extra[f] = np.array(extra, np.uint32)
                        learned_used = True
        if len(up):
            s.cache.stream_bricks(f, up, self.store.gather(up))
        s.tree.update_residency()
        st = self.stats.cpu().numpy()
        miss = float(st[2]) / max(float(st[4]), 1.0)
        rec = dict(frame=f, missing=miss, requested=int(nu), uploads=int(len(up)), extra=int(len(up) - len(plain)),
                   learned=learned_used, bytes=int(len(up)) * s.cache.slot_stride)
        self.log.append(rec)
        return rec

    def _dense(self, ids):
        # history is indexed by the library's dense order (channel, level, z, y, x)
        out = []
        for i in ids:
            c, l, b = self.s.vol.decode(int(i))
            nx, ny, nz = self.s.nb[l]
            off = int(sum(int(np.prod(self.s.nb[k])) for k in range(l)))
            per = int(sum(int(np.prod(self.s.nb[k])) for k in range(self.s.vol.n_levels)))
            out.append(c * per + off + (b[2] * ny + b[1]) * nx + b[0])
        return np.array(out, np.int64)


def first_below(log, thr=0.01, hold=1):
    """First frame from which the missing-sample fraction stays below thr
    for `hold` frames (None if never)."""
    for i in range(len(log)):
        win = log[i:i + hold]
        if len(win) == hold and all(r["missing"] < thr for r in win):
            return log[i]["frame"]
    return None


def run_path(scene, store, cams, chans, W, H, U, step, policy, net=None, empty_state=None, lr=3e-3,
             train=True, lod_bias=1.0, threshold=0.5, train_steps=4, gate=0.5, probe=32):
    """One camera path from an empty cache; returns the loop's per-frame
    log and a summary."""
    if empty_state is not None:
        restore_state(scene, empty_state)
    loop = StreamingLoop(scene, store, chans, W, H, U, step, policy=policy, net=net, lr=lr,
                         threshold=threshold, lod_bias=lod_bias, train=train, train_steps=train_steps, gate=gate,
                         probe=probe)
    for f, cam in enumerate(cams, start=1):
        loop.frame(f, cam)
    log = loop.log
    miss = np.array([r["missing"] for r in log])
    # frames to converge: the first frame from which fewer than 1 % of the
    # channel samples miss their desired brick for 5 frames in a row
    return log, dict(missing_curve=[round(float(x), 5) for x in miss], frames=len(log),
                     frames_to_converge=first_below(log, 0.01, hold=5), first_below_1pct=first_below(log, 0.01),
                     mean_missing=float(miss.mean()), bytes_streamed=int(sum(r["bytes"] for r in log)),
                     uploads=int(sum(r["uploads"] for r in log)), extra=int(sum(r["extra"] for r in log)),
                     learned_frames=int(sum(1 for r in log if r["learned"])),
                     precision=loop.precision() if policy == "learned" else None)


def save_state(scene):
    """Device buffers and host mirror of a scene's cache and octree."""
    dev = {("c", k): v.clone() for k, v in scene.cache.t.items() if k not in ("scratch", "slots")}
    dev.update({("t", k): v.clone() for k, v in scene.tree.t.items() if k != "scratch"})
    torch.cuda.synchronize()
    return dev, scene.cache.save_state()


def restore_state(scene, state):
    dev, host = state
    for (kind, k), v in dev.items():
        (scene.cache.t if kind == "c" else scene.tree.t)[k].copy_(v)
    torch.cuda.synchronize()
    scene.cache.load_state(host)
