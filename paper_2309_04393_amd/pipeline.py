"""Host-side frame loop over the C ABI: scene set-up from a volume source,
brick staging, rendering and plain request-driven streaming.

A volume source is anything with the generator's interface: dims, spacing,
n_channels, bits, n_levels, bricks(c, l, coords, B) -> [n][E][E][E] and
leaf_minmax(c, leaf, leaf_grid) -> [n_leaves][2] (the data server's bricks
and metadata answers).
"""
from __future__ import annotations

import numpy as np
import torch

from . import resoct


class GpuScene:
    def __init__(self, src, brick: int, leaf, depth: int, n_slots: int, max_batch: int = 4096,
                 start_level: int = 0, device="cuda", set_metadata=True, cache_channels=None, slots=None):
        self.src = src
        self.device = device
        m = src.n_channels if cache_channels is None else int(cache_channels)
        assert 1 <= m <= src.n_channels
        self.vol = resoct.Volume(src.dims, src.spacing, m, 1 if src.bits == 8 else 2,
                                 brick, src.n_levels)
        self.cache = resoct.Cache(self.vol, n_slots, max_batch, device=device, slots=slots)
        self.tree = resoct.Octree(self.cache, leaf, depth, start_level, device=device)
        self.B = brick
        self.E = brick + 2
        self.leaf = tuple(leaf)
        self.ldims, self.lf, self.nb = self.vol.levels()
        self.np_dtype = np.uint8 if src.bits == 8 else np.uint16
        if set_metadata:
            for c in range(m):
                self.set_metadata(c, src.leaf_minmax(self.channel_map[c], self.leaf, self.tree.leaf_grid))

    @property
    def channel_map(self) -> list:
        """Cache channel c holds the source's channel channel_map[c] (Sec. 5.2:
        the octree and page tables reference m of the n channels at a time);
        the map is the cache's (the library's host state)."""
        return self.cache.channel_map()

    def set_metadata(self, c, leaf_mm: np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(leaf_mm, dtype=np.uint16).reshape(-1).view(np.int16))
        t = t.to(self.device).view(torch.uint16)
        self.tree.set_leaf_metadata(c, t)
        torch.cuda.current_stream().synchronize()

    def set_unknown(self, c: int):
        """Every leaf of cache channel c unknown ([0, max raw value]) until
        brick data give it metadata (Sec. 5.2, Sec. 5.3)."""
        self.tree.set_leaf_unknown(c)
        torch.cuda.current_stream().synchronize()

    def exchange_channel(self, c: int, src_channel: int, metadata: str = "server"):
        """Run-time channel exchange (Sec. 5.2): cache channel c now holds the
        source's channel src_channel.  The old channel's bricks leave the
        cache, the channel gets the new data's metadata ("server") or unknown
        leaves ("unknown": [0, max raw value], refined later from bricks),
        and the residency masks are updated; the new bricks arrive through
        the usual request-driven uploads."""
        self.cache.evict_channel(c)
        self.cache.set_channel_map(c, int(src_channel))
        if metadata == "server":
            self.set_metadata(c, self.src.leaf_minmax(int(src_channel), self.leaf, self.tree.leaf_grid))
        else:
            self.set_unknown(c)
        self.tree.update_residency()

    # ------------------------------------------------------------- bricks
    def all_ids(self, channels=None, levels=None):
        ids = []
        for c in (range(self.vol.n_channels) if channels is None else channels):
            for l in (range(self.vol.n_levels) if levels is None else levels):
                nx, ny, nz = self.nb[l]
                for bz in range(nz):
                    for by in range(ny):
                        for bx in range(nx):
                            ids.append(self.vol.encode(c, l, (bx, by, bz)))
        return np.array(ids, dtype=np.uint32)

    def stage(self, ids) -> torch.Tensor:
        """Fetch the bricks of `ids` from the source and pack them at the
        cache's slot stride in device memory."""
        n = len(ids)
        stride = self.cache.slot_stride
        host = np.zeros((max(n, 1), stride), np.uint8)
        nbytes = self.E ** 3 * (1 if self.np_dtype == np.uint8 else 2)
        # (source channel, level, brick) of each ID
        dec = [(int(r[0]), int(r[1]), (int(r[2]), int(r[3]), int(r[4]))) for r in self.cache.source_bricks(ids)]
        if hasattr(self.src, "bricks_multi"):
            # one generator pass per brick position serves every channel there
            groups = {}
            for i, (c, l, b) in enumerate(dec):
                groups.setdefault(l, {}).setdefault(b, []).append((i, c))
            for l, pos in groups.items():
                coords = list(pos.keys())
                chs = sorted({c for lst in pos.values() for _, c in lst})
                cidx = {c: k for k, c in enumerate(chs)}
                br = self.src.bricks_multi(l, coords, self.B, chs)
                raw = np.ascontiguousarray(br).view(np.uint8).reshape(len(coords), len(chs), nbytes)
                for p_i, b in enumerate(coords):
                    for (i, c) in pos[b]:
                        host[i, :nbytes] = raw[p_i, cidx[c]]
        else:
            groups = {}
            for i, (c, l, b) in enumerate(dec):
                groups.setdefault((c, l), []).append((i, b))
            for (c, l), lst in groups.items():
                br = self.src.bricks(c, l, [b for _, b in lst], self.B)
                raw = np.ascontiguousarray(br).view(np.uint8).reshape(len(lst), nbytes)
                for k, (i, _) in enumerate(lst):
                    host[i, :nbytes] = raw[k]
        return torch.from_numpy(host.reshape(-1)).to(self.device)

    def upload(self, frame: int, ids, staged: torch.Tensor = None) -> np.ndarray:
        ids = np.asarray(ids, dtype=np.uint32)
        flags = np.zeros(0, np.uint8)
        for s in range(0, len(ids), self.cache.max_batch):
            part = ids[s:s + self.cache.max_batch]
            st = self.stage(part) if staged is None else staged[s * self.cache.slot_stride:]
            flags = np.concatenate([flags, self.cache.stream_bricks(frame, part, st)])
        return flags

    # ------------------------------------------------------------- frames
    def tf_tensor(self, channels) -> torch.Tensor:
        return torch.from_numpy(np.stack([np.asarray(ch["tf"], np.float32) for ch in channels])) \
            .contiguous().to(self.device)

    def render(self, frame, cam, W, H, step, channels, tf_dev=None, out=None, aov=False, bricks=False, **kw):
        tf_dev = self.tf_tensor(channels) if tf_dev is None else tf_dev
        out = torch.empty(H * W * 4, dtype=torch.float32, device=self.device) if out is None else out
        aov_t = torch.zeros(H * W * self.vol.n_levels, dtype=torch.int32, device=self.device) if aov else None
        rb_t = torch.empty(H * W * (1 + len(channels)), dtype=torch.int32, device=self.device) if bricks else None
        fd = resoct.frame_desc(frame, cam, W, H, step, channels, tf_dev, self.vol.n_levels, aov=aov_t,
                               bricks=rb_t, **kw)
        self.tree.render(fd, out)
        res = {"rgba": out, "fd": fd, "tf": tf_dev}
        if aov:
            res["aov"] = aov_t
        if bricks:
            res["bricks"] = rb_t.view(H, W, 1 + len(channels))[..., 0]
        return res
