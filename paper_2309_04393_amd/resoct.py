"""Thin ctypes binding of libresoct.so (the C ABI in include/resoct.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory (each buffer the *_query calls
size) and streams.  Importing this module fails loudly when the built
library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# RESOCT_LIB selects another build of the same library (same ABI)
LIB_PATH = os.environ.get("RESOCT_LIB", os.path.join(HERE, "_lib", "libresoct.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                      "python paper_2309_04393_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)

MAX_CHANNELS = 16
MAX_LEVELS = 16
INVALID = 0xFFFFFFFF
NOALLOC_MAX_PAIRS = 262144  # RO_NOALLOC_MAX_PAIRS
SNAPSHOT_SLOTS = 1
PROJ_ORTHO, PROJ_PERSP = 0, 1
RENDER_NO_SKIP, RENDER_AOV, RENDER_ADAPTIVE_STEP, RENDER_HOMOGENEOUS, RENDER_BRICKS = 1, 2, 4, 8, 16
RENDER_CHANNEL_RATES, RENDER_NODES, RENDER_TRAVERSAL_DEPTH = 32, 64, 128

c_i32, c_u32, c_u64, c_sz, c_vp, c_dbl = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double)


class VolumeDesc(ctypes.Structure):
    _fields_ = [("dims", c_i32 * 3), ("spacing", c_dbl * 3), ("n_channels", c_i32),
                ("bytes_per_voxel", c_i32), ("brick", c_i32), ("n_levels", c_i32)]


class CacheDesc(ctypes.Structure):
    _fields_ = [("n_slots", c_u32), ("max_batch", c_u32)]


class CacheSizes(ctypes.Structure):
    _fields_ = [("slots", c_sz), ("page_table", c_sz), ("counters", c_sz), ("slot_brick", c_sz),
                ("stamps", c_sz), ("seqs", c_sz), ("scratch", c_sz), ("slot_stride", c_sz)]


class CacheBuffers(ctypes.Structure):
    _fields_ = [("slots", c_vp), ("page_table", c_vp), ("counters", c_vp), ("slot_brick", c_vp),
                ("stamps", c_vp), ("seqs", c_vp), ("scratch", c_vp)]


class OctreeDesc(ctypes.Structure):
    _fields_ = [("leaf", c_i32 * 3), ("depth", c_i32), ("start_level", c_i32)]


class OctreeSizes(ctypes.Structure):
    _fields_ = [("node_meta", c_sz), ("node_mask", c_sz), ("node_flags", c_sz), ("scratch", c_sz),
                ("leaf_level", c_sz), ("n_nodes", c_u64), ("n_leaves", c_u64), ("leaf_grid", c_i32 * 3)]


class OctreeBuffers(ctypes.Structure):
    _fields_ = [("node_meta", c_vp), ("node_mask", c_vp), ("node_flags", c_vp), ("scratch", c_vp),
                ("leaf_level", c_vp)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("frame", c_u32), ("projection", c_i32), ("eye", c_dbl * 3), ("forward", c_dbl * 3),
                ("right", c_dbl * 3), ("up", c_dbl * 3), ("tx", c_dbl), ("ty", c_dbl),
                ("width", c_i32), ("height", c_i32), ("step", c_dbl), ("lod_bias", c_dbl),
                ("n_vis", c_i32), ("vis", c_i32 * MAX_CHANNELS), ("lod_lo", c_i32 * MAX_CHANNELS),
                ("lod_hi", c_i32 * MAX_CHANNELS), ("win_lo", c_u32 * MAX_CHANNELS),
                ("win_hi", c_u32 * MAX_CHANNELS), ("tf_dev", c_vp), ("term_alpha", ctypes.c_float),
                ("start_level", c_i32), ("flags", c_u32), ("aov_dev", c_vp), ("stats_dev", c_vp),
                ("bricks_dev", c_vp), ("nodes_dev", c_vp)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_P = ctypes.POINTER
_sig("ro_last_error", ctypes.c_char_p, [])
_sig("ro_volume_create", c_i32, [_P(VolumeDesc), _P(c_vp)])
_sig("ro_volume_destroy", None, [c_vp])
_sig("ro_volume_levels", c_i32, [c_vp, c_vp, c_vp, c_vp])
_sig("ro_volume_brick_count", c_i32, [c_vp, _P(c_u64)])
_sig("ro_brick_id_encode", c_i32, [c_vp, c_u32, c_u32, _P(c_u32 * 3), _P(c_u32)])
_sig("ro_brick_id_decode", c_i32, [c_vp, c_u32, _P(c_u32), _P(c_u32), _P(c_u32 * 3)])
_sig("ro_cache_query", c_i32, [c_vp, _P(CacheDesc), _P(CacheSizes)])
_sig("ro_cache_create", c_i32, [c_vp, _P(CacheDesc), _P(CacheBuffers), c_vp, _P(c_vp)])
_sig("ro_cache_destroy", None, [c_vp])
_sig("ro_stream_bricks", c_i32, [c_vp, c_u32, c_u32, c_vp, c_vp, c_vp, c_vp])
_sig("ro_read_requests", c_i32, [c_vp, c_u32, c_vp, c_vp, _P(c_u32), _P(c_u64), c_vp])
_sig("ro_read_requests_noalloc", c_i32, [c_vp, c_u32, c_vp, c_vp, _P(c_u32), _P(c_u64), c_vp])
_sig("ro_read_usage", c_i32, [c_vp, c_u32, c_u32, c_vp, _P(c_u32), c_vp])
_sig("ro_cache_evict_channel", c_i32, [c_vp, c_u32, c_vp])
_sig("ro_cache_set_channel_map", c_i32, [c_vp, c_u32, c_u32])
_sig("ro_cache_get_channel_map", c_i32, [c_vp, c_vp])
_sig("ro_cache_source_bricks", c_i32, [c_vp, c_u32, c_vp, c_vp])
_sig("ro_cache_page_table_host", c_i32, [c_vp, c_vp, c_u64])
_sig("ro_cache_state_size", c_i32, [c_vp, _P(c_sz)])
_sig("ro_cache_save_state", c_i32, [c_vp, c_vp, c_sz])
_sig("ro_cache_load_state", c_i32, [c_vp, c_vp, c_sz])
_sig("ro_octree_query", c_i32, [c_vp, _P(OctreeDesc), _P(OctreeSizes)])
_sig("ro_octree_create", c_i32, [c_vp, _P(OctreeDesc), _P(OctreeBuffers), c_vp, _P(c_vp)])
_sig("ro_octree_destroy", None, [c_vp])
_sig("ro_octree_set_leaf_metadata", c_i32, [c_vp, c_u32, c_vp, c_vp])
_sig("ro_octree_leaf_metadata_from_bricks", c_i32, [c_vp, c_u32, c_vp, c_vp])
_sig("ro_octree_set_leaf_unknown", c_i32, [c_vp, c_u32, c_vp])
_sig("ro_update_residency", c_i32, [c_vp, c_vp])
_sig("ro_rebuild_residency", c_i32, [c_vp, c_vp])
_sig("ro_render", c_i32, [c_vp, _P(FrameDesc), c_vp, c_vp])
_sig("ro_snapshot_size", c_i32, [c_vp, c_u32, _P(c_sz)])
_sig("ro_snapshot", c_i32, [c_vp, c_u32, c_vp, c_sz, _P(c_sz), c_vp])
_sig("ro_restore", c_i32, [c_vp, c_vp, c_sz, c_vp])
_sig("ro_mlp_query", c_i32, [_P(c_sz), _P(c_sz)])
_sig("ro_mlp_create", c_i32, [c_vp, c_vp, _P(c_vp)])
_sig("ro_mlp_destroy", None, [c_vp])
_sig("ro_mlp_set_weights", c_i32, [c_vp, c_vp, c_vp])
_sig("ro_mlp_get_weights", c_i32, [c_vp, c_vp, c_vp])
_sig("ro_mlp_forward", c_i32, [c_vp, c_vp, c_u32, c_vp, c_vp])
_sig("ro_mlp_gradients", c_i32, [c_vp, c_vp, c_vp, c_vp, c_u32, c_vp, c_vp, c_vp])
_sig("ro_mlp_train_step", c_i32, [c_vp, c_vp, c_vp, c_vp, c_u32, ctypes.c_float, c_vp, c_vp])


class ResoctError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.ro_last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _check(code, where):
    if code != 0:
        raise ResoctError(code, where)


def last_error() -> str:
    return _lib.ro_last_error().decode(errors="replace")


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_vp(stream.cuda_stream)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(c_vp)


def _dev_ptr(t: torch.Tensor):
    return c_vp(t.data_ptr())


def _alloc(nbytes: int, device) -> torch.Tensor:
    # 256-byte aligned: the caching allocator returns 512-byte aligned blocks
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Volume:
    def __init__(self, dims, spacing, n_channels, bytes_per_voxel, brick, n_levels):
        d = VolumeDesc()
        d.dims[:] = [int(x) for x in dims]
        d.spacing[:] = [float(x) for x in spacing]
        d.n_channels, d.bytes_per_voxel, d.brick, d.n_levels = n_channels, bytes_per_voxel, brick, n_levels
        h = c_vp()
        _check(_lib.ro_volume_create(ctypes.byref(d), ctypes.byref(h)), "ro_volume_create")
        self.h = h
        self.desc = d
        self.n_channels, self.n_levels, self.brick = n_channels, n_levels, brick
        self.bytes_per_voxel = bytes_per_voxel
        self.dims = tuple(int(x) for x in dims)

    def __del__(self, _destroy=_lib.ro_volume_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def levels(self):
        L = self.n_levels
        d = np.zeros((L, 3), np.int32)
        f = np.zeros((L, 3), np.int32)
        nb = np.zeros((L, 3), np.int32)
        _check(_lib.ro_volume_levels(self.h, _np_ptr(d), _np_ptr(f), _np_ptr(nb)), "ro_volume_levels")
        return d, f, nb

    def brick_count(self) -> int:
        n = c_u64()
        _check(_lib.ro_volume_brick_count(self.h, ctypes.byref(n)), "ro_volume_brick_count")
        return int(n.value)

    def encode(self, c, l, b) -> int:
        arr = (c_u32 * 3)(*[int(x) for x in b])
        out = c_u32()
        _check(_lib.ro_brick_id_encode(self.h, c, l, ctypes.byref(arr), ctypes.byref(out)),
               "ro_brick_id_encode")
        return int(out.value)

    def decode(self, id_):
        c, l, b = c_u32(), c_u32(), (c_u32 * 3)()
        _check(_lib.ro_brick_id_decode(self.h, id_, ctypes.byref(c), ctypes.byref(l), ctypes.byref(b)),
               "ro_brick_id_decode")
        return int(c.value), int(l.value), tuple(int(x) for x in b)


class Cache:
    def __init__(self, vol: Volume, n_slots: int, max_batch: int, device="cuda", stream=None, slots=None):
        """slots: optionally the caller's device buffer for the slot pool (a
        contiguous uint8 tensor of at least the queried size, 256-byte
        aligned); the other buffers are allocated here."""
        self.vol = vol
        d = CacheDesc(n_slots, max_batch)
        sz = CacheSizes()
        _check(_lib.ro_cache_query(vol.h, ctypes.byref(d), ctypes.byref(sz)), "ro_cache_query")
        self.sizes = sz
        self.slot_stride = int(sz.slot_stride)
        self.n_slots, self.max_batch = n_slots, max_batch
        self.t = {name: _alloc(getattr(sz, name), device) for name in
                  ("page_table", "counters", "slot_brick", "stamps", "seqs", "scratch")}
        if slots is None:
            self.t["slots"] = _alloc(sz.slots, device)
        else:
            if (slots.dtype != torch.uint8 or not slots.is_cuda or not slots.is_contiguous()
                    or slots.numel() < int(sz.slots) or slots.data_ptr() % 256):
                raise ValueError(f"slots: a contiguous uint8 device tensor of at least {int(sz.slots)} bytes, "
                                 "256-byte aligned")
            self.t["slots"] = slots
        b = CacheBuffers(*[self.t[n].data_ptr() for n in
                           ("slots", "page_table", "counters", "slot_brick", "stamps", "seqs", "scratch")])
        h = c_vp()
        _check(_lib.ro_cache_create(vol.h, ctypes.byref(d), ctypes.byref(b), _stream(stream),
                                    ctypes.byref(h)), "ro_cache_create")
        self.h = h
        self.n_bricks = vol.brick_count()

    def __del__(self, _destroy=_lib.ro_cache_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def staging(self, n: int, device="cuda") -> torch.Tensor:
        return torch.zeros(max(n, 1) * self.slot_stride, dtype=torch.uint8, device=device)

    def stream_bricks(self, frame: int, ids, staged: torch.Tensor, stream=None) -> np.ndarray:
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        n = len(ids)
        flags = np.zeros(max(n, 1), np.uint8)
        if n:
            assert staged.numel() >= n * self.slot_stride
        _check(_lib.ro_stream_bricks(self.h, frame, n, _np_ptr(ids), _dev_ptr(staged) if n else None,
                                     _np_ptr(flags), _stream(stream)), "ro_stream_bricks")
        return flags[:n]

    def _pinned(self, name: str, n: int) -> np.ndarray:
        """A reusable page-locked uint32 host buffer of at least n entries (the
        device-to-host copies of the readbacks then need no staging)."""
        buf = getattr(self, name, None)
        if buf is None or buf.numel() < n:
            buf = torch.empty(max(n, 1), dtype=torch.int32, pin_memory=True)
            setattr(self, name, buf)
        return buf.numpy().view(np.uint32)

    def read_requests(self, cap: int, stream=None):
        ids = self._pinned("_rq_ids", cap)
        cnt = self._pinned("_rq_cnt", cap)
        nu, tot = c_u32(), c_u64()
        _check(_lib.ro_read_requests(self.h, cap, _np_ptr(ids), _np_ptr(cnt), ctypes.byref(nu),
                                     ctypes.byref(tot), _stream(stream)), "ro_read_requests")
        k = min(cap, nu.value)
        return ids[:k].copy(), cnt[:k].copy(), int(nu.value), int(tot.value)

    def read_requests_noalloc(self, cap: int, stream=None):
        """ro_read_requests_noalloc: the same readback with the library's fixed work space."""
        ids = np.zeros(max(cap, 1), np.uint32)
        cnt = np.zeros(max(cap, 1), np.uint32)
        nu, tot = c_u32(), c_u64()
        _check(_lib.ro_read_requests_noalloc(self.h, cap, _np_ptr(ids), _np_ptr(cnt), ctypes.byref(nu),
                                             ctypes.byref(tot), _stream(stream)), "ro_read_requests_noalloc")
        k = min(cap, nu.value)
        return ids[:k], cnt[:k], int(nu.value), int(tot.value)

    def read_usage(self, frame: int, cap: int = None, stream=None):
        cap = self.n_slots if cap is None else cap
        out = self._pinned("_us_out", cap)
        n = c_u32()
        _check(_lib.ro_read_usage(self.h, frame, cap, _np_ptr(out), ctypes.byref(n), _stream(stream)),
               "ro_read_usage")
        return out[:min(cap, n.value)].copy(), int(n.value)

    def save_state(self) -> np.ndarray:
        n = c_sz()
        _check(_lib.ro_cache_state_size(self.h, ctypes.byref(n)), "ro_cache_state_size")
        blob = np.zeros(n.value, np.uint8)
        _check(_lib.ro_cache_save_state(self.h, _np_ptr(blob), n.value), "ro_cache_save_state")
        return blob

    def load_state(self, blob: np.ndarray):
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(_lib.ro_cache_load_state(self.h, _np_ptr(blob), blob.size), "ro_cache_load_state")

    def evict_channel(self, channel: int, stream=None):
        _check(_lib.ro_cache_evict_channel(self.h, channel, _stream(stream)), "ro_cache_evict_channel")

    def set_channel_map(self, cache_channel: int, source_channel: int):
        _check(_lib.ro_cache_set_channel_map(self.h, cache_channel, source_channel), "ro_cache_set_channel_map")

    def channel_map(self) -> list:
        out = np.zeros(self.vol.n_channels, np.uint32)
        _check(_lib.ro_cache_get_channel_map(self.h, _np_ptr(out)), "ro_cache_get_channel_map")
        return [int(x) for x in out]

    def source_bricks(self, ids) -> np.ndarray:
        """[n][5] (source channel, level, bx, by, bz) of brick IDs."""
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        out = np.zeros((max(len(ids), 1), 5), np.uint32)
        _check(_lib.ro_cache_source_bricks(self.h, len(ids), _np_ptr(ids), _np_ptr(out)), "ro_cache_source_bricks")
        return out[:len(ids)]

    def page_table_host(self) -> np.ndarray:
        out = np.zeros(self.n_bricks, np.uint32)
        _check(_lib.ro_cache_page_table_host(self.h, _np_ptr(out), self.n_bricks),
               "ro_cache_page_table_host")
        return out


class Octree:
    def __init__(self, cache: Cache, leaf, depth, start_level=0, device="cuda", stream=None):
        self.cache = cache
        d = OctreeDesc()
        d.leaf[:] = [int(x) for x in leaf]
        d.depth, d.start_level = depth, start_level
        sz = OctreeSizes()
        _check(_lib.ro_octree_query(cache.vol.h, ctypes.byref(d), ctypes.byref(sz)), "ro_octree_query")
        self.sizes = sz
        self.n_nodes, self.n_leaves = int(sz.n_nodes), int(sz.n_leaves)
        self.leaf_grid = tuple(int(x) for x in sz.leaf_grid)
        names = ("node_meta", "node_mask", "node_flags", "scratch", "leaf_level")
        self.t = {name: _alloc(getattr(sz, name), device) for name in names}
        b = OctreeBuffers(*[self.t[n].data_ptr() for n in names])
        h = c_vp()
        _check(_lib.ro_octree_create(cache.h, ctypes.byref(d), ctypes.byref(b), _stream(stream),
                                     ctypes.byref(h)), "ro_octree_create")
        self.h = h
        self.depth = depth

    def __del__(self, _destroy=_lib.ro_octree_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def set_leaf_metadata(self, channel: int, leaf_mm: torch.Tensor, stream=None):
        assert leaf_mm.dtype == torch.uint16 and leaf_mm.is_contiguous()
        assert leaf_mm.numel() == 2 * self.n_leaves
        _check(_lib.ro_octree_set_leaf_metadata(self.h, channel, _dev_ptr(leaf_mm), _stream(stream)),
               "ro_octree_set_leaf_metadata")

    def set_leaf_unknown(self, channel: int, stream=None):
        _check(_lib.ro_octree_set_leaf_unknown(self.h, channel, _stream(stream)), "ro_octree_set_leaf_unknown")

    def leaf_levels(self) -> np.ndarray:
        """Metadata level of every leaf and channel, [n_leaves][m] (255 unknown)."""
        torch.cuda.current_stream().synchronize()
        m = self.cache.vol.n_channels
        return self.t["leaf_level"][: self.n_leaves * m].cpu().numpy().reshape(self.n_leaves, m)

    def leaf_metadata_from_bricks(self, ids, stream=None):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        _check(_lib.ro_octree_leaf_metadata_from_bricks(self.h, len(ids), _np_ptr(ids),
                                                        _stream(stream)),
               "ro_octree_leaf_metadata_from_bricks")

    def snapshot(self, slots: bool = False, stream=None) -> np.ndarray:
        """ro_snapshot: the octree's and its cache's state as a host blob."""
        flags = SNAPSHOT_SLOTS if slots else 0
        n, used = c_sz(), c_sz()
        _check(_lib.ro_snapshot_size(self.h, flags, ctypes.byref(n)), "ro_snapshot_size")
        blob = np.empty(n.value, np.uint8)
        _check(_lib.ro_snapshot(self.h, flags, _np_ptr(blob), n.value, ctypes.byref(used), _stream(stream)),
               "ro_snapshot")
        return blob[:used.value]

    def restore(self, blob: np.ndarray, stream=None):
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(_lib.ro_restore(self.h, _np_ptr(blob), blob.size, _stream(stream)), "ro_restore")

    def update_residency(self, stream=None):
        _check(_lib.ro_update_residency(self.h, _stream(stream)), "ro_update_residency")

    def rebuild_residency(self, stream=None):
        _check(_lib.ro_rebuild_residency(self.h, _stream(stream)), "ro_rebuild_residency")

    def masks(self) -> np.ndarray:
        m = self.cache.vol.n_channels
        return self.t["node_mask"][:2 * self.n_nodes * m].view(torch.int16).cpu().numpy() \
            .view(np.uint16).reshape(self.n_nodes, m)

    def meta(self) -> np.ndarray:
        m = self.cache.vol.n_channels
        a = self.t["node_meta"][:4 * self.n_nodes * m].view(torch.int32).cpu().numpy().view(np.uint32)
        a = a.reshape(self.n_nodes, m)
        return np.stack([a & 0xFFFF, a >> 16], axis=-1).astype(np.uint16)

    def render(self, fd: FrameDesc, rgba: torch.Tensor, stream=None):
        assert rgba.dtype == torch.float32 and rgba.is_contiguous()
        assert rgba.numel() >= 4 * fd.width * fd.height
        _check(_lib.ro_render(self.h, ctypes.byref(fd), _dev_ptr(rgba), _stream(stream)), "ro_render")


def frame_desc(frame: int, cam: dict, W: int, H: int, step: float, channels: list, tf_dev: torch.Tensor,
               n_levels: int, term_alpha=0.99, lod_bias=1.0, start_level=-1, flags=0,
               aov: torch.Tensor = None, stats: torch.Tensor = None, bricks: torch.Tensor = None,
               nodes: torch.Tensor = None):
    """channels: list of {c, lo, hi, W0, W1} in visible-slot order (lo / hi
    default to the full level range); tf_dev is a device float32 tensor
    [n_vis][256][4] in the same order."""
    fd = FrameDesc()
    fd.frame = frame
    fd.projection = PROJ_ORTHO if cam["proj"] == "ortho" else PROJ_PERSP
    fd.eye[:] = cam["eye"]
    fd.forward[:] = cam["F"]
    fd.right[:] = cam["R"]
    fd.up[:] = cam["U"]
    fd.tx, fd.ty = cam["tx"], cam["ty"]
    fd.width, fd.height = W, H
    fd.step, fd.lod_bias = step, lod_bias
    fd.n_vis = len(channels)
    for j, ch in enumerate(channels):
        fd.vis[j] = ch["c"]
        fd.lod_lo[j] = ch.get("lo", 0)
        fd.lod_hi[j] = ch.get("hi", n_levels - 1)
        fd.win_lo[j], fd.win_hi[j] = ch["W0"], ch["W1"]
    assert tf_dev.dtype == torch.float32 and tf_dev.is_contiguous()
    assert tf_dev.numel() >= len(channels) * 1024
    fd.tf_dev = tf_dev.data_ptr()
    fd.term_alpha = term_alpha
    fd.start_level = start_level
    fd.flags = flags | (RENDER_AOV if aov is not None else 0) | (RENDER_BRICKS if bricks is not None else 0)
    fd.aov_dev = aov.data_ptr() if aov is not None else None
    if bricks is not None:
        assert bricks.dtype == torch.int32 and bricks.numel() >= W * H * (1 + len(channels))
    fd.bricks_dev = bricks.data_ptr() if bricks is not None else None
    fd.flags |= RENDER_NODES if nodes is not None else 0
    fd.nodes_dev = nodes.data_ptr() if nodes is not None else None
    fd.stats_dev = stats.data_ptr() if stats is not None else None
    return fd


MLP_KEYS = (("W1", (24, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 9)), ("b3", (9,)))


def _pack_weights(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float32).reshape(-1) for k, _ in MLP_KEYS])


def _unpack_weights(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for k, shp in MLP_KEYS:
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp).copy()
        o += n
    return out


class Mlp:
    """The request predictor's parameters and optimiser state on the device."""

    def __init__(self, device="cuda"):
        pb, wb = c_sz(), c_sz()
        _check(_lib.ro_mlp_query(ctypes.byref(pb), ctypes.byref(wb)), "ro_mlp_query")
        self.params = _alloc(pb.value, device)
        self.work = _alloc(wb.value, device)
        h = c_vp()
        _check(_lib.ro_mlp_create(_dev_ptr(self.params), _dev_ptr(self.work), ctypes.byref(h)), "ro_mlp_create")
        self.h = h

    def __del__(self, _destroy=_lib.ro_mlp_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def set_weights(self, p: dict, stream=None):
        flat = np.ascontiguousarray(_pack_weights(p))
        _check(_lib.ro_mlp_set_weights(self.h, _np_ptr(flat), _stream(stream)), "ro_mlp_set_weights")

    def get_weights(self, stream=None) -> dict:
        flat = np.zeros(sum(int(np.prod(s)) for _, s in MLP_KEYS), np.float32)
        _check(_lib.ro_mlp_get_weights(self.h, _np_ptr(flat), _stream(stream)), "ro_mlp_get_weights")
        return _unpack_weights(flat)

    def forward(self, x: torch.Tensor, z: torch.Tensor = None, stream=None) -> torch.Tensor:
        assert x.dtype == torch.float16 and x.is_contiguous() and x.shape[1] == 32
        rows = x.shape[0]
        z = torch.empty((rows, 16), dtype=torch.float32, device=x.device) if z is None else z
        _check(_lib.ro_mlp_forward(self.h, _dev_ptr(x), rows, _dev_ptr(z), _stream(stream)), "ro_mlp_forward")
        return z

    def gradients(self, x, y, mask, stream=None):
        flat = np.zeros(sum(int(np.prod(s)) for _, s in MLP_KEYS), np.float32)
        loss = ctypes.c_float()
        _check(_lib.ro_mlp_gradients(self.h, _dev_ptr(x), _dev_ptr(y), _dev_ptr(mask), x.shape[0], _np_ptr(flat),
                                     ctypes.byref(loss), _stream(stream)), "ro_mlp_gradients")
        return _unpack_weights(flat), float(loss.value)

    def train_step(self, x, y, mask, lr: float, want_loss=False, stream=None):
        loss = ctypes.c_float()
        _check(_lib.ro_mlp_train_step(self.h, _dev_ptr(x), _dev_ptr(y), _dev_ptr(mask), x.shape[0], lr,
                                      ctypes.byref(loss) if want_loss else None, _stream(stream)),
               "ro_mlp_train_step")
        return float(loss.value) if want_loss else None


_sig("ro_pf_query", c_i32, [c_vp, _P(c_u32), _P(c_sz), _P(c_sz)])
_sig("ro_pf_create", c_i32, [c_vp, c_vp, c_vp, c_vp, _P(c_vp)])
_sig("ro_pf_destroy", None, [c_vp])
_sig("ro_pf_record", c_i32, [c_vp, c_u32, c_vp])
_sig("ro_pf_features", c_i32, [c_vp, _P(FrameDesc), c_vp, c_vp])
_sig("ro_pf_labels", c_i32, [c_vp, c_vp, c_vp, c_vp])
_sig("ro_pf_candidates", c_i32, [c_vp, c_vp, ctypes.c_float, c_u32, c_vp, c_vp, _P(c_u32), c_vp])


class PrefetchRows:
    """Predictor rows, brick history and candidate scores of one octree."""

    def __init__(self, tree: Octree, device="cuda", stream=None):
        rows, hb, sb = c_u32(), c_sz(), c_sz()
        _check(_lib.ro_pf_query(tree.h, ctypes.byref(rows), ctypes.byref(hb), ctypes.byref(sb)), "ro_pf_query")
        self.rows = int(rows.value)
        self.hist = _alloc(hb.value, device)
        self.score = _alloc(sb.value, device)
        h = c_vp()
        _check(_lib.ro_pf_create(tree.h, _dev_ptr(self.hist), _dev_ptr(self.score), _stream(stream),
                                 ctypes.byref(h)), "ro_pf_create")
        self.h = h
        self.tree = tree

    def __del__(self, _destroy=_lib.ro_pf_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def record(self, frame: int, stream=None):
        _check(_lib.ro_pf_record(self.h, frame, _stream(stream)), "ro_pf_record")

    def features(self, fd: FrameDesc, x: torch.Tensor, stream=None):
        assert x.dtype == torch.float16 and x.shape == (self.rows, 32)
        _check(_lib.ro_pf_features(self.h, ctypes.byref(fd), _dev_ptr(x), _stream(stream)), "ro_pf_features")

    def labels(self, y: torch.Tensor, mask: torch.Tensor, stream=None):
        assert y.shape == (self.rows, 16) and mask.shape == (self.rows, 16)
        _check(_lib.ro_pf_labels(self.h, _dev_ptr(y), _dev_ptr(mask), _stream(stream)), "ro_pf_labels")

    def candidates(self, z: torch.Tensor, threshold=0.5, cap=1 << 16, stream=None):
        ids = np.zeros(max(cap, 1), np.uint32)
        pr = np.zeros(max(cap, 1), np.float32)
        n = c_u32()
        _check(_lib.ro_pf_candidates(self.h, _dev_ptr(z), threshold, cap, _np_ptr(ids), _np_ptr(pr), ctypes.byref(n),
                                     _stream(stream)), "ro_pf_candidates")
        k = min(cap, n.value)
        return ids[:k], pr[:k]


SERVE_GRAPH = 1
_sig("ro_serve_query", c_i32, [c_u32, c_u32, _P(c_sz)])
_sig("ro_serve_create", c_i32, [c_vp, c_u32, c_u32, c_vp, _P(c_vp)])
_sig("ro_serve_destroy", None, [c_vp])
_sig("ro_serve_prepare", c_i32, [c_vp, c_u32, c_vp, c_vp, c_i32])
_sig("ro_serve_submit", c_i32, [c_vp, c_u32, _P(c_u64)])
_sig("ro_serve_poll", c_i32, [c_vp, c_u64, _P(c_i32)])
_sig("ro_serve_wait", c_i32, [c_vp, c_u64])
_sig("ro_serve_work_items", c_i32, [c_i32, c_i32, _P(c_u32)])
_sig("ro_serve_request_done", c_i32, [c_vp, c_u64, c_u32, _P(c_i32)])
_sig("ro_serve_enqueue", c_i32, [c_vp, c_vp, c_vp, _P(c_u64)])
_sig("ro_serve_done", c_i32, [c_vp, c_u64, _P(c_i32)])
_sig("ro_serve_drain", c_i32, [c_vp])
E_CAPACITY = -2


def serve_work_items(W: int, H: int) -> int:
    """Work items (queue entries) a W x H request takes in a serving batch."""
    n = c_u32()
    _check(_lib.ro_serve_work_items(W, H, ctypes.byref(n)), "ro_serve_work_items")
    return int(n.value)


class Server:
    """Batched multi-request rendering over one octree (persistent tile-queue
    kernel, two alternating batch halves with their own streams)."""

    def __init__(self, tree: Octree, max_requests=64, max_tiles=1 << 16, device="cuda"):
        nb = c_sz()
        _check(_lib.ro_serve_query(max_requests, max_tiles, ctypes.byref(nb)), "ro_serve_query")
        self.buf = _alloc(nb.value, device)
        h = c_vp()
        _check(_lib.ro_serve_create(tree.h, max_requests, max_tiles, _dev_ptr(self.buf), ctypes.byref(h)),
               "ro_serve_create")
        self.h = h
        self.tree = tree
        self.max_requests, self.max_tiles = max_requests, max_tiles

    def __del__(self, _destroy=_lib.ro_serve_destroy):
        # bound when the class is created: module globals may be gone at interpreter exit
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def prepare(self, fds, outs, full_channels=False):
        n = len(fds)
        assert n == len(outs) and n >= 1
        for fd, o in zip(fds, outs):
            assert o.dtype == torch.float32 and o.is_contiguous() and o.numel() >= 4 * fd.width * fd.height
        arr = (FrameDesc * n)(*fds)
        ptrs = (c_vp * n)(*[o.data_ptr() for o in outs])
        _check(_lib.ro_serve_prepare(self.h, n, ctypes.cast(arr, c_vp), ctypes.cast(ptrs, c_vp),
                                     1 if full_channels else 0), "ro_serve_prepare")

    def submit(self, graph=False) -> int:
        t = c_u64()
        _check(_lib.ro_serve_submit(self.h, SERVE_GRAPH if graph else 0, ctypes.byref(t)), "ro_serve_submit")
        return int(t.value)

    def launch(self, fds, outs, graph=False) -> int:
        self.prepare(fds, outs, full_channels=graph)
        return self.submit(graph)

    def poll(self, ticket: int) -> bool:
        d = c_i32()
        _check(_lib.ro_serve_poll(self.h, ticket, ctypes.byref(d)), "ro_serve_poll")
        return bool(d.value)

    def wait(self, ticket: int):
        _check(_lib.ro_serve_wait(self.h, ticket), "ro_serve_wait")

    def request_done(self, ticket: int, r: int) -> bool:
        d = c_i32()
        _check(_lib.ro_serve_request_done(self.h, ticket, r, ctypes.byref(d)), "ro_serve_request_done")
        return bool(d.value)

    def enqueue(self, fd, out):
        """Continuous admission of one request; its ticket, or None when
        every request slot is busy or the ring is full (nothing admitted)."""
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= 4 * fd.width * fd.height
        t = c_u64()
        code = _lib.ro_serve_enqueue(self.h, ctypes.byref(fd), _dev_ptr(out), ctypes.byref(t))
        if code == E_CAPACITY:
            return None
        _check(code, "ro_serve_enqueue")
        return int(t.value)

    def done(self, ticket: int) -> bool:
        d = c_i32()
        _check(_lib.ro_serve_done(self.h, ticket, ctypes.byref(d)), "ro_serve_done")
        return bool(d.value)

    def drain(self):
        _check(_lib.ro_serve_drain(self.h), "ro_serve_drain")
