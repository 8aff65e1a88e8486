"""CPU oracle for the residency-octree hot path (test infrastructure).

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  It loads liboracle.so (plain C, FP64, built with gcc from
oracle.c) and the numpy MLP reference in oracle/mlp.py.  It never touches the
GPU library.

Conventions shared with every caller (they are properties of the inputs, not
of any implementation): brick IDs (c*k + l) << 24 | bz << 16 | by << 8 | bx;
transfer-function windows as raw values in 24.8 fixed point; cameras given by
eye, forward, right, up and the two half extents (ortho) or half-angle
tangents (perspective); leaf metadata per channel as [n_leaves][2] uint16 over
the padded leaf grid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
MAXC = 16
MAXL = 16


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Volume(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 3), ("spacing", ctypes.c_double * 3),
                ("n_channels", ctypes.c_int), ("bits", ctypes.c_int), ("B", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("leaf", ctypes.c_int * 3), ("depth", ctypes.c_int)]


class Frame(ctypes.Structure):
    _fields_ = [("proj", ctypes.c_int), ("eye", ctypes.c_double * 3), ("F", ctypes.c_double * 3),
                ("R", ctypes.c_double * 3), ("U", ctypes.c_double * 3), ("tx", ctypes.c_double),
                ("ty", ctypes.c_double), ("W", ctypes.c_int), ("H", ctypes.c_int),
                ("delta", ctypes.c_double), ("lod_bias", ctypes.c_double), ("nvis", ctypes.c_int),
                ("vis", ctypes.c_int * MAXC), ("lod_lo", ctypes.c_int * MAXC),
                ("lod_hi", ctypes.c_int * MAXC), ("W0", ctypes.c_uint32 * MAXC),
                ("W1", ctypes.c_uint32 * MAXC), ("tf", ctypes.c_void_p * MAXC),
                ("term_alpha", ctypes.c_double), ("term_margin", ctypes.c_double), ("adaptive", ctypes.c_int),
                ("homogeneous", ctypes.c_int), ("channel_rates", ctypes.c_int),
                ("traversal_depth", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_longlong), ("channel_samples", ctypes.c_longlong),
                ("missing", ctypes.c_longlong), ("amb_samples", ctypes.c_longlong),
                ("amb_pixels", ctypes.c_longlong)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, ci, cll = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong
        PV = ctypes.POINTER(Volume)
        L.or_level_info.restype = ci
        L.or_level_info.argtypes = [PV, vp, vp, vp]
        L.or_brick_count.restype = cll
        L.or_brick_count.argtypes = [PV]
        L.or_brick_id.restype = ctypes.c_uint32
        L.or_brick_id.argtypes = [ci] * 6
        L.or_brick_id_decode.restype = None
        L.or_brick_id_decode.argtypes = [ci, ctypes.c_uint32, vp, vp, vp, vp, vp]
        L.or_dense_ids.restype = ci
        L.or_dense_ids.argtypes = [PV, vp]
        L.or_node_count.restype = cll
        L.or_node_count.argtypes = [PV, vp, vp]
        L.or_meta_all.restype = ci
        L.or_meta_all.argtypes = [PV, vp, vp]
        L.or_masks.restype = ci
        L.or_masks.argtypes = [PV, vp, vp]
        L.or_tf_empty.restype = ci
        L.or_tf_empty.argtypes = [ctypes.c_uint32] * 4 + [vp]
        L.or_render.restype = ci
        L.or_render.argtypes = [PV, vp, vp, vp, vp, vp, ctypes.POINTER(Frame), ci, ci, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp, vp, ctypes.POINTER(Stats), ci]
        L.or_brute.restype = ci
        L.or_brute.argtypes = [PV, vp, ci, ctypes.POINTER(Frame), vp]
        L.or_plain_policy.restype = ci
        L.or_plain_policy.argtypes = [cll, vp, vp, vp, ci, vp]
        L.or_stream.restype = ci
        L.or_stream.argtypes = [cll, ci, vp, vp, vp, vp, vp, ctypes.c_uint32, ci, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_volume(dims, spacing, n_channels, bits, B, n_levels, leaf, depth) -> Volume:
    v = Volume()
    v.dims[:] = [int(x) for x in dims]
    v.spacing[:] = [float(x) for x in spacing]
    v.n_channels, v.bits, v.B, v.n_levels, v.depth = n_channels, bits, B, n_levels, depth
    v.leaf[:] = [int(x) for x in leaf]
    return v


def level_info(V: Volume):
    L = V.n_levels
    d = np.zeros((L, 3), np.int32)
    f = np.zeros((L, 3), np.int32)
    nb = np.zeros((L, 3), np.int32)
    assert lib().or_level_info(ctypes.byref(V), _p(d), _p(f), _p(nb)) == 0
    return d, f, nb


def brick_count(V: Volume) -> int:
    return int(lib().or_brick_count(ctypes.byref(V)))


def dense_ids(V: Volume) -> np.ndarray:
    out = np.zeros(brick_count(V), np.uint32)
    lib().or_dense_ids(ctypes.byref(V), _p(out))
    return out


def brick_id(n_levels, c, l, bx, by, bz) -> int:
    return int(lib().or_brick_id(n_levels, c, l, bx, by, bz))


def brick_id_decode(n_levels, id_):
    vals = [ctypes.c_int() for _ in range(5)]
    lib().or_brick_id_decode(n_levels, id_, *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)  # c, l, bx, by, bz


def node_count(V: Volume):
    off = np.zeros(V.depth + 2, np.int64)
    n = np.zeros((V.depth + 1, 3), np.int32)
    tot = lib().or_node_count(ctypes.byref(V), _p(off), _p(n))
    if tot < 0:
        raise ValueError("tree does not fit the volume")
    return int(tot), off, n


def meta_all(V: Volume, leaf_mm: np.ndarray) -> np.ndarray:
    """leaf_mm [C][n_leaves][2] -> node metadata [n_nodes][C][2]."""
    tot, _, _ = node_count(V)
    lm = np.ascontiguousarray(leaf_mm, dtype=np.uint16)
    out = np.zeros((tot, V.n_channels, 2), np.uint16)
    assert lib().or_meta_all(ctypes.byref(V), _p(lm), _p(out)) == 0
    return out


def leaf_meta_from_bricks(V: Volume, levels, leaf_mm: np.ndarray, brick_ids, leaf_level=None):
    """Sec. 5.3, metadata computed on the client from fetched brick voxels
    (plain numpy over the definition).  levels[c][l]: level arrays [z][y][x];
    leaf_mm: [C][n_leaves][2] before the call; brick_ids: IDs of the bricks
    whose data are used.  Returns the new leaf metadata: each leaf of the
    padded leaf grid inside a brick's extent gets, for the brick's channel,
    [min, max] of the voxels of the brick's level that overlap the leaf box
    grown by one voxel of that level, clamped to the level's grid ([0, 0] if
    nothing is left).  Bricks are applied coarsest level first, so where
    several cover a leaf the finest level's values stay.  With leaf_level
    ([C][n_leaves], where each leaf's metadata came from: 0 the server or
    level-0 data, l level-l data, 255 unknown) a leaf takes a brick's values
    only when the brick's level is at most its entry, which then becomes the
    brick's level (finer data refine, coarser never replace); the result is
    then (metadata, levels)."""
    d, f, nb = level_info(V)
    _, _, n = node_count(V)
    ng = [int(x) for x in n[V.depth]]
    lf = [int(x) for x in V.leaf]
    out = np.array(leaf_mm, dtype=np.uint16, copy=True)
    lev = None if leaf_level is None else np.array(leaf_level, dtype=np.uint8, copy=True)
    bricks = sorted({brick_id_decode(V.n_levels, int(i)) for i in brick_ids}, key=lambda t: -t[1])
    for c, l, bx, by, bz in bricks:
        arr = levels[c][l]
        b = (bx, by, bz)
        rng = []
        for a in range(3):
            e0 = b[a] * V.B * int(f[l][a])  # the brick's extent in L0 voxels
            e1 = e0 + V.B * int(f[l][a])
            rng.append(range(min(e0 // lf[a], ng[a]), min(e1 // lf[a], ng[a])))
        for lz in rng[2]:
            for ly in rng[1]:
                for lx in rng[0]:
                    box = []
                    for a, li in enumerate((lx, ly, lz)):
                        x0, x1, fa = li * lf[a], (li + 1) * lf[a], int(f[l][a])
                        box.append((max(x0 // fa - 1, 0), min((x1 - 1) // fa + 1, int(d[l][a]) - 1)))
                    k = (lz * ng[1] + ly) * ng[0] + lx
                    if lev is not None:
                        if l > lev[c, k]:
                            continue
                        lev[c, k] = l
                    if any(lo > hi for lo, hi in box):
                        out[c, k] = (0, 0)
                        continue
                    (x0, x1), (y0, y1), (z0, z1) = box
                    sub = arr[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
                    out[c, k] = (sub.min(), sub.max())
    return out if lev is None else (out, lev)


def masks(V: Volume, res_slot: np.ndarray) -> np.ndarray:
    tot, _, _ = node_count(V)
    out = np.zeros((tot, V.n_channels), np.uint16)
    rs = np.ascontiguousarray(res_slot, dtype=np.int32)
    assert lib().or_masks(ctypes.byref(V), _p(rs), _p(out)) == 0
    return out


def tf_empty(mn, mx, W0, W1, tf) -> bool:
    t = np.ascontiguousarray(tf, dtype=np.float32)
    return bool(lib().or_tf_empty(mn, mx, W0, W1, _p(t)))


def make_frame(cam: dict, W, H, delta, channels: list, term_alpha=0.99, lod_bias=1.0,
               term_margin=1e-5, adaptive=False, homogeneous=False, channel_rates=False, traversal_depth=False):
    """channels: list of dicts {c, lo, hi, W0, W1, tf (256x4 float32)} in
    visible-slot order.  Returns (Frame, keepalive)."""
    fr = Frame()
    fr.proj = 0 if cam["proj"] == "ortho" else 1
    fr.eye[:] = cam["eye"]
    fr.F[:] = cam["F"]
    fr.R[:] = cam["R"]
    fr.U[:] = cam["U"]
    fr.tx, fr.ty = cam["tx"], cam["ty"]
    fr.W, fr.H = W, H
    fr.delta, fr.lod_bias, fr.term_alpha = delta, lod_bias, term_alpha
    fr.term_margin = term_margin
    fr.adaptive = 1 if adaptive else 0
    fr.homogeneous = 1 if homogeneous else 0
    fr.channel_rates = 1 if channel_rates else 0
    fr.traversal_depth = 1 if traversal_depth else 0
    fr.nvis = len(channels)
    keep = []
    for j, ch in enumerate(channels):
        fr.vis[j] = ch["c"]
        fr.lod_lo[j] = ch.get("lo", 0)
        fr.lod_hi[j] = ch.get("hi", MAXL - 1)
        fr.W0[j], fr.W1[j] = ch["W0"], ch["W1"]
        t = np.ascontiguousarray(ch["tf"], dtype=np.float32)
        keep.append(t)
        fr.tf[j] = t.ctypes.data
    return fr, keep


def _level_ptrs(V: Volume, levels):
    """levels[c][l] numpy arrays -> (void* array, keepalive)."""
    arrs = []
    ptrs = (ctypes.c_void_p * (V.n_channels * V.n_levels))()
    for c in range(V.n_channels):
        for l in range(V.n_levels):
            a = levels[c][l]
            if a is None:
                ptrs[c * V.n_levels + l] = None
                continue
            a = np.ascontiguousarray(a)
            arrs.append(a)
            ptrs[c * V.n_levels + l] = a.ctypes.data
    return ptrs, arrs


class Source(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("fetch", ctypes.c_void_p)]


def source_from_generator(gen):
    """Voxel source backed by the generator's region query (for volumes
    too large to hold as level arrays)."""
    import synth
    s = Source()
    s.ctx = gen._ctx
    s.fetch = ctypes.cast(synth.lib().synth_cells_region, ctypes.c_void_p).value
    return s


def render(V: Volume, levels, res_slot, leaf_mm, frame: Frame, n_slots: int, aov=False,
           n_threads=0, source: Source = None, rows=None, boxes=None):
    """O1.  Returns dict with rgba [H][W][4] f64, counts [dense] u32,
    used [slots] u8, amb_pix, amb_counts, amb_used, alt_rgba / alt_pix (the
    other outcome of one early-termination decision within the margin),
    required_bricks [H][W] u32, aov, stats.  With
    `source` (and levels None) voxels come from the generator; `rows`
    = (row0, row1) restricts the frame to a band of rows; `boxes`
    [C][L][6] (origin, size) says that levels[c][l] holds only that window
    of the level (samples outside it read NaN)."""
    W, H = frame.W, frame.H
    nb = brick_count(V)
    rs = np.ascontiguousarray(res_slot, dtype=np.int32)
    # the usage arrays are indexed by slot: cover every slot the resident set names
    n_slots = max(int(n_slots), int(rs.max()) + 1 if rs.size else 0)
    rgba = np.zeros((H, W, 4), np.float64)
    counts = np.zeros(nb, np.uint32)
    used = np.zeros(max(n_slots, 1), np.uint8)
    amb_pix = np.zeros((H, W), np.uint8)
    amb_counts = np.zeros(nb, np.uint32)
    amb_used = np.zeros(max(n_slots, 1), np.uint8)
    alt_rgba = np.zeros((H, W, 4), np.float64)
    alt_pix = np.zeros((H, W), np.uint8)
    reqb = np.zeros((H, W), np.uint32)
    aov_a = np.zeros((H, W, V.n_levels), np.uint32) if aov else None
    if levels is not None:
        ptrs, keep = _level_ptrs(V, levels)
    else:
        ptrs, keep = None, None
    lm = np.ascontiguousarray(leaf_mm, dtype=np.uint16)
    st = Stats()
    r0, r1 = rows if rows is not None else (0, 0)
    bx = None if boxes is None else np.ascontiguousarray(boxes, dtype=np.int32)
    rc = lib().or_render(ctypes.byref(V), ptrs, _p(bx), ctypes.byref(source) if source is not None else None,
                         _p(rs), _p(lm), ctypes.byref(frame), r0, r1, _p(rgba),
                         _p(counts), _p(used), _p(aov_a), _p(amb_pix), _p(amb_counts),
                         _p(amb_used), _p(alt_rgba), _p(alt_pix), _p(reqb), ctypes.byref(st), n_threads)
    assert rc == 0
    return dict(rgba=rgba, counts=counts, used=used[:n_slots], amb_pix=amb_pix,
                amb_counts=amb_counts, amb_used=amb_used[:n_slots], aov=aov_a,
                alt_rgba=alt_rgba, alt_pix=alt_pix, required_bricks=reqb,
                stats=dict(samples=st.samples, channel_samples=st.channel_samples,
                           missing=st.missing, amb_samples=st.amb_samples,
                           amb_pixels=st.amb_pixels))


def brute(V: Volume, levels, lam: int, frame: Frame):
    rgba = np.zeros((frame.H, frame.W, 4), np.float64)
    ptrs, keep = _level_ptrs(V, levels)
    assert lib().or_brute(ctypes.byref(V), ptrs, lam, ctypes.byref(frame), _p(rgba)) == 0
    return rgba


class CacheSim:
    """O3 state: slot contents, LRU stamps and upload sequence numbers."""

    def __init__(self, V: Volume, n_slots: int):
        self.V = V
        self.S = n_slots
        self.total = brick_count(V)
        self.ids = dense_ids(V)
        self.id_to_dense = {int(x): i for i, x in enumerate(self.ids)}
        self.per_channel = self.total // V.n_channels
        self.res_slot = np.full(self.total, -1, np.int32)
        self.slot_brick = np.full(n_slots, -1, np.int64)
        self.stamp = np.zeros(n_slots, np.uint32)
        self.seq = np.zeros(n_slots, np.uint32)
        self.seq_next = ctypes.c_uint32(0)

    def dense_of(self, ids):
        return np.array([self.id_to_dense[int(i)] for i in ids], dtype=np.int64)

    def stream(self, frame_no: int, up_dense):
        up = np.ascontiguousarray(np.asarray(up_dense, dtype=np.int64))
        n = len(up)
        flags = np.zeros(max(n, 1), np.uint8)
        ev = np.zeros(max(n, 1), np.int64)
        so = np.zeros(max(n, 1), np.int32)
        rc = lib().or_stream(self.total, self.S, _p(self.res_slot), _p(self.slot_brick),
                             _p(self.stamp), _p(self.seq), ctypes.byref(self.seq_next),
                             frame_no, n, _p(up), _p(flags), _p(ev), _p(so))
        assert rc == 0
        return flags[:n], ev[:n], so[:n]

    def evict_channel(self, c: int):
        """Sec. 5.2 channel exchange: every resident brick of cache channel c
        leaves the cache and its slot becomes free (dense indices are
        channel-major: channel c owns [c P, (c + 1) P))."""
        for s in range(self.S):
            b = int(self.slot_brick[s])
            if b >= 0 and b // self.per_channel == c:
                self.res_slot[b] = -1
                self.slot_brick[s] = -1

    def touch(self, frame_no: int, used: np.ndarray):
        """Usage recorded by a frame: stamp = frame for every slot read."""
        self.stamp[np.nonzero(used[:self.S])[0]] = frame_no

    def page_table(self):
        """{brick ID: slot} of the resident set."""
        d = np.nonzero(self.res_slot >= 0)[0]
        return {int(self.ids[i]): int(self.res_slot[i]) for i in d}

    def plain_policy(self, counts: np.ndarray, U: int):
        out = np.zeros(max(U, 1), np.int64)
        n = lib().or_plain_policy(self.total, _p(np.ascontiguousarray(counts, dtype=np.uint32)),
                                  _p(self.ids), _p(self.res_slot), U, _p(out))
        assert n >= 0
        return out[:n]
