"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package is the stand-in for the paper's data server (Sec. 4 System
Overview): it produces a bricked multi-resolution multi-channel volume
hierarchy, conservative per-leaf metadata (the server "with metadata
queries"), camera paths and transfer-function tables.  It contains no part of
the rendering method (no page tables, trees, sampling, classification or
compositing); it is imported by the tests, the bench and the smoke check, and
its output bytes feed both sides.

Recipes (all deterministic from the seed):
  * blob volume: sum of Gaussian blobs (sigma 2-6 voxels, amplitude 0.3-1.0)
    plus uniform noise 0.02, clamped to [0,1], rounded to u8/u16; coarser
    levels by a 2x box filter (mean of the existing children, rounded half
    up), halving the axes chosen by the level schedule;
  * cell volume: Poisson-placed ellipsoidal cells (semi-axes U[4,10] voxels,
    density 2e-4 per voxel), shared geometry across channels and
    channel-specific lognormal intensity (mu 7, sigma 1), optionally modulated
    by a low-frequency tissue mask and per-channel gain.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
             os.path.join(_HERE, "synth.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        c_int, c_double, c_u64, c_vp = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
        L.synth_key.restype = c_u64
        L.synth_key.argtypes = [c_u64, c_u64, c_u64]
        L.synth_blobs.restype = c_int
        L.synth_blobs.argtypes = [c_int, c_int, c_int, c_int, c_double, c_double, c_double,
                                  c_double, c_double, c_u64, c_int, c_vp]
        L.synth_downsample.restype = c_int
        L.synth_downsample.argtypes = [c_vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_vp]
        L.synth_cells_create.restype = c_vp
        L.synth_cells_create.argtypes = [c_int, c_int, c_int, c_int, c_double, c_double, c_double,
                                         c_double, c_double, c_u64, c_int, c_double, c_double, c_int]
        L.synth_cells_destroy.argtypes = [c_vp]
        L.synth_cells_region.restype = c_int
        L.synth_cells_region.argtypes = [c_vp, c_vp, c_int, c_int, c_int, c_int, c_int, c_int,
                                         c_int, c_vp, c_vp]
        L.synth_cells_bricks.restype = c_int
        L.synth_cells_bricks.argtypes = [c_vp, c_vp, c_vp, c_int, c_int, c_vp, c_int, c_vp, c_vp]
        L.synth_cells_leaf_max.restype = c_int
        L.synth_cells_leaf_max.argtypes = [c_vp, c_vp, c_vp, c_vp]
        L.synth_cells_count.restype = ctypes.c_longlong
        L.synth_cells_count.argtypes = [c_vp]
        L.synth_tissue.restype = c_double
        L.synth_tissue.argtypes = [c_vp, c_double, c_double]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------- levels

def level_schedule(dims, spacing, n_levels):
    """Per-level dims and per-axis L0 factors.

    Axis a is halved going from level l-1 to l iff its spacing at l-1 is
    below twice the smallest spacing at l-1; halved dims are ceil(n/2).
    Returns (dims_l [L][3], factor_l [L][3], halve_l [L][3])."""
    d = [int(x) for x in dims]
    s = [float(x) for x in spacing]
    f = [1, 1, 1]
    out_d, out_f, out_h = [tuple(d)], [tuple(f)], [(0, 0, 0)]
    for _ in range(1, n_levels):
        m = min(s)
        h = tuple(1 if s[a] < 2 * m else 0 for a in range(3))
        for a in range(3):
            if h[a]:
                d[a] = (d[a] + 1) // 2
                s[a] *= 2
                f[a] *= 2
        out_d.append(tuple(d))
        out_f.append(tuple(f))
        out_h.append(h)
    return out_d, out_f, out_h


def _halo_bricks_from_array(arr: np.ndarray, B: int, coords) -> np.ndarray:
    """Cut (B+2)^3 bricks with a 1-voxel halo from a full level array
    [z][y][x]: voxel indices b*B-1 .. b*B+B per axis, clamped to the array."""
    nz, ny, nx = arr.shape
    out = np.empty((len(coords), B + 2, B + 2, B + 2), dtype=arr.dtype)
    for i, (bx, by, bz) in enumerate(coords):
        zi = np.clip(np.arange(bz * B - 1, bz * B + B + 1), 0, nz - 1)
        yi = np.clip(np.arange(by * B - 1, by * B + B + 1), 0, ny - 1)
        xi = np.clip(np.arange(bx * B - 1, bx * B + B + 1), 0, nx - 1)
        out[i] = arr[np.ix_(zi, yi, xi)]
    return out


class BlobVolume:
    """Small volumes held as full level arrays: levels[c][l] is [z][y][x]."""

    def __init__(self, dims, n_channels=1, bits=8, spacing=(1, 1, 1), n_levels=3,
                 n_blobs=40, sigma=(2.0, 6.0), amp=(0.3, 1.0), noise=0.02, seed=1):
        self.dims = tuple(int(x) for x in dims)
        self.spacing = tuple(float(x) for x in spacing)
        self.n_channels = n_channels
        self.bits = bits
        self.dtype = np.uint8 if bits == 8 else np.uint16
        self.n_levels = n_levels
        self.level_dims, self.level_f, halve = level_schedule(self.dims, self.spacing, n_levels)
        L = lib()
        self.levels = []
        for c in range(n_channels):
            nx, ny, nz = self.dims
            a0 = np.empty((nz, ny, nx), dtype=self.dtype)
            rc = L.synth_blobs(nx, ny, nz, n_blobs, sigma[0], sigma[1], amp[0], amp[1], noise,
                               seed * 1000003 + c, bits, _ptr(a0))
            assert rc == 0
            lv = [a0]
            for l in range(1, n_levels):
                src = lv[-1]
                dx, dy, dz = self.level_dims[l]
                dst = np.empty((dz, dy, dx), dtype=self.dtype)
                h = halve[l]
                rc = L.synth_downsample(_ptr(np.ascontiguousarray(src)), bits, src.shape[2],
                                        src.shape[1], src.shape[0], h[0], h[1], h[2], _ptr(dst))
                assert rc == 0
                lv.append(dst)
            self.levels.append(lv)

    def bricks(self, c, l, coords, B):
        return _halo_bricks_from_array(self.levels[c][l], B, coords)

    def leaf_minmax(self, c, leaf, nleaf):
        """Exact per-leaf [min, max] of the L0 values in the leaf box dilated
        by one voxel on every side, clamped to the volume (the server's
        metadata answer).  Leaves entirely outside the volume get [0, 0]."""
        a = self.levels[c][0]
        nz, ny, nx = a.shape
        lx, ly, lz = leaf
        out = np.zeros((nleaf[2], nleaf[1], nleaf[0], 2), dtype=np.uint16)
        for z in range(nleaf[2]):
            z0, z1 = max(z * lz - 1, 0), min((z + 1) * lz + 1, nz)
            for y in range(nleaf[1]):
                y0, y1 = max(y * ly - 1, 0), min((y + 1) * ly + 1, ny)
                for x in range(nleaf[0]):
                    x0, x1 = max(x * lx - 1, 0), min((x + 1) * lx + 1, nx)
                    if z0 >= z1 or y0 >= y1 or x0 >= x1:
                        continue
                    blk = a[z0:z1, y0:y1, x0:x1]
                    out[z, y, x, 0] = blk.min()
                    out[z, y, x, 1] = blk.max()
        return out.reshape(-1, 2)


class CellVolume:
    """Cell-like tissue volumes produced on demand (any level, any brick)."""

    def __init__(self, dims, n_channels, spacing=(1, 1, 4), n_levels=7, density=2e-4,
                 radius=(4.0, 10.0), mu=7.0, sigma=1.0, seed=2, tissue=False,
                 tissue_feature=2048.0, gain_feature=1024.0, region=64):
        self.dims = tuple(int(x) for x in dims)
        self.spacing = tuple(float(x) for x in spacing)
        self.n_channels = n_channels
        self.bits = 16
        self.dtype = np.uint16
        self.n_levels = n_levels
        self.level_dims, self.level_f, _ = level_schedule(self.dims, self.spacing, n_levels)
        self._ctx = lib().synth_cells_create(self.dims[0], self.dims[1], self.dims[2], n_channels,
                                             density, radius[0], radius[1], mu, sigma, seed,
                                             1 if tissue else 0, tissue_feature, gain_feature,
                                             region)
        if not self._ctx:
            raise ValueError("bad cell volume parameters")

    def __del__(self):
        try:
            if self._ctx:
                lib().synth_cells_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass

    def region(self, l, x0, y0, z0, nx, ny, nz, channels=None):
        ch = np.arange(self.n_channels, dtype=np.int32) if channels is None else \
            np.asarray(channels, dtype=np.int32)
        f = np.asarray(self.level_f[l], dtype=np.int32)
        out = np.empty((len(ch), nz, ny, nx), dtype=np.uint16)
        rc = lib().synth_cells_region(self._ctx, _ptr(f), x0, y0, z0, nx, ny, nz, len(ch),
                                      _ptr(ch), _ptr(out))
        assert rc == 0
        return out

    def level_array(self, c, l):
        d = self.level_dims[l]
        return self.region(l, 0, 0, 0, d[0], d[1], d[2], [c])[0]

    def bricks_multi(self, l, coords, B, channels=None):
        """Halo bricks for all listed channels: [n][nch][B+2]^3."""
        ch = np.arange(self.n_channels, dtype=np.int32) if channels is None else \
            np.asarray(channels, dtype=np.int32)
        co = np.ascontiguousarray(np.asarray(coords, dtype=np.int32).reshape(-1, 3))
        f = np.asarray(self.level_f[l], dtype=np.int32)
        ld = np.asarray(self.level_dims[l], dtype=np.int32)
        out = np.empty((len(co), len(ch), B + 2, B + 2, B + 2), dtype=np.uint16)
        if len(co):
            rc = lib().synth_cells_bricks(self._ctx, _ptr(f), _ptr(ld), B, len(co), _ptr(co),
                                          len(ch), _ptr(ch), _ptr(out))
            assert rc == 0
        return out

    def bricks(self, c, l, coords, B):
        return self.bricks_multi(l, coords, B, [c])[:, 0]

    def leaf_max_all(self, leaf, nleaf):
        """[nch][n_leaves] conservative per-leaf maxima (min is 0)."""
        lf = np.asarray(leaf, dtype=np.int32)
        nl = np.asarray(nleaf, dtype=np.int32)
        out = np.empty((self.n_channels, int(np.prod(nleaf))), dtype=np.uint16)
        rc = lib().synth_cells_leaf_max(self._ctx, _ptr(lf), _ptr(nl), _ptr(out))
        assert rc == 0
        return out

    def leaf_minmax(self, c, leaf, nleaf, _cache={}):
        key = (id(self), tuple(leaf), tuple(nleaf))
        if key not in _cache:
            _cache.clear()
            _cache[key] = self.leaf_max_all(leaf, nleaf)
        mx = _cache[key][c]
        out = np.zeros((mx.size, 2), dtype=np.uint16)
        out[:, 1] = mx
        return out

    def n_cells(self):
        return int(lib().synth_cells_count(self._ctx))


# ---------------------------------------------------------------- cameras

def _norm(v):
    v = np.asarray(v, dtype=np.float64)
    return v / math.sqrt(float(v @ v))


def camera_ortho(center, forward, up, half_w, half_h):
    """Orthographic camera: pixel (i, j) (row 0 = top) has origin
    center + a*half_w*R + b*half_h*U with a = (2i+1-W)/W, b = (H-2j-1)/H and
    direction F."""
    F = _norm(forward)
    R = _norm(np.cross(F, up))
    U = np.cross(R, F)
    return dict(proj="ortho", eye=[float(x) for x in center], F=[float(x) for x in F],
                R=[float(x) for x in R], U=[float(x) for x in U], tx=float(half_w), ty=float(half_h))


def camera_ortho_axis(dims_xy, W, H, z0=-0.25):
    """Axis-aligned orthographic view along +z covering [0,nx) x [0,ny) with
    rays through pixel centres; with power-of-two sizes every sample
    coordinate is a dyadic rational."""
    nx, ny = dims_xy
    return dict(proj="ortho", eye=[nx / 2.0, ny / 2.0, z0], F=[0.0, 0.0, 1.0],
                R=[1.0, 0.0, 0.0], U=[0.0, 1.0, 0.0], tx=nx / 2.0, ty=ny / 2.0)


def camera_persp(eye, target, up, fov_y_deg, aspect):
    """Perspective camera: pixel (i, j) has direction
    normalize(F + a*tx*R + b*ty*U), tx = aspect*tan(fov/2), ty = tan(fov/2)."""
    eye = np.asarray(eye, dtype=np.float64)
    F = _norm(np.asarray(target, dtype=np.float64) - eye)
    R = _norm(np.cross(F, up))
    U = np.cross(R, F)
    ty = math.tan(math.radians(fov_y_deg) / 2.0)
    return dict(proj="persp", eye=[float(x) for x in eye], F=[float(x) for x in F],
                R=[float(x) for x in R], U=[float(x) for x in U], tx=float(aspect * ty), ty=float(ty),
                fov_y=float(math.radians(fov_y_deg)))


def camera_oblique_ortho(dims, spacing, seed, W, H):
    """A seeded oblique orthographic view covering the whole volume."""
    s = np.random.default_rng(seed)
    ext = np.asarray(dims, dtype=np.float64) * np.asarray(spacing, dtype=np.float64)
    c = ext / 2.0
    az, el = s.uniform(0, 2 * math.pi), s.uniform(-1.2, 1.2)
    d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    r = float(np.linalg.norm(ext)) / 2.0
    up = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    return camera_ortho(c - d * (r + 1.0), d, up, r * W / max(W, H), r * H / max(W, H))


def orbit_path(dims, spacing, n_frames, elevation_deg=40.0, az_step_deg=3.0, fov_y_deg=45.0,
               aspect=1.0, az0_deg=0.0):
    """Orbit about the slide normal (+z) around the volume center at a
    radius that fits the bounding sphere in the vertical field of view."""
    ext = np.asarray(dims, dtype=np.float64) * np.asarray(spacing, dtype=np.float64)
    c = ext / 2.0
    rad = float(np.linalg.norm(ext)) / 2.0
    dist = rad / math.sin(math.radians(fov_y_deg) / 2.0)
    el = math.radians(elevation_deg)
    cams = []
    for f in range(n_frames):
        az = math.radians(az0_deg + az_step_deg * f)
        eye = c + dist * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        cams.append(camera_persp(eye, c, [0.0, 0.0, 1.0], fov_y_deg, aspect))
    return cams


def flythrough_path(dims, spacing, n_frames, end_target, d1=60.0, tilt_deg=30.0, fov_y_deg=45.0,
                    aspect=16.0 / 9.0):
    """Zoom from a whole-slide view to a close-up: distance
    D(f) = D0 (D1/D0)^(f/(n-1)), target moving linearly from the slide centre
    to end_target, view direction -z tilted by tilt_deg about the x axis."""
    ext = np.asarray(dims, dtype=np.float64) * np.asarray(spacing, dtype=np.float64)
    c = ext / 2.0
    rad = float(np.linalg.norm(ext)) / 2.0
    d0 = rad / math.sin(math.radians(fov_y_deg) / 2.0)
    tilt = math.radians(tilt_deg)
    back = np.array([0.0, -math.sin(tilt), math.cos(tilt)])  # eye offset direction
    cams = []
    for f in range(n_frames):
        s = f / max(n_frames - 1, 1)
        D = d0 * (d1 / d0) ** s
        tgt = c + (np.asarray(end_target, dtype=np.float64) - c) * s
        cams.append(camera_persp(tgt + D * back, tgt, [0.0, 1.0, 0.0], fov_y_deg, aspect))
    return cams


def random_path(dims, spacing, seed, n_frames, d1=60.0, fov_y_deg=45.0, aspect=1.0,
                n_way=6):
    """Catmull-Rom path through seeded waypoints: target uniform over the
    slide's xy, distance log-uniform in [d1, D0], azimuth U[0, 2pi),
    elevation U[30, 70] degrees."""
    rng = np.random.default_rng(seed)
    ext = np.asarray(dims, dtype=np.float64) * np.asarray(spacing, dtype=np.float64)
    rad = float(np.linalg.norm(ext)) / 2.0
    d0 = rad / math.sin(math.radians(fov_y_deg) / 2.0)
    way = []
    for _ in range(n_way):
        tgt = np.array([rng.uniform(0, ext[0]), rng.uniform(0, ext[1]), ext[2] / 2.0])
        dist = math.exp(rng.uniform(math.log(d1), math.log(d0)))
        az = rng.uniform(0, 2 * math.pi)
        el = math.radians(rng.uniform(30, 70))
        way.append(np.concatenate([tgt, [math.log(dist), az, el]]))
    way = np.array(way)
    # unwrap azimuth so the spline does not spin
    for i in range(1, n_way):
        while way[i, 4] - way[i - 1, 4] > math.pi:
            way[i, 4] -= 2 * math.pi
        while way[i, 4] - way[i - 1, 4] < -math.pi:
            way[i, 4] += 2 * math.pi
    P = np.vstack([way[:1], way, way[-1:]])
    cams = []
    for f in range(n_frames):
        s = f / max(n_frames - 1, 1) * (n_way - 1)
        k = min(int(s), n_way - 2)
        u = s - k
        p0, p1, p2, p3 = P[k], P[k + 1], P[k + 2], P[k + 3]
        q = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                   + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
        tgt, dist, az, el = q[:3], math.exp(q[3]), q[4], q[5]
        el = min(max(el, math.radians(20)), math.radians(80))
        eye = tgt + dist * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                                     math.sin(el)])
        cams.append(camera_persp(eye, tgt, [0.0, 0.0, 1.0], fov_y_deg, aspect))
    return cams


# ---------------------------------------------------------- transfer functions

def tf_ramp():
    """Entry i = (x, x, x, x), x = i/255."""
    x = np.arange(256, dtype=np.float64) / 255.0
    return np.stack([x, x, x, x], axis=1).astype(np.float32)


def hue_rgb(h):
    h = (h % 1.0) * 6.0
    k = int(h) % 6
    f = h - int(h)
    tab = [(1, f, 0), (1 - f, 1, 0), (0, 1, f), (0, 1 - f, 1), (f, 0, 1), (1, 0, 1 - f)]
    return tab[k]


def tf_hue(h, alpha_scale=0.1):
    """Constant hue colour, alpha = alpha_scale * x, x = i/255."""
    x = np.arange(256, dtype=np.float64) / 255.0
    r, g, b = hue_rgb(h)
    t = np.stack([np.full(256, r), np.full(256, g), np.full(256, b), alpha_scale * x], axis=1)
    return t.astype(np.float32)


def window_fx(lo_raw, hi_raw):
    """Transfer-function window in raw units as 24.8 fixed point."""
    return int(round(lo_raw * 256)), int(round(hi_raw * 256))


# ----------------------------------------------------------------- configs

class ArrayVolume(BlobVolume):
    """A volume given by its level-0 arrays (one [z][y][x] array per
    channel); coarser levels by the same 2x box filter as BlobVolume."""

    def __init__(self, arrays, bits=8, spacing=(1, 1, 1), n_levels=3):
        a0 = [np.ascontiguousarray(a) for a in arrays]
        nz, ny, nx = a0[0].shape
        self.dims = (nx, ny, nz)
        self.spacing = tuple(float(x) for x in spacing)
        self.n_channels = len(a0)
        self.bits = bits
        self.dtype = np.uint8 if bits == 8 else np.uint16
        self.n_levels = n_levels
        self.level_dims, self.level_f, halve = level_schedule(self.dims, self.spacing, n_levels)
        L = lib()
        self.levels = []
        for a in a0:
            assert a.shape == (nz, ny, nx) and a.dtype == self.dtype
            lv = [a]
            for l in range(1, n_levels):
                src = lv[-1]
                dx, dy, dz = self.level_dims[l]
                dst = np.empty((dz, dy, dx), dtype=self.dtype)
                h = halve[l]
                rc = L.synth_downsample(_ptr(src), bits, src.shape[2], src.shape[1], src.shape[0],
                                        h[0], h[1], h[2], _ptr(dst))
                assert rc == 0
                lv.append(dst)
            self.levels.append(lv)


def plateau_volume(n_channels=2, seed=5, dims=(64, 64, 64), n_levels=3):
    """u8 volume of constant-valued boxes on a zero background with one
    Gaussian blob (the only varying data): per channel c, box i holds value
    v_i + 17 c.  Large parts of it are homogeneous in every channel (the
    background and box interiors), the blob's leaves in none."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    boxes = []
    for i in range(4):
        lo = rng.integers(0, (nx * 3) // 4, 3)
        ext = rng.integers(nx // 4, nx // 2, 3)
        boxes.append((lo, lo + ext, int(rng.integers(60, 200))))
    cen = rng.uniform(0.3, 0.7, 3) * np.array([nx, ny, nz])
    blob = np.exp(-0.5 * (((x - cen[0]) ** 2 + (y - cen[1]) ** 2 + (z - cen[2]) ** 2) / 5.0 ** 2))
    out = []
    for c in range(n_channels):
        a = np.zeros((nz, ny, nx), np.float64)
        for lo, hi, v in boxes:
            a[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = v + 17 * c
        a = np.maximum(a, np.round(230 * blob))
        out.append(np.clip(a, 0, 255).astype(np.uint8))
    return ArrayVolume(out, 8, (1, 1, 1), n_levels)


def box_plateau_volume(dims=(1024, 1024, 64), n_channels=4, seed=6, n_boxes=24, spacing=(1, 1, 4), n_levels=6):
    """u16 volume of constant-valued axis-aligned boxes on a zero background:
    per channel c, box i holds (v_i + 17 c) * 256 (later boxes over earlier
    ones).  The background and the box interiors are homogeneous in every
    channel, the leaves on box faces are not."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    out = [np.zeros((nz, ny, nx), np.uint16) for _ in range(n_channels)]
    for _ in range(n_boxes):
        ext = (int(rng.integers(nx // 16, nx // 4)), int(rng.integers(ny // 16, ny // 4)),
               int(rng.integers(max(1, nz // 4), max(2, nz // 2))))
        lo = [int(rng.integers(0, dims[a] - ext[a] + 1)) for a in range(3)]
        v = int(rng.integers(60, 200))
        for c in range(n_channels):
            out[c][lo[2]:lo[2] + ext[2], lo[1]:lo[1] + ext[1], lo[0]:lo[0] + ext[0]] = (v + 17 * c) * 256
    return ArrayVolume(out, 16, spacing, n_levels)


def config1_volume(seed=1):
    """64^3 u8, 40 blobs, noise 0.02, 3 levels."""
    return BlobVolume((64, 64, 64), n_channels=1, bits=8, n_levels=3, seed=seed)


def config2_volume(seed=2, dims=(2048, 2048, 64), n_channels=4):
    return CellVolume(dims, n_channels, spacing=(1, 1, 4), n_levels=7, seed=seed)


def config3_volume(seed=3, dims=(8192, 8192, 192), n_channels=16):
    return CellVolume(dims, n_channels, spacing=(1, 1, 3), n_levels=9, seed=seed, tissue=True)


# ------------------------------------------------------------ network init

def mlp_init(seed=7, sizes=(24, 64, 64, 9)):
    """Seeded initial weights of the request predictor (He-uniform for the
    ReLU layers, small output layer, zero biases), float32, input-major."""
    rng = np.random.default_rng(seed)
    p = {}
    for i in range(3):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        lim = math.sqrt(6.0 / fan_in) * (0.25 if i == 2 else 1.0)
        p[f"W{i + 1}"] = rng.uniform(-lim, lim, size=(fan_in, fan_out)).astype(np.float32)
        p[f"b{i + 1}"] = np.zeros(fan_out, np.float32)
    return p
