"""FP64 reference of the brick-request predictor's rows, history, labels and
candidates (test infrastructure; only tests, the smoke check and the bench's
CPU-baseline leg use it).

The predictor is not part of the paper; these definitions are this
project's.  Plain numpy loops over the definitions, no blocking.

Rows: one per (channel c, L0 brick position p), row = c * P + p,
p = (pz * nby + py) * nbx + px over the L0 brick grid.
History: one byte per brick (dense order: channel, level, z, y, x); bits 0-3
= requested in the last four frames (bit 0 newest), bits 4-7 = read in them.
Features of a row for the camera of a frame, with q the brick centre in
world units, v = q - eye, zf = v.F, pix = 2 ty / H (one pixel at unit
distance) and t = |v| (perspective) or max(zf, 1e-6) (orthographic):
   0  clamp(log2(B sx / footprint), -8, 8) / 8, footprint = bias pix (ortho)
      or t bias pix (perspective): the brick's edge in pixels
   1  clamp(log2(t / D_1), -8, 8) / 8, D_l = f_l sx / (bias pix)
   2  desired level at q / 8 (levels l >= 1 with t >= D_l; orthographic:
      with bias pix >= f_l sx)
   3  q in front of the camera and inside the image (0/1)
   4,5 projected image coordinates clamped to [-2, 2], / 2
   6  (pz + 1/2) / nbz
   7  fraction of the brick's tree leaves whose value range is not empty
      under the channel's window and table (0 if the channel is not shown)
   8..11 requested bits, 12..15 read bits of the row's L0 brick
  16..23 residency of the level-l brick covering p (0 for l >= levels)
Labels (for rows whose features were taken four frames earlier): level l
(l < min(levels, 9)) is 1 iff the history byte of the level-l brick covering
p is non-zero; mask 1 for those levels.
Candidates: per brick that is not resident, the largest sigmoid(z) over the
rows covering it at its level, when above the threshold.
"""
from __future__ import annotations

import math

import numpy as np

from . import level_info, node_count, tf_empty


class Geometry:
    """Brick grids and tree leaves of an oracle volume description."""

    def __init__(self, V):
        self.V = V
        d, f, nb = level_info(V)
        self.L = V.n_levels
        self.m = V.n_channels
        self.B = V.B
        self.f = f.astype(np.int64)
        self.nb = nb.astype(np.int64)
        self.sizes = [int(np.prod(nb[l])) for l in range(self.L)]
        self.loff = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.per_channel = int(self.loff[-1])
        self.P = self.sizes[0]
        tot, off, n = node_count(V)
        self.leaf_off = int(off[V.depth])
        self.nleaf = n[V.depth].astype(np.int64)
        self.leaf = np.array(V.leaf, np.int64)

    def dense(self, c, l, bx, by, bz):
        nx, ny = self.nb[l][0], self.nb[l][1]
        return c * self.per_channel + self.loff[l] + (bz * ny + by) * nx + bx

    def row_pos(self, p):
        nx, ny = self.nb[0][0], self.nb[0][1]
        return p % nx, (p // nx) % ny, p // (nx * ny)

    def cover(self, c, l, px, py, pz):
        """Dense index of the level-l brick covering L0 brick (px, py, pz)."""
        return self.dense(c, l, px // self.f[l][0], py // self.f[l][1], pz // self.f[l][2])


def record(hist, counts, res_slot, stamp, frame):
    """New history bytes after a frame: shift the four-frame windows, then
    set bit 0 for requested bricks (count > 0) and bit 4 for read ones
    (resident with the slot stamped by this frame)."""
    h = np.asarray(hist, np.uint8).astype(np.int64)
    req = (np.asarray(counts) != 0).astype(np.int64)
    rs = np.asarray(res_slot, np.int64)
    use = np.zeros_like(req)
    r = rs >= 0
    use[r] = (np.asarray(stamp)[rs[r]] == frame).astype(np.int64)
    return (((h << 1) & 0xEE) | req | (use << 4)).astype(np.uint8)


def features(G: Geometry, cam: dict, H: int, lod_bias: float, channels: list, tfs, meta, hist, res_slot,
             margin=1e-9):
    """([rows][24] float64, [rows] bool).  channels: [{c, W0, W1}] in
    visible-slot order, tfs: [n_vis][256][4]; meta: node metadata
    [n_nodes][m][2]; res_slot: per dense brick, >= 0 if resident.  The
    second output marks rows with a threshold decision (desired level,
    inside the image) within `margin` (relative) of its threshold, where
    rounding may decide it either way."""
    sp = np.array(G.V.spacing, np.float64)
    eye, F, R, U = (np.array(cam[k], np.float64) for k in ("eye", "F", "R", "U"))
    ortho = cam["proj"] == "ortho"
    tx, ty = float(cam["tx"]), float(cam["ty"])
    pix = 2.0 * ty / H
    D = [0.0] + [float(G.f[l][0]) * sp[0] / (lod_bias * pix) for l in range(1, G.L)]
    pixb = pix * lod_bias
    B = float(G.B)
    lx = int(round(math.log2(G.B // G.leaf[0])))
    ly = int(round(math.log2(G.B // G.leaf[1])))
    lz = int(round(math.log2(G.B // G.leaf[2])))
    slot_of = {}
    for j, ch in enumerate(channels):
        slot_of[int(ch["c"])] = j  # the last visible slot of a channel
    out = np.zeros((G.m * G.P, 24), np.float64)
    amb = np.zeros(G.m * G.P, bool)
    nbz = float(G.nb[0][2])
    near = lambda a, b: abs(a - b) <= margin * max(abs(a), abs(b), 1.0)
    for c in range(G.m):
        for p in range(G.P):
            row = c * G.P + p
            px, py, pz = (int(v) for v in G.row_pos(p))
            q = np.array([(px + 0.5) * B * sp[0], (py + 0.5) * B * sp[1], (pz + 0.5) * B * sp[2]])
            v = q - eye
            zf, xr, yu = float(v @ F), float(v @ R), float(v @ U)
            if ortho:
                t = max(zf, 1e-6)
                sx, sy = xr / tx, yu / ty
                foot = pixb
            else:
                t = max(math.sqrt(float(v @ v)), 1e-6)
                zz = max(zf, 1e-6)
                sx, sy = xr / (zz * tx), yu / (zz * ty)
                foot = t * pixb
            f = out[row]
            f[0] = min(max(math.log2(B * sp[0] / foot), -8.0), 8.0) / 8.0
            f[1] = min(max(math.log2(t / D[1]), -8.0), 8.0) / 8.0 if G.L > 1 else 0.0
            if ortho:
                lod = sum(1 for l in range(1, G.L) if pixb >= float(G.f[l][0]) * sp[0])
            else:
                lod = sum(1 for l in range(1, G.L) if t >= D[l])
            f[2] = lod / 8.0
            f[3] = 1.0 if (zf > 0.0 and abs(sx) <= 1.0 and abs(sy) <= 1.0) else 0.0
            amb[row] = near(zf, 0.0) or near(abs(sx), 1.0) or near(abs(sy), 1.0) or (
                any(near(pixb, float(G.f[l][0]) * sp[0]) for l in range(1, G.L)) if ortho
                else any(near(t, D[l]) for l in range(1, G.L)))
            f[4] = min(max(sx, -2.0), 2.0) / 2.0
            f[5] = min(max(sy, -2.0), 2.0) / 2.0
            f[6] = (pz + 0.5) / nbz
            j = slot_of.get(c)
            if j is not None:
                ch = channels[j]
                ne = tot = 0
                for az in range(1 << lz):
                    for ay in range(1 << ly):
                        for ax in range(1 << lx):
                            gx, gy, gz = (px << lx) + ax, (py << ly) + ay, (pz << lz) + az
                            leaf = G.leaf_off + (gz * G.nleaf[1] + gy) * G.nleaf[0] + gx
                            mn, mx = int(meta[leaf, c, 0]), int(meta[leaf, c, 1])
                            tot += 1
                            if not tf_empty(mn, mx, int(ch["W0"]), int(ch["W1"]), tfs[j]):
                                ne += 1
                f[7] = ne / tot
            h = int(hist[G.dense(c, 0, px, py, pz)])
            for k in range(4):
                f[8 + k] = (h >> k) & 1
                f[12 + k] = (h >> (4 + k)) & 1
            for l in range(min(G.L, 8)):
                f[16 + l] = 1.0 if res_slot[G.cover(c, l, px, py, pz)] >= 0 else 0.0
    return out, amb


def labels(G: Geometry, hist):
    y = np.zeros((G.m * G.P, 16), np.uint8)
    mask = np.zeros((G.m * G.P, 16), np.uint8)
    for c in range(G.m):
        for p in range(G.P):
            px, py, pz = (int(v) for v in G.row_pos(p))
            for l in range(min(G.L, 9)):
                y[c * G.P + p, l] = 1 if hist[G.cover(c, l, px, py, pz)] != 0 else 0
                mask[c * G.P + p, l] = 1
    return y, mask


def candidates(G: Geometry, z, threshold, res_slot):
    """{dense brick: best probability} of non-resident bricks above the
    threshold."""
    best = {}
    for c in range(G.m):
        for p in range(G.P):
            px, py, pz = (int(v) for v in G.row_pos(p))
            for l in range(min(G.L, 9)):
                pr = 1.0 / (1.0 + math.exp(-float(z[c * G.P + p, l])))
                if not pr > threshold:
                    continue
                b = int(G.cover(c, l, px, py, pz))
                if res_slot[b] >= 0:
                    continue
                best[b] = max(best.get(b, 0.0), pr)
    return best
