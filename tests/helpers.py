"""Shared test helpers: scene set-up from the synthetic generator and
comparison utilities.  Nothing here computes the rendering method."""
from __future__ import annotations

import numpy as np

import synth


def tiny_blob_scene(dims=(64, 64, 64), n_channels=1, bits=8, B=16, n_levels=3, leaf=(8, 8, 8),
                    depth=3, seed=1, spacing=(1, 1, 1), n_blobs=40):
    vol = synth.BlobVolume(dims, n_channels=n_channels, bits=bits, n_levels=n_levels, seed=seed,
                           spacing=spacing, n_blobs=n_blobs)
    return vol


def leaf_grid(dims, leaf, depth):
    """Padded leaf grid of the generalised 2^k tree (power-of-two leaves per axis)."""
    n = []
    for a in range(3):
        nl = -(-dims[a] // leaf[a])
        s = 0
        while (1 << s) < nl:
            s += 1
        assert s <= depth
        n.append(1 << s)
    return tuple(n)


def single_sample_camera(point, delta=1000.0):
    """One-pixel orthographic camera whose ray has exactly one sample (k=1)
    at `point` (world units) for any volume smaller than delta."""
    p = np.asarray(point, dtype=np.float64)
    return dict(proj="ortho", eye=[float(p[0]), float(p[1]), float(p[2] - delta)],
                F=[0.0, 0.0, 1.0], R=[1.0, 0.0, 0.0], U=[0.0, 1.0, 0.0], tx=0.5, ty=0.5)


def ids_counts(counts: np.ndarray, ids: np.ndarray) -> dict:
    nz = np.nonzero(counts)[0]
    return {int(ids[i]): int(counts[i]) for i in nz}
