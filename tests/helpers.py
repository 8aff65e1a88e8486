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


def gpu_rgba(t, H, W):
    return t.detach().float().cpu().numpy()[: H * W * 4].reshape(H, W, 4).astype(np.float64)


def compare_images(gpu, ref, amb_pix, max_abs=1e-3, mean_abs=1e-5, max_amb_frac=1e-3, alt=None):
    """Per RGBA channel: max abs <= max_abs and mean abs <= mean_abs over the
    pixels that are not ambiguous; the ambiguous fraction stays small.  With
    alt = (alt_rgba, alt_pix) from the oracle, a pixel whose one termination
    decision was a close call is compared with whichever of its two valid
    values it is nearer (by the largest channel difference)."""
    ok = amb_pix == 0
    frac = 1.0 - ok.mean()
    d = np.abs(gpu - ref)
    if alt is not None:
        a_rgba, a_pix = alt
        da = np.abs(gpu - a_rgba)
        use = (a_pix != 0) & (da.max(axis=-1) < d.max(axis=-1))
        d = np.where(use[..., None], da, d)
    d = d[ok]
    mx = d.max(axis=0) if d.size else np.zeros(4)
    mn = d.mean(axis=0) if d.size else np.zeros(4)
    assert frac <= max_amb_frac, f"ambiguous pixel fraction {frac}"
    assert (mx <= max_abs).all(), f"max abs per channel {mx}"
    assert (mn <= mean_abs).all(), f"mean abs per channel {mn}"
    return dict(max_abs=mx.tolist(), mean_abs=mn.tolist(), amb_frac=frac)


def oracle_alt(o):
    """The (alt_rgba, alt_pix) pair of an oracle frame for compare_images."""
    return o["alt_rgba"], o["alt_pix"]


def aov_mask(o):
    """Pixels whose per-level read counts are unique: no ambiguous sample and
    no close termination call (the GPU may take one sample more or less)."""
    return (o["amb_pix"] == 0) & (o["alt_pix"] == 0)


def compare_requests(gpu_ids, gpu_counts, oracle_counts, oracle_amb, dense_ids):
    """Bit-exact multiset outside the tolerated set: for every brick the GPU
    count lies in [oracle, oracle + ambiguous samples that requested it]."""
    g = {int(i): int(c) for i, c in zip(gpu_ids, gpu_counts)}
    o = ids_counts(oracle_counts, dense_ids)
    a = ids_counts(oracle_amb, dense_ids)
    keys = set(g) | set(o)
    bad = [(hex(k), g.get(k, 0), o.get(k, 0), a.get(k, 0)) for k in sorted(keys)
           if not (o.get(k, 0) <= g.get(k, 0) <= o.get(k, 0) + a.get(k, 0))]
    assert not bad, f"{len(bad)} request counts differ, first: {bad[:8]}"
    return len(g)


def compare_usage(gpu_slots, oracle_used, oracle_amb_used):
    g = set(int(s) for s in gpu_slots)
    o = set(np.nonzero(oracle_used)[0].tolist())
    a = set(np.nonzero(oracle_amb_used)[0].tolist())
    assert o <= g, f"slots read by the oracle but not the GPU: {sorted(o - g)[:8]}"
    assert g <= o | a, f"slots read by the GPU only: {sorted(g - o - a)[:8]}"
