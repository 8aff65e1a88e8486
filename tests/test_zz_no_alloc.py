"""ro_read_requests_noalloc (the readback for callers that cannot allocate)
returns what ro_read_requests returns for the same counters, on two calls in
a row, the second over fewer requests; its limits are rejected."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_04393_amd import resoct  # noqa: E402
from paper_2309_04393_amd.pipeline import GpuScene  # noqa: E402


def _chans(n):
    return [dict(c=c, lo=0, hi=5, W0=300 * 256, W1=8000 * 256, tf=synth.tf_hue(c / n, 0.1)) for c in range(n)]


@pytest.fixture(scope="module")
def scene():
    src = synth.CellVolume((512, 512, 64), 4, spacing=(1, 1, 4), n_levels=6, seed=2)
    sc = GpuScene(src, 32, (16, 16, 4), 5, n_slots=64, max_batch=128)
    ids = sc.all_ids()
    # a sparse resident set: most samples miss their desired brick
    sc.upload(0, ids[::97][:64])
    sc.tree.update_residency()
    return sc


def _render(sc, frame, size):
    cam = synth.orbit_path(sc.src.dims, sc.src.spacing, 4)[1]
    sc.render(frame, cam, size, size, 0.5, _chans(4))
    torch.cuda.synchronize()


@pytest.mark.parametrize("size", [96, 40])
def test_noalloc_readback_equals_readback(scene, size):
    """Same frame rendered twice: counters are identical sums, so both
    readbacks must agree exactly (IDs, counts, distinct count, total); the
    second parameter renders a smaller viewport, so the fixed work space
    holds fewer pairs than after the first call."""
    cap = 1 << 16
    _render(scene, 1, size)
    ids_a, cnt_a, nu_a, tot_a = scene.cache.read_requests(cap)
    _render(scene, 1, size)
    ids_b, cnt_b, nu_b, tot_b = scene.cache.read_requests_noalloc(cap)
    print(f"noalloc size {size}: {nu_a} bricks, {tot_a} samples", flush=True)
    assert nu_a > 0 and tot_a > 0
    assert (nu_a, tot_a) == (nu_b, tot_b)
    assert np.array_equal(ids_a, ids_b) and np.array_equal(cnt_a, cnt_b)
    # the counters are clear after either readback
    _, _, nu_c, tot_c = scene.cache.read_requests_noalloc(cap)
    assert nu_c == 0 and tot_c == 0


def test_noalloc_capped_and_rejected(scene):
    _render(scene, 2, 64)
    ids_a, cnt_a, nu_a, tot_a = scene.cache.read_requests(7)
    _render(scene, 2, 64)
    ids_b, cnt_b, nu_b, tot_b = scene.cache.read_requests_noalloc(7)
    assert (nu_a, tot_a) == (nu_b, tot_b) and len(ids_b) == min(7, nu_a)
    assert np.array_equal(ids_a, ids_b) and np.array_equal(cnt_a, cnt_b)
    with pytest.raises(resoct.ResoctError):
        scene.cache.read_requests_noalloc(resoct.NOALLOC_MAX_PAIRS + 1)
