"""The predictor's row kernels against the FP64 reference: history bytes
over a streaming loop, 24 features per row, labels and candidates."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from oracle import prefetch as opf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_04393_amd import resoct  # noqa: E402
from tests.test_gpu_render import Pair, _report  # noqa: E402
from tests.test_gpu_stream import _cells, _chans, _plain  # noqa: E402

BINARY = [3] + list(range(8, 24))
CONT = [0, 1, 2, 4, 5, 6, 7]


@pytest.fixture(scope="module")
def cells():
    return _cells()


def _uncertain(o):
    """Bricks whose request or read bit the tolerated ambiguous samples can
    set on the GPU but the oracle does not."""
    return ((o["counts"] == 0) & (o["amb_counts"] > 0))


def test_rows_history_labels_candidates(cells):
    p = Pair(cells, 32, (16, 16, 4), 5, n_slots=300, max_batch=128)
    g = p.gpu
    pf = resoct.PrefetchRows(g.tree)
    G = opf.Geometry(p.V)
    assert pf.rows == G.m * G.P
    total = G.m * G.per_channel
    meta = oracle.meta_all(p.V, p.leaf_mm)
    cams = synth.orbit_path(cells.dims, cells.spacing, 8, az_step_deg=9.0)
    chans = _chans(4)
    tfs = np.stack([c["tf"] for c in chans])
    hist_o = np.zeros(total, np.uint8)
    x = torch.zeros((pf.rows, 32), dtype=torch.float16, device="cuda")
    for f in range(1, 6):
        # the frame, then the history update, then the request readback (which
        # clears the counters the history reads)
        r = g.render(f, cams[f], 96, 96, 0.5, chans, lod_bias=0.7)
        pf.record(f)
        torch.cuda.synchronize()
        g_ids, g_cnt, nu, tot = g.cache.read_requests(1 << 20)
        fr, keep = oracle.make_frame(cams[f], 96, 96, 0.5, chans, term_margin=1e-6, lod_bias=0.7)
        o = oracle.render(p.V, cells.levels, p.sim.res_slot, p.leaf_mm, fr, p.S)
        p.sim.touch(f, o["used"])
        assert not _uncertain(o).any() and not ((o["used"] == 0) & (o["amb_used"] > 0)).any()
        hist_o = opf.record(hist_o, o["counts"], p.sim.res_slot, p.sim.stamp, f)
        hist_g = pf.hist[:total].cpu().numpy()
        bad = np.nonzero(hist_g != hist_o)[0]
        assert len(bad) == 0, f"history differs at frame {f}: {[(int(b), int(hist_g[b]), int(hist_o[b])) for b in bad[:6]]}"
        # features on the frame's cache state (before its uploads)
        pf.features(r["fd"], x)
        want, amb = opf.features(G, cams[f], 96, 0.7, chans, tfs, meta, hist_o, p.sim.res_slot)
        got = x[:, :24].float().cpu().numpy().astype(np.float64)
        ok = ~amb
        assert np.array_equal(got[ok][:, BINARY], want[ok][:, BINARY]), "binary features differ"
        err = np.abs(got[ok][:, CONT] - want[ok][:, CONT].astype(np.float16).astype(np.float64))
        assert err.max() <= 2.0 ** -10, f"continuous features differ by {err.max()}"
        if f >= 2:
            y = torch.zeros((pf.rows, 16), dtype=torch.uint8, device="cuda")
            m = torch.zeros_like(y)
            pf.labels(y, m)
            yo, mo = opf.labels(G, hist_o)
            assert np.array_equal(y.cpu().numpy(), yo) and np.array_equal(m.cpu().numpy(), mo)
        # the plain policy's uploads, from the oracle's requests (equal to the GPU's)
        up = p.ids[p.sim.plain_policy(o["counts"], 64)]
        assert np.array_equal(up, _plain(g_ids, g_cnt, 64))
        p.upload(f, up)
        p.gpu.tree.update_residency()
        _report(f"pf-frame-{f}", rows=pf.rows, ambiguous_rows=int(amb.sum()), in_view=int(want[:, 3].sum()),
                hist_nonzero=int((hist_o != 0).sum()))
    # candidates from seeded logits
    rng = np.random.default_rng(9)
    z = (2.5 * rng.normal(size=(pf.rows, 16))).astype(np.float32)
    thr = 0.6
    ids, pr = pf.candidates(torch.from_numpy(z).cuda(), thr, cap=1 << 20)
    best = opf.candidates(G, z.astype(np.float64), thr, p.sim.res_slot)
    near = {b for b, v in best.items() if abs(v - thr) < 1e-6}
    want = {int(p.ids[b]): v for b, v in best.items() if b not in near}
    got = {int(i): float(v) for i, v in zip(ids, pr)}
    assert np.all(np.diff(ids.astype(np.int64)) > 0), "candidates not in ascending ID order"
    assert set(want) <= set(got) and set(got) - set(want) <= {int(p.ids[b]) for b in near}
    assert max(abs(got[i] - want[i]) for i in want) <= 1e-6
    _report("pf-candidates", n=len(got), near_threshold=len(near))


def test_learned_policy_gains_over_plain_streaming():
    """The predictor trained online along three camera paths, then both
    policies on two held-out paths from an empty cache with the same upload
    budget (4-channel 2048 x 2048 x 64 cells, 2 GiB cache, 1024 x 1024
    views, 512 bricks per frame): the learned policy leaves fewer channel
    samples without their desired brick (it only changes which bricks are
    streamed)."""
    from paper_2309_04393_amd.pipeline import GpuScene
    from paper_2309_04393_amd.prefetch import BrickStore, run_path, save_state
    from tests.helpers import leaf_grid
    import bench
    src = synth.config2_volume()
    leaf = (16, 16, 4)
    lg = leaf_grid(src.dims, leaf, 7)
    scene = GpuScene(src, 32, leaf, 7, 27318, max_batch=512, start_level=2, set_metadata=False)
    mx = src.leaf_max_all(leaf, lg)
    for c in range(src.n_channels):
        mm = np.zeros((mx.shape[1], 2), np.uint16)
        mm[:, 1] = mx[c]
        scene.set_metadata(c, mm)
    store = BrickStore(scene)
    empty = save_state(scene)
    chans = [dict(ch, hi=src.n_levels - 1) for ch in bench.channels(src.n_channels, 2)]
    net = resoct.Mlp()
    net.set_weights(synth.mlp_init(7))
    path = lambda s: synth.random_path(src.dims, src.spacing, s, 120)
    for s in (1000, 1001, 1002):
        run_path(scene, store, path(s), chans, 1024, 1024, 512, 0.5, "learned", net, empty)
    res = []
    for s in (1010, 1012):
        _, p = run_path(scene, store, path(s), chans, 1024, 1024, 512, 0.5, "plain", None, empty)
        _, q = run_path(scene, store, path(s), chans, 1024, 1024, 512, 0.5, "learned", net, empty)
        res.append((p, q))
        _report(f"pf-eval-{s}", plain_missing=round(p["mean_missing"], 4), learned_missing=round(q["mean_missing"], 4),
                plain_converge=p["frames_to_converge"], learned_converge=q["frames_to_converge"],
                plain_bytes=p["bytes_streamed"], learned_bytes=q["bytes_streamed"], extra=q["extra"],
                precision=q["precision"])
    plain = np.mean([p["mean_missing"] for p, _ in res])
    learned = np.mean([q["mean_missing"] for _, q in res])
    assert learned < plain, (plain, learned)
