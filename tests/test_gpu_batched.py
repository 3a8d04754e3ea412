"""Batched persistent launch: every item's output equals its own per-image
run bit for bit (same arithmetic per pixel) and the oracle; hipGraph replay
with new tensors of the same signature; uneven 96-scene workload."""
import numpy as np
import pytest

from gpu_helpers import D4_TOL, int_scene, require_gpu, say, strided_view, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


def small_batch(rng, dev, n=12):
    scenes, host = [], []
    for i in range(n):
        H = int(2 * rng.integers(1, 80))
        W = int(2 * rng.integers(1, 300))
        B = int(rng.integers(1, 6))
        w = "haar" if i % 2 == 0 else "d4"
        pan, ms = int_scene(rng, H, W, B)
        gain = None if i % 3 else rng.uniform(0.5, 1.5, B).astype(np.float32)
        host.append((w, pan, ms, gain))
        scenes.append(dict(pan=to_dev(pan, dev), ms=to_dev(ms, dev), wavelet=w,
                           gain=None if gain is None else to_dev(gain, dev)))
    return scenes, host


@pytest.mark.parametrize("graph", [False, True])
def test_small_batch_matches_per_image_and_oracle(dev, fz, oracle, graph):
    rng = np.random.default_rng(123)
    scenes, host = small_batch(rng, dev)
    say("batched small", "graph" if graph else "eager")
    outs = fz.fuse_batched(scenes, graph=graph)
    for s, o, (w, pan, ms, gain) in zip(scenes, outs, host):
        single = fz.fuse(s["pan"], s["ms"], w, s["gain"])
        assert torch.equal(o, single)
        ref = oracle.fuse(w, pan.astype(np.float64), ms.astype(np.float64),
                          None if gain is None else gain.astype(np.float64))
        got = o.cpu().numpy()
        if w == "haar" and gain is None:
            assert np.array_equal(got, ref.astype(np.float32))
        else:
            assert np.abs(got - ref).max() <= D4_TOL


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_variants_match_per_image(dev, fz, variant, graph):
    """Persistent rolling (1), persistent one-shot (2) and flat (3) batched
    launches give the per-image outputs bit for bit, including D4 scenes on
    the 128-bit path (LDS-staged tiles in the flat variant), ragged widths
    and band counts above one staged band group."""
    rng = np.random.default_rng(600 + variant)
    shapes = [(64, 1288, 3, "d4"), (34, 136, 9, "d4"), (2, 8, 2, "d4"), (130, 516, 5, "haar"), (66, 262, 4, "d4"),
              (18, 4070, 2, "d4"), (256, 256, 6, "haar")]
    scenes = []
    for H, W, B, w in shapes:
        pan, ms = int_scene(rng, H, W, B)
        scenes.append(dict(pan=to_dev(pan, dev), ms=to_dev(ms, dev), wavelet=w))
    ctx = fz.context(dev)
    say("batched variant", variant, "graph", graph)
    try:
        ctx.force_tile(0, 0, 0, variant)
        outs = fz.fuse_batched(scenes, graph=graph)
        outs2 = fz.fuse_batched(scenes, graph=graph)  # replay / relaunch
    finally:
        ctx.force_tile(0, 0, 0, 0)
    for s, o, o2 in zip(scenes, outs, outs2):
        ref = fz.fuse(s["pan"], s["ms"], s["wavelet"])
        assert torch.equal(o, ref)
        assert torch.equal(o2, ref)


@pytest.mark.parametrize("bands_at_once,tuning", [(2, True), (0, False)])
def test_flat_batch_per_scene_shapes(dev, fz, monkeypatch, bands_at_once, tuning):
    """The flat form with per-scene shapes (each D4 scene staged with 1 or 2
    rows per wavefront, or as one-shot wavefronts, as its own per-image tile
    says; with tuning on, the scenes' size classes are tuned first): every
    output equals its per-image call bit for bit."""
    monkeypatch.setenv("DWT_FUSE_FORCE_BATCH", "3,3,%d,2,2" % bands_at_once)
    rng = np.random.default_rng(910 + bands_at_once)
    scenes = []
    for H, W, B, w, pad in [(64, 1288, 3, "d4", 0), (34, 1030, 6, "d4", 0), (66, 262, 5, "d4", 2),
                            (130, 516, 5, "haar", 0), (18, 4070, 2, "d4", 4), (2, 8, 1, "d4", 0),
                            (1026, 2050, 3, "d4", 0), (40, 132, 4, "d4", 1)]:
        pan, ms = int_scene(rng, H, W, B)
        if pad:
            scenes.append(dict(pan=strided_view(pan, dev, pad, 0), ms=strided_view(ms, dev, pad, 0), wavelet=w))
        else:
            scenes.append(dict(pan=to_dev(pan, dev), ms=to_dev(ms, dev), wavelet=w))
    ctx = fz.Context(dev.index or 0)  # created after the variable is set
    ctx.bind_stream()
    ctx.set_tuning(tuning)
    arr, outs, keep = fz.make_items(scenes)
    say("flat batch per-scene shapes", bands_at_once, tuning)
    ctx.check(ctx.lib.dwt_fuse_run_batched(ctx.handle, arr, len(scenes), 0), "dwt_fuse_run_batched")
    torch.cuda.synchronize()
    for s, o in zip(scenes, outs):
        assert torch.equal(o, fz.fuse(s["pan"], s["ms"], s["wavelet"]))


@pytest.mark.parametrize("rows,bands_at_once,order", [(2, 0, 3), (2, 2, 3), (1, 1, 3), (1, 3, 1), (2, 2, 0)])
def test_flat_batch_forms_match_per_image(dev, fz, rows, bands_at_once, order):
    """The flat grid with staged tiles of 1 or 2 rows per wavefront, staging
    every band or 1-3 bands at a time, in each unit order, over scenes with
    16-byte, 8-byte and misaligned rows and band counts above the group size:
    every output equals its per-image call bit for bit."""
    rng = np.random.default_rng(700 + rows * 10 + bands_at_once)
    scenes = []
    for i, (H, W, B, w, pad) in enumerate([(64, 1288, 3, "d4", 0), (34, 1030, 6, "d4", 0), (66, 262, 5, "d4", 2),
                                           (130, 516, 5, "haar", 0), (18, 4070, 2, "d4", 4), (2, 8, 1, "d4", 0),
                                           (256, 254, 6, "haar", 6), (40, 132, 4, "d4", 1)]):
        pan, ms = int_scene(rng, H, W, B)
        if pad:
            scenes.append(dict(pan=strided_view(pan, dev, pad, 0), ms=strided_view(ms, dev, pad, 0), wavelet=w))
        else:
            scenes.append(dict(pan=to_dev(pan, dev), ms=to_dev(ms, dev), wavelet=w))
    for s in scenes:  # outputs start as NaN, so an item that a form skips shows
        B, H, W = s["ms"].shape[0], s["pan"].shape[0], s["pan"].shape[1]
        s["out"] = torch.full((B, H, W), float("nan"), device=dev)
    ctx = fz.context(dev)
    say("flat batch form", rows, bands_at_once, order)
    try:
        ctx.force_tile(rows, 0, 0, 3)
        ctx.force_band_split(bands_at_once)
        ctx.force_order(order)
        outs = fz.fuse_batched(scenes)
    finally:
        ctx.force_tile(0, 0, 0, 0)
        ctx.force_band_split(0)
        ctx.force_order(-1)
    for s, o in zip(scenes, outs):
        assert torch.equal(o, fz.fuse(s["pan"], s["ms"], s["wavelet"]))


def test_batch_with_pitches_and_misalignment(dev, fz):
    rng = np.random.default_rng(9)
    scenes = []
    for i, (pad, off) in enumerate([(0, 0), (6, 0), (2, 2), (1, 1), (3, 0)]):
        pan, ms = int_scene(rng, 40 + 2 * i, 130 + 4 * i, 2)
        scenes.append(dict(pan=strided_view(pan, dev, pad, off), ms=strided_view(ms, dev, pad, off),
                           wavelet="d4" if i % 2 else "haar"))
    say("batched pitches")
    outs = fz.fuse_batched(scenes)
    for s, o in zip(scenes, outs):
        assert torch.equal(o, fz.fuse(s["pan"], s["ms"], s["wavelet"]))


def test_graph_replay_with_new_tensors(dev, fz):
    """Same signature, new tensors: the replay reads the refreshed table.
    Eager work and synchronisations sit between the replays."""
    rng = np.random.default_rng(44)
    shapes = [(64, 130, 3, "haar"), (130, 66, 2, "d4"), (2, 2, 1, "d4"), (258, 514, 4, "d4")]
    for rep in range(4):
        scenes = []
        for H, W, B, w in shapes:
            pan, ms = int_scene(rng, H, W, B)
            scenes.append(dict(pan=to_dev(pan, dev), ms=to_dev(ms, dev), wavelet=w))
        say("graph replay", rep)
        outs = fz.fuse_batched(scenes, graph=True)
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device=dev) * 2).sum().item()  # eager work between replays
        for s, o in zip(scenes, outs):
            assert torch.equal(o, fz.fuse(s["pan"], s["ms"], s["wavelet"]))


def test_back_to_back_launches_reset_queues(dev, fz):
    rng = np.random.default_rng(8)
    scenes, _ = small_batch(rng, dev, n=20)
    say("batched back-to-back")
    first = [o.clone() for o in fz.fuse_batched(scenes)]
    for _ in range(5):
        again = fz.fuse_batched(scenes)
    torch.cuda.synchronize()
    for a, b in zip(first, again):
        assert torch.equal(a, b)


def test_uneven_96_scene_workload(dev, fz, oracle):
    from paper_1803_00737_amd import synth

    layout = synth.uneven_batch()
    assert len(layout) == 96
    scenes = []
    for sc in layout:
        pan, ms = synth.make_scene(sc.H, sc.W, sc.B, sc.seed, device=dev)
        scenes.append(dict(pan=pan, ms=ms, wavelet=sc.wavelet))
    torch.cuda.synchronize()
    say("uneven 96 batched")
    outs = fz.fuse_batched(scenes, graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for i, (s, o, sc) in enumerate(zip(scenes, outs, layout)):
        single = fz.fuse(s["pan"], s["ms"], sc.wavelet)
        assert torch.equal(o, single), i
        # sampled oracle check: corners and random pixels
        pts = [(0, 0, 0), (sc.B - 1, sc.H - 1, sc.W - 1), (0, sc.H - 1, 0), (sc.B - 1, 0, sc.W - 1)]
        pts += [(int(rng.integers(sc.B)), int(rng.integers(sc.H)), int(rng.integers(sc.W))) for _ in range(12)]
        b, y, x = map(np.array, zip(*pts))
        ref = oracle.fuse_points(sc.wavelet, s["pan"].cpu().numpy(), s["ms"].cpu().numpy(), None, b, y, x)
        got = o.cpu().numpy()[b, y, x]
        if sc.wavelet == "haar":
            assert np.array_equal(got, ref.astype(np.float32)), i
        else:
            assert np.abs(got - ref).max() <= D4_TOL, i
