"""Pins for the 8-bit code and the kappa-scaled replacement of the oracle.

8-bit code (section 3 stores images at 8 bits per pixel; the rounding rule is
this implementation's reading): nearest integer, ties to even, clamp to
[0, 255], NaN -> 0.  Pinned against hand-worked values, numpy's rint (an
independent round-half-even) and Python's own round() on quarter values.

kappa (LL <- kappa * MS): pinned by closed forms on flat images, the identity
fuse(PAN, LL(PAN) / kappa, kappa) = PAN, linearity in kappa and, for the
DC-matched D4 value kappa = 2, by reproducing a smooth PAN from its own 2x2
block means.
"""
import numpy as np
import pytest


HAND = [(0.5, 0), (1.5, 2), (2.5, 2), (-0.5, 0), (-1.5, 0), (254.5, 254), (255.5, 255), (253.5, 254),
        (300.0, 255), (-3.0, 0), (127.49999, 127), (127.5000001, 128), (3.25, 3), (3.75, 4), (0.0, 0),
        (-0.0, 0), (255.0, 255), (float("nan"), 0), (float("inf"), 255), (float("-inf"), 0), (1e300, 255),
        (-1e300, 0), (0.49999999999999994, 0)]


def test_quantize_hand_values(oracle):
    v = np.array([a for a, _ in HAND])
    want = np.array([b for _, b in HAND], dtype=np.uint8)
    assert np.array_equal(oracle.quantize_u8(v), want)


def test_quantize_matches_rint_and_clip(oracle):
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(128, 90, 20000), np.arange(-40, 1100) / 4.0, np.arange(-10, 270) + 0.5])
    want = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    assert np.array_equal(oracle.quantize_u8(v), want)
    q = oracle.quantize_u8(v.reshape(-1, 7)[: 100])
    assert q.shape == (100, 7)


def test_haar_u8_of_integer_inputs_is_exact(oracle):
    """Haar outputs of integer inputs are quarter values; their 8-bit codes
    follow from Python's round() (ties to even) on the exact quarters."""
    rng = np.random.default_rng(2)
    pan = rng.integers(0, 256, (16, 24)).astype(np.float64)
    ms = rng.integers(0, 256, (2, 8, 12)).astype(np.float64)
    out = oracle.fuse("haar", pan, ms)
    quarters = np.rint(out * 4).astype(np.int64)
    assert np.array_equal(quarters / 4.0, out)
    want = np.array([min(255, max(0, round(int(q) / 4))) for q in quarters.ravel()], dtype=np.uint8)
    assert np.array_equal(oracle.quantize_u8(out).ravel(), want)


@pytest.mark.parametrize("w,dc", [("haar", 1.0), ("d4", 0.5)])
@pytest.mark.parametrize("kappa", [1.0, 2.0, 0.5])
def test_kappa_flat(oracle, w, dc, kappa):
    """Flat PAN c, flat MS m: details vanish, so the output is flat at
    kappa * m times the synthesis DC gain (1 for Haar, 1/2 for D4)."""
    pan = np.full((8, 12), 37.0)
    ms = np.full((1, 4, 6), 90.0)
    out = oracle.fuse(w, pan, ms, kappa=kappa)
    assert np.allclose(out, kappa * 90.0 * dc, atol=1e-10)


@pytest.mark.parametrize("w", ["haar", "d4"])
@pytest.mark.parametrize("kappa", [2.0, 0.75])
def test_kappa_identity_and_linearity(oracle, w, kappa):
    rng = np.random.default_rng(3)
    H, W = 12, 20
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    ll = oracle.dwt2_fwd(w, pan)[: H // 2, : W // 2]
    assert np.allclose(oracle.fuse(w, pan, ll[None] / kappa, kappa=kappa)[0], pan, atol=1e-9)
    ms = rng.integers(0, 256, (2, H // 2, W // 2)).astype(np.float64)
    g = [0.7, 1.3]
    f0 = oracle.fuse(w, pan, ms, g, kappa=0.0)
    f1 = oracle.fuse(w, pan, ms, g)
    fk = oracle.fuse(w, pan, ms, g, kappa=kappa)
    assert np.allclose(fk, f0 + kappa * (f1 - f0), atol=1e-9)
    # kappa = 0 leaves only the (scaled) detail part of PAN, the same for every band up to its gain
    assert np.allclose(f0[0] / g[0], f0[1] / g[1], atol=1e-9)


def test_dc_matched_d4_reproduces_smooth_pan(oracle):
    """With MS = the 2x2 block means of a smooth PAN (what a sensor at half
    the resolution sees), D4 with kappa = 2 returns PAN up to the small
    smoothing error, while kappa = 1 loses half the mean level (the dark
    D4 images the paper reports)."""
    H, W = 64, 64
    y, x = np.mgrid[0:H, 0:W]
    pan = 120 + 40 * np.sin(2 * np.pi * x / W) * np.cos(2 * np.pi * y / H)
    ms = pan.reshape(H // 2, 2, W // 2, 2).mean(axis=(1, 3))[None]
    assert oracle.dc_kappa("d4") == 2.0 and oracle.dc_kappa("haar") == 1.0
    e2 = np.sqrt(((oracle.fuse("d4", pan, ms, kappa=2.0)[0] - pan) ** 2).mean())
    e1 = oracle.fuse("d4", pan, ms)[0] - pan
    assert e2 < 1.0
    assert abs(e1.mean() + pan.mean() / 2) < 1.0
    eh = np.sqrt(((oracle.fuse("haar", pan, ms)[0] - pan) ** 2).mean())
    assert eh < 1e-9 * pan.max() + 1e-9  # Haar's LL is the block mean itself


def test_quality_closed_forms(oracle):
    """sse and sums against hand-derived values and numpy's own sums; the
    ERGAS-style score of a constant error c on a flat reference mu is
    100 * (1/2) * c / mu."""
    H, W = 6, 10
    ref = np.full((2, H, W), 80.0)
    fused = ref.copy()
    fused[0] += 4.0
    fused[1, 2, 3] -= 5.0
    q = oracle.quality(fused, ref)
    assert np.array_equal(q["sse"], [16.0 * H * W, 25.0])
    assert np.array_equal(q["sum_ref"], [80.0 * H * W] * 2)
    assert np.allclose(q["rmse"], [4.0, 5.0 / np.sqrt(H * W)])
    one = oracle.quality(fused[:1], ref[:1])
    assert abs(one["ergas"] - 100 * 0.5 * 4.0 / 80.0) < 1e-12
    rng = np.random.default_rng(5)
    a, b = rng.normal(100, 30, (3, 17, 9)), rng.normal(100, 30, (3, 17, 9))
    q = oracle.quality(a, b)
    assert np.allclose(q["sse"], ((a - b) ** 2).sum(axis=(1, 2)), rtol=1e-13)
    assert np.allclose(q["sum_ref"], b.sum(axis=(1, 2)), rtol=1e-13)
    assert np.all(oracle.quality(b, b)["sse"] == 0)
