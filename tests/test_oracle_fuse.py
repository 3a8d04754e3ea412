"""Pins of the oracle's fusion (section 2: forward 2D DWT of PAN, LL replaced
by an MS band, inverse 2D DWT), against forms computed by other code paths:

  * Haar closed form: out = up(m) + gain * (PAN - up(blockmean2x2(PAN)))
    (Eq. 1-2 / 11-12 with the /2 normalisation);
  * D4 projection form: out = gain * PAN + L^T (m - gain * L PAN) with
    L = Hc (x) Hr built from the FFT evaluation of Eq. 3-6 (orthonormal
    transform, so the inverse of the detail part is PAN minus its LL part);
  * fuse(PAN, LL(PAN)) = PAN; flat inputs; cyclic-shift equivariance;
  * the single-pixel evaluation equals the full-image one.
"""
import numpy as np
import pytest

from test_oracle_transforms import fft_forward, matrix_of


def up(a):
    return np.repeat(np.repeat(a, 2, axis=0), 2, axis=1)


def blockmean(x):
    H, W = x.shape
    return x.reshape(H // 2, 2, W // 2, 2).mean(axis=(1, 3))


def lowpass_rows(oracle, wavelet, N):
    M = matrix_of(lambda v: fft_forward(oracle.filters(), wavelet, v), N)
    return M[: N // 2]


def d4_projection(oracle, pan, ms, gain):
    H, W = pan.shape
    Hc, Hr = lowpass_rows(oracle, "d4", H), lowpass_rows(oracle, "d4", W)
    out = []
    for b in range(ms.shape[0]):
        c = ms[b] - gain[b] * (Hc @ pan @ Hr.T)
        out.append(gain[b] * pan + Hc.T @ c @ Hr)
    return np.stack(out)


def scene(rng, H, W, B):
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    ms = rng.integers(0, 256, (B, H // 2, W // 2)).astype(np.float64)
    return pan, ms


SHAPES = [(2, 2), (2, 6), (4, 4), (6, 10), (16, 8), (34, 18), (64, 64)]


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_ms_equal_to_ll_reproduces_pan(oracle, wavelet, H, W):
    rng = np.random.default_rng(H * 7 + W)
    pan, _ = scene(rng, H, W, 1)
    ll = oracle.dwt2_fwd(wavelet, pan)[: H // 2, : W // 2]
    out = oracle.fuse(wavelet, pan, ll[None])[0]
    if wavelet == "haar":
        assert np.array_equal(out, pan)
    else:
        assert np.abs(out - pan).max() < 1e-11


@pytest.mark.parametrize("H,W", SHAPES)
def test_haar_closed_form_exact(oracle, H, W):
    rng = np.random.default_rng(H * 13 + W)
    pan, ms = scene(rng, H, W, 3)
    out = oracle.fuse("haar", pan, ms)
    for b in range(3):
        ref = up(ms[b]) + (pan - up(blockmean(pan)))
        assert np.array_equal(out[b], ref)
    # every value is a multiple of 1/4 below 2^10: exact in float32
    assert np.array_equal(out * 4, np.rint(out * 4))
    assert np.array_equal(out.astype(np.float32).astype(np.float64), out)


@pytest.mark.parametrize("H,W", SHAPES)
def test_haar_closed_form_with_gain(oracle, H, W):
    rng = np.random.default_rng(H * 17 + W)
    pan, ms = scene(rng, H, W, 2)
    gain = np.array([0.3, 1.7])
    out = oracle.fuse("haar", pan, ms, gain)
    for b in range(2):
        ref = up(ms[b]) + gain[b] * (pan - up(blockmean(pan)))
        assert np.abs(out[b] - ref).max() < 1e-12


@pytest.mark.parametrize("H,W", SHAPES)
def test_d4_projection_form(oracle, H, W):
    rng = np.random.default_rng(H * 19 + W)
    pan, ms = scene(rng, H, W, 3)
    gain = np.array([1.0, 0.5, 1.6])
    out = oracle.fuse("d4", pan, ms, gain)
    np.testing.assert_allclose(out, d4_projection(oracle, pan, ms, gain), rtol=0, atol=1e-10)


def test_flat_inputs(oracle):
    pan = np.full((8, 10), 120.0)
    ms = np.full((1, 4, 5), 80.0)
    assert np.array_equal(oracle.fuse("haar", pan, ms)[0], np.full((8, 10), 80.0))
    # D4 LL of a flat image is 2c, so the unscaled replacement gives m/2
    assert np.abs(oracle.fuse("d4", pan, ms)[0] - 40.0).max() < 1e-12


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_cyclic_shift_equivariance(oracle, wavelet):
    rng = np.random.default_rng(5)
    pan, ms = scene(rng, 12, 16, 2)
    out = oracle.fuse(wavelet, pan, ms)
    for r, c in [(1, 0), (0, 3), (2, 5)]:
        o2 = oracle.fuse(wavelet, np.roll(pan, (2 * r, 2 * c), (0, 1)), np.roll(ms, (r, c), (1, 2)))
        assert np.abs(o2 - np.roll(out, (2 * r, 2 * c), (1, 2))).max() < 1e-11


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_gain_zero_keeps_only_ms(oracle, wavelet):
    rng = np.random.default_rng(9)
    pan, ms = scene(rng, 8, 12, 1)
    out = oracle.fuse(wavelet, pan, ms, [0.0])[0]
    if wavelet == "haar":
        assert np.array_equal(out, up(ms[0]))
    else:
        Hc, Hr = lowpass_rows(oracle, "d4", 8), lowpass_rows(oracle, "d4", 12)
        assert np.abs(out - Hc.T @ ms[0] @ Hr).max() < 1e-12


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_bands_are_independent(oracle, wavelet):
    rng = np.random.default_rng(11)
    pan, ms = scene(rng, 10, 14, 3)
    gain = [0.9, 1.1, 1.3]
    out = oracle.fuse(wavelet, pan, ms, gain)
    for b in range(3):
        assert np.array_equal(out[b], oracle.fuse(wavelet, pan, ms[b:b + 1], [gain[b]])[0])


@pytest.mark.parametrize("H,W", [(2, 2), (4, 6), (18, 10), (32, 64)])
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_point_equals_full(oracle, wavelet, H, W):
    rng = np.random.default_rng(H * 3 + W)
    pan, ms = scene(rng, H, W, 2)
    gain = [1.0, 0.7]
    out = oracle.fuse(wavelet, pan, ms, gain)
    pts = [(b, y, x) for b in range(2) for y in {0, 1, H - 2, H - 1, H // 2} for x in {0, 1, W - 2, W - 1, W // 2}]
    pts += [(1, int(rng.integers(H)), int(rng.integers(W))) for _ in range(20)]
    b, y, x = map(np.array, zip(*pts))
    vals = oracle.fuse_points(wavelet, pan, ms, gain, b, y, x)
    assert np.array_equal(vals, out[b, y, x])


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(2, 2), (2, 8), (6, 4), (16, 10), (34, 22), (40, 64)])
def test_row_strips_stitch_to_the_whole_image(oracle, wavelet, H, W):
    """The row-strip entry point evaluates only the coefficient and PAN rows
    its output rows need, with the same arithmetic: any partition of the rows
    into strips (odd and even cuts, single rows, strips touching the top and
    bottom wrap) stitches to the whole-image fusion bit for bit, with gains
    and kappa; an empty strip is empty and out-of-range strips are rejected."""
    rng = np.random.default_rng(H * 100 + W)
    B = 3
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    ms = rng.integers(0, 256, (B, H // 2, W // 2)).astype(np.float64)
    gain = np.array([1.0, 0.75, 1.3])
    for kappa in (1.0, 2.0):
        full = oracle.fuse(wavelet, pan, ms, gain, kappa)
        cuts = sorted(set([0, H] + [int(c) for c in rng.integers(0, H + 1, 4)]))
        for cuts_ in (cuts, list(range(H + 1))):
            parts = [oracle.fuse_rows(wavelet, pan, ms, a, b, gain, kappa) for a, b in zip(cuts_[:-1], cuts_[1:])]
            assert np.array_equal(np.concatenate(parts, axis=1), full)
    assert oracle.fuse_rows(wavelet, pan, ms, 1, 1).shape == (B, 0, W)
    for a, b in ((-1, 1), (0, H + 1), (2, 1)):
        with pytest.raises(ValueError):
            oracle.fuse_rows(wavelet, pan, ms, a, b)

