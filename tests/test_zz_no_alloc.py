"""dwt_fuse_backward_noalloc (the backward entry point for callers that cannot
allocate device memory) against dwt_fuse_backward, through the C ABI: same
kernels, so grad_pan, grad_ms and grad_gain must agree bit for bit, on two
calls in a row with the second input smaller than the first (the static
scratch keeps the first call's partial sums, which the second must not
read).  Also: the oracle on a small scene, every LDS-staged / rolling /
scalar adjoint kind, the size limit of the static scratch (rejected before
any launch, outputs untouched), and outputs left as NULL."""
import numpy as np
import pytest

from gpu_helpers import int_scene, require_gpu, say, to_dev, torch

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 16 * 1024 * 1024


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


def outputs_like(pan, gy, dev, fill=float("nan")):
    B, H, W = gy.shape
    return (torch.full((H, W), fill, device=dev), torch.full((B, H // 2, W // 2), fill, device=dev),
            torch.full((B,), fill, device=dev))


def both(fz, dev, wavelet, pan, gy, gain=None):
    ref = fz.fuse_backward(pan, gy, wavelet, gain)
    got = fz.fuse_backward_noalloc(pan, gy, *outputs_like(pan, gy, dev), wavelet=wavelet, gain=gain)
    torch.cuda.synchronize()
    return ref, got


def assert_same(ref, got, what):
    for name, r, g in zip(("grad_pan", "grad_ms", "grad_gain"), ref, got):
        assert torch.equal(r, g), (what, name, float((r - g).abs().max()))


# (wavelet, H, W, B, pan row offset): LDS-staged D4 (B >= 5, or a scene too
# small for rolling units), band-unrolled rolling D4 and Haar, band groups
# above the rolling kernel's band limit, 8-byte rows, scalar rows (one column
# per lane: twice the partial slots).
CASES = [("d4", 512, 512, 6, 0), ("d4", 2048, 2048, 4, 0), ("haar", 1024, 1032, 3, 0), ("d4", 130, 1030, 9, 0),
         ("d4", 258, 1026, 3, 0), ("haar", 96, 200, 12, 0), ("d4", 300, 640, 2, 1), ("haar", 64, 130, 5, 1)]


@pytest.mark.parametrize("wavelet,H,W,B,off", CASES)
def test_matches_backward_two_calls_second_smaller(dev, fz, wavelet, H, W, B, off):
    rng = np.random.default_rng(H + W + B)
    for H_, W_ in ((H, W), (H // 2 if (H // 2) % 2 == 0 else H // 2 + 1, W // 2 if (W // 2) % 2 == 0 else W // 2 + 1)):
        pan = rng.integers(0, 256, (H_, W_)).astype(np.float32)
        gy = rng.normal(size=(B, H_, W_)).astype(np.float32)
        gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
        if off:  # rows starting at an odd float offset: the scalar path
            pbuf = torch.zeros(H_ * W_ + off, device=dev)
            p = pbuf[off:].view(H_, W_)
            p.copy_(to_dev(pan, dev))
            gbuf = torch.zeros(B * H_ * W_ + off, device=dev)
            g = gbuf[off:].view(B, H_, W_)
            g.copy_(to_dev(gy, dev))
        else:
            p, g = to_dev(pan, dev), to_dev(gy, dev)
        say("noalloc backward", wavelet, H_, W_, B, "offset", off)
        ref, got = both(fz, dev, wavelet, p, g, to_dev(gain, dev))
        assert_same(ref, got, (wavelet, H_, W_, B, off))


def test_matches_oracle(dev, fz, oracle):
    rng = np.random.default_rng(3)
    for wavelet in ("haar", "d4"):
        pan, _ = int_scene(rng, 66, 134, 3)
        gy = rng.normal(size=(3, 66, 134)).astype(np.float32)
        gain = np.array([1.0, 0.75, 1.25], np.float32)
        say("noalloc backward vs oracle", wavelet)
        gp, gm, gg = fz.fuse_backward_noalloc(to_dev(pan, dev), to_dev(gy, dev),
                                              *outputs_like(None, gy, dev), wavelet=wavelet,
                                              gain=to_dev(gain, dev))
        rp, rm, rg = oracle.fuse_backward(wavelet, pan.astype(np.float64), gain.astype(np.float64),
                                          gy.astype(np.float64))
        assert np.abs(gp.cpu().numpy() - rp).max() <= 16e-5 * max(1.0, np.abs(rp).max())
        assert np.abs(gm.cpu().numpy() - rm).max() <= 16e-5 * max(1.0, np.abs(rm).max())
        # detail part of PAN, D = PAN - P PAN, from the oracle's fusion with gain 1 and zero MS
        D = oracle.fuse(wavelet, pan.astype(np.float64), np.zeros((1, 33, 67)))[0]
        for b in range(3):
            assert abs(float(gg[b]) - rg[b]) <= 1e-5 * np.abs(gy[b] * D).sum() + 1e-6


def test_outputs_may_be_null(dev, fz):
    rng = np.random.default_rng(4)
    pan = to_dev(rng.integers(0, 256, (128, 256)).astype(np.float32), dev)
    gy = to_dev(rng.normal(size=(3, 128, 256)).astype(np.float32), dev)
    ref = fz.fuse_backward(pan, gy, "d4")
    gp, gm, gg = outputs_like(pan, gy, dev)
    say("noalloc backward, grad_gain only / no grad_gain")
    fz.fuse_backward_noalloc(pan, gy, None, None, gg, wavelet="d4")
    fz.fuse_backward_noalloc(pan, gy, gp, gm, None, wavelet="d4")
    torch.cuda.synchronize()
    assert torch.equal(gg, ref[2]) and torch.equal(gp, ref[0]) and torch.equal(gm, ref[1])


def test_scratch_limit(dev, fz):
    """A one-column-pair Haar image 2^22 rows tall with 2 bands needs
    2^21 slots x 2 bands x 4 bytes = 16 MiB of partial sums plus the chunk
    sums: more than the static scratch, so the call is rejected before any
    launch (outputs untouched) while dwt_fuse_backward handles it; half as
    tall fits and matches dwt_fuse_backward bit for bit."""
    from paper_1803_00737_amd import _lib

    rng = np.random.default_rng(5)
    for H, fits in (((1 << 21), True), ((1 << 22), False)):
        pan = to_dev(rng.integers(0, 256, (H, 2)).astype(np.float32), dev)
        gy = to_dev(rng.normal(size=(2, H, 2)).astype(np.float32), dev)
        ref = fz.fuse_backward(pan, gy, "haar")
        outs = outputs_like(pan, gy, dev, fill=7.0)
        say("noalloc scratch limit", H, fits)
        if fits:
            fz.fuse_backward_noalloc(pan, gy, *outs, wavelet="haar")
            torch.cuda.synchronize()
            assert_same(ref, outs, ("limit", H))
        else:
            with pytest.raises(_lib.DwtFuseError) as ei:
                fz.fuse_backward_noalloc(pan, gy, *outs, wavelet="haar")
            assert ei.value.status == 2 and "static scratch" in str(ei.value)
            torch.cuda.synchronize()
            for t in outs:
                assert bool((t == 7.0).all())
