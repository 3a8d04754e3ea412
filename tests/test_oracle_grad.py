"""Pins of the oracle's transpose of the fusion map (the gradient rule the
adjoint kernel must reproduce):

  * dense Jacobians built from unit impulses through the forward oracle, then
    J^T y compared with the backward oracle (brute force, 8x8 and 6x10);
  * the closed forms implied by the linear structure: Haar dL/dm = 2x2 block
    sum of y, dL/dPAN = sum_b gain_b (y_b - up(blockmean(y_b))); D4
    dL/dm = L y, dL/dPAN = sum_b gain_b (y_b - L^T L y_b); dL/dgain_b =
    <y_b, PAN - (LL part of PAN)>;
  * FP64 central finite differences of an MSE loss on a 32x32 crop (exact up
    to rounding, since the loss is quadratic in every input).
"""
import numpy as np
import pytest

from test_oracle_fuse import blockmean, lowpass_rows, up


def fuse_flat(oracle, wavelet, H, W, B, gain):
    n_pan, n_ms = H * W, B * (H // 2) * (W // 2)

    def f(v):
        pan = v[:n_pan].reshape(H, W)
        ms = v[n_pan:].reshape(B, H // 2, W // 2)
        return oracle.fuse(wavelet, pan, ms, gain).reshape(-1)

    return f, n_pan + n_ms


@pytest.mark.parametrize("H,W", [(8, 8), (6, 10), (2, 4)])
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_backward_is_jacobian_transpose(oracle, wavelet, H, W):
    B = 2
    gain = np.array([0.7, 1.3])
    f, n = fuse_flat(oracle, wavelet, H, W, B, gain)
    J = np.stack([f(np.eye(n)[j]) for j in range(n)], axis=1)  # linear map: columns are impulse responses
    rng = np.random.default_rng(H + W)
    gy = rng.normal(size=(B, H, W))
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    gp, gm, gg = oracle.fuse_backward(wavelet, pan, gain, gy)
    JTy = J.T @ gy.reshape(-1)
    assert np.abs(gp.reshape(-1) - JTy[: H * W]).max() < 1e-12
    assert np.abs(gm.reshape(-1) - JTy[H * W:]).max() < 1e-12
    # the output is linear in each gain: central difference is exact up to rounding
    ms = rng.integers(0, 256, (B, H // 2, W // 2)).astype(np.float64)
    for b in range(B):
        e = np.zeros(B)
        e[b] = 0.5
        d = (oracle.fuse(wavelet, pan, ms, gain + e) - oracle.fuse(wavelet, pan, ms, gain - e)) / 1.0
        assert abs((d * gy).sum() - gg[b]) < 1e-9 * max(1.0, abs(gg[b]))


def test_haar_closed_forms(oracle):
    rng = np.random.default_rng(3)
    H, W, B = 12, 10, 3
    gain = np.array([1.0, 0.4, 2.0])
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    gy = rng.normal(size=(B, H, W))
    gp, gm, gg = oracle.fuse_backward("haar", pan, gain, gy)
    blocksum = lambda y: 4 * blockmean(y)
    for b in range(B):
        assert np.abs(gm[b] - blocksum(gy[b])).max() < 1e-12
        assert abs(gg[b] - (gy[b] * (pan - up(blockmean(pan)))).sum()) < 1e-9
    ref = sum(gain[b] * (gy[b] - up(blockmean(gy[b]))) for b in range(B))
    assert np.abs(gp - ref).max() < 1e-12


def test_d4_closed_forms(oracle):
    rng = np.random.default_rng(4)
    H, W, B = 16, 12, 2
    gain = np.array([0.8, 1.25])
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    gy = rng.normal(size=(B, H, W))
    gp, gm, gg = oracle.fuse_backward("d4", pan, gain, gy)
    Hc, Hr = lowpass_rows(oracle, "d4", H), lowpass_rows(oracle, "d4", W)
    L = lambda y: Hc @ y @ Hr.T
    LT = lambda c: Hc.T @ c @ Hr
    D = pan - LT(L(pan))
    for b in range(B):
        assert np.abs(gm[b] - L(gy[b])).max() < 1e-12
        assert abs(gg[b] - (gy[b] * D).sum()) < 1e-9
    ref = sum(gain[b] * (gy[b] - LT(L(gy[b]))) for b in range(B))
    assert np.abs(gp - ref).max() < 1e-12


@pytest.mark.parametrize("wavelet", ["d4", "haar"])
def test_mse_finite_differences_32x32(oracle, wavelet):
    rng = np.random.default_rng(32)
    H = W = 32
    B = 4
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    ms = rng.integers(0, 256, (B, 16, 16)).astype(np.float64)
    gain = np.ones(B)
    target = pan[None] * rng.uniform(0.8, 1.2, B)[:, None, None]
    count = B * H * W

    def loss(p, m, g):
        return ((oracle.fuse(wavelet, p, m, g) - target) ** 2).sum() / count

    out = oracle.fuse(wavelet, pan, ms, gain)
    gy = 2.0 * (out - target) / count
    gp, gm, gg = oracle.fuse_backward(wavelet, pan, gain, gy)
    eps = 0.5
    for _ in range(6):
        y, x = rng.integers(0, H, 2)
        d = np.zeros_like(pan)
        d[y, x] = eps
        fd = (loss(pan + d, ms, gain) - loss(pan - d, ms, gain)) / (2 * eps)
        assert abs(fd - gp[y, x]) < 1e-10
        b, i, j = rng.integers(0, B), rng.integers(0, 16), rng.integers(0, 16)
        d = np.zeros_like(ms)
        d[b, i, j] = eps
        fd = (loss(pan, ms + d, gain) - loss(pan, ms - d, gain)) / (2 * eps)
        assert abs(fd - gm[b, i, j]) < 1e-10
    for b in range(B):
        e = np.zeros(B)
        e[b] = 1e-3
        fd = (loss(pan, ms, gain + e) - loss(pan, ms, gain - e)) / 2e-3
        assert abs(fd - gg[b]) < 1e-7 * max(1.0, abs(gg[b]))
