"""Pins of the oracle's 1D and 2D transforms (Eq. 1-6 forward, Eq. 11-16
inverse, section 2 row/column order).

Independent evaluations used here:
  * the D4 forward transform as a circular correlation computed with numpy's
    FFT (a_i = sum_k h_k s_{(2i+k) mod N}, periodic extension);
  * hand-computed Haar values;
  * dense matrices built from unit impulses (orthogonality, inverse =
    transpose, Haar synthesis * analysis = identity);
  * closed forms for constant and linear inputs and shift equivariance.
"""
import math

import numpy as np
import pytest

SIZES = [2, 4, 6, 8, 34, 256]


def fft_forward(filters, wavelet, s):
    """a_i = sum_k h_k s_{(2i+k) mod N}, d_i likewise with g, via the FFT."""
    s = np.asarray(s, dtype=np.float64)
    N = s.shape[0]
    if wavelet == "haar":
        h, g = np.array([0.5, 0.5]), np.array([0.5, -0.5])
    else:
        h, g = filters["h"], filters["g"]

    def corr(f):
        fp = np.zeros(N)
        for k, v in enumerate(f):
            fp[k % N] += v
        return np.real(np.fft.ifft(np.fft.fft(s) * np.conj(np.fft.fft(fp))))

    return np.concatenate([corr(h)[0::2], corr(g)[0::2]])


def matrix_of(fn, N):
    return np.stack([fn(np.eye(N)[j]) for j in range(N)], axis=1)


def test_haar_hand_values(oracle):
    # Eq. 1-2 on [1, 3, 5, 7]: a = [(1+3)/2, (5+7)/2], d = [(1-3)/2, (5-7)/2]
    assert list(oracle.dwt1_fwd("haar", [1, 3, 5, 7])) == [2.0, 6.0, -1.0, -1.0]
    # Eq. 11-12: s_2i = a_i + d_i, s_2i+1 = a_i - d_i
    assert list(oracle.dwt1_inv("haar", [2, 6, -1, -1])) == [1.0, 3.0, 5.0, 7.0]
    assert list(oracle.dwt1_fwd("haar", [4, 4])) == [4.0, 0.0]


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_forward_matches_fft_correlation(oracle, wavelet, N):
    rng = np.random.default_rng(N)
    s = rng.integers(0, 256, N).astype(np.float64)
    ref = fft_forward(oracle.filters(), wavelet, s)
    np.testing.assert_allclose(oracle.dwt1_fwd(wavelet, s), ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("N", SIZES)
def test_perfect_reconstruction_1d(oracle, N):
    rng = np.random.default_rng(100 + N)
    s = rng.integers(0, 256, N).astype(np.float64)
    assert np.array_equal(oracle.dwt1_inv("haar", oracle.dwt1_fwd("haar", s)), s)
    assert np.abs(oracle.dwt1_inv("d4", oracle.dwt1_fwd("d4", s)) - s).max() < 1e-12


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_d4_matrix_orthogonal_and_inverse_is_transpose(oracle, N):
    Wf = matrix_of(lambda v: oracle.dwt1_fwd("d4", v), N)
    Wi = matrix_of(lambda v: oracle.dwt1_inv("d4", v), N)
    assert np.abs(Wf @ Wf.T - np.eye(N)).max() < 1e-15
    assert np.abs(Wi - Wf.T).max() < 1e-16  # Eq. 13-16 are exactly the transpose of Eq. 3-6


@pytest.mark.parametrize("N", [2, 4, 8])
def test_haar_matrices(oracle, N):
    A = matrix_of(lambda v: oracle.dwt1_fwd("haar", v), N)
    S = matrix_of(lambda v: oracle.dwt1_inv("haar", v), N)
    assert np.array_equal(S @ A, np.eye(N))
    assert np.array_equal(S, 2 * A.T)  # /2 normalisation: not orthonormal
    half = N // 2
    for i in range(half):
        assert A[i, 2 * i] == A[i, 2 * i + 1] == 0.5
        assert A[half + i, 2 * i] == 0.5 and A[half + i, 2 * i + 1] == -0.5


def test_d4_length_two_is_orthonormal_haar(oracle):
    s = np.array([3.0, 7.0])
    a, d = oracle.dwt1_fwd("d4", s)
    assert abs(a - 10 / math.sqrt(2)) < 1e-14 and abs(d + 4 / math.sqrt(2)) < 1e-14


@pytest.mark.parametrize("N", [4, 8, 34])
def test_d4_constant_and_ramp(oracle, N):
    c = oracle.dwt1_fwd("d4", np.full(N, 5.0))
    assert np.abs(c[: N // 2] - 5.0 * math.sqrt(2)).max() < 1e-13
    assert np.abs(c[N // 2:]).max() < 1e-13
    ramp = oracle.dwt1_fwd("d4", 3.0 + 0.5 * np.arange(N))
    d = ramp[N // 2:]
    assert np.abs(d[:-1]).max() < 1e-13  # interior detail of a ramp vanishes
    assert abs(d[-1]) > 1e-3  # the wrap-around element (Eq. 6) sees the jump


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_transposes_1d(oracle, wavelet):
    N = 10
    for fn, fnT in ((oracle.dwt1_fwd, oracle.dwt1_fwd_T), (oracle.dwt1_inv, oracle.dwt1_inv_T)):
        M = matrix_of(lambda v: fn(wavelet, v), N)
        MT = matrix_of(lambda v: fnT(wavelet, v), N)
        assert np.abs(MT - M.T).max() < 1e-16


def test_d4_shift_equivariance_1d(oracle):
    rng = np.random.default_rng(7)
    N = 16
    s = rng.normal(size=N)
    c0 = oracle.dwt1_fwd("d4", s)
    c1 = oracle.dwt1_fwd("d4", np.roll(s, -2))
    h = N // 2
    assert np.abs(c1[:h] - np.roll(c0[:h], -1)).max() < 1e-14
    assert np.abs(c1[h:] - np.roll(c0[h:], -1)).max() < 1e-14


# ---- 2D -----------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(2, 2), (4, 6), (6, 10), (34, 8), (16, 16)])
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_2d_is_rows_then_columns_fft(oracle, wavelet, H, W):
    """X = Wc x Wr^T with both 1D matrices built from the FFT evaluation."""
    f = oracle.filters()
    Wr = matrix_of(lambda v: fft_forward(f, wavelet, v), W)
    Wc = matrix_of(lambda v: fft_forward(f, wavelet, v), H)
    rng = np.random.default_rng(H * 100 + W)
    x = rng.integers(0, 256, (H, W)).astype(np.float64)
    np.testing.assert_allclose(oracle.dwt2_fwd(wavelet, x), Wc @ x @ Wr.T, rtol=0, atol=1e-10)


@pytest.mark.parametrize("H,W", [(2, 2), (4, 6), (6, 10), (34, 8), (64, 48)])
def test_perfect_reconstruction_2d(oracle, H, W):
    rng = np.random.default_rng(H + W)
    x = rng.integers(0, 256, (H, W)).astype(np.float64)
    assert np.array_equal(oracle.dwt2_inv("haar", oracle.dwt2_fwd("haar", x)), x)
    assert np.abs(oracle.dwt2_inv("d4", oracle.dwt2_fwd("d4", x)) - x).max() < 1e-11


def test_2d_flat_image(oracle):
    x = np.full((8, 12), 37.0)
    Xh = oracle.dwt2_fwd("haar", x)
    assert np.array_equal(Xh[:4, :6], np.full((4, 6), 37.0))
    Xh[:4, :6] = 0
    assert not Xh.any()
    Xd = oracle.dwt2_fwd("d4", x)
    assert np.abs(Xd[:4, :6] - 74.0).max() < 1e-12  # LL gain (sum h)^2 = 2
    Xd[:4, :6] = 0
    assert np.abs(Xd).max() < 1e-12


def test_bruteforce_8x8_dense(oracle):
    n = 64

    def dense(fn):
        return np.stack([fn(np.eye(n)[j].reshape(8, 8)).reshape(-1) for j in range(n)], axis=1)

    Wd = dense(lambda v: oracle.dwt2_fwd("d4", v))
    Wdi = dense(lambda v: oracle.dwt2_inv("d4", v))
    assert np.abs(Wd @ Wd.T - np.eye(n)).max() < 1e-14
    assert np.abs(Wdi - Wd.T).max() < 1e-15
    A = dense(lambda v: oracle.dwt2_fwd("haar", v))
    S = dense(lambda v: oracle.dwt2_inv("haar", v))
    assert np.array_equal(S @ A, np.eye(n))


def test_invalid_sizes_rejected(oracle):
    with pytest.raises(ValueError):
        oracle.dwt1_fwd("d4", np.zeros(5))
    with pytest.raises(ValueError):
        oracle.dwt2_fwd("haar", np.zeros((3, 4)))
    with pytest.raises(ValueError):
        oracle.dwt1_fwd("d4", np.zeros(0))
