"""The paper's multi-pass GPU pipeline (section 3, comparator): parity with
the oracle (Haar bit-exact, D4 <= 1e-3) and with the fused kernels."""
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


@pytest.mark.parametrize("H,W", [(2, 2), (4, 6), (34, 70), (130, 258), (64, 1288), (66, 4070)])
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_multipass_matches_oracle_and_fused(dev, fz, oracle, wavelet, H, W):
    rng = np.random.default_rng(H * 31 + W)
    pan, ms = int_scene(rng, H, W, 3)
    say("multipass", wavelet, H, W)
    got = fz.fuse_multipass(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    ref = oracle.fuse(wavelet, pan.astype(np.float64), ms.astype(np.float64))
    fused = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    if wavelet == "haar":
        assert np.array_equal(got, ref.astype(np.float32))
        assert np.array_equal(got, fused)
    else:
        assert np.abs(got - ref).max() <= D4_TOL
        assert np.abs(got - fused).max() <= D4_TOL


def test_multipass_pitched(dev, fz, oracle):
    rng = np.random.default_rng(4)
    pan, ms = int_scene(rng, 34, 70, 2)
    say("multipass pitched")
    out = strided_view(np.zeros((2, 34, 70), np.float32), dev, 6, 0)
    fz.fuse_multipass(strided_view(pan, dev, 2, 2), strided_view(ms, dev, 3, 1), "d4", out=out)
    ref = oracle.fuse("d4", pan.astype(np.float64), ms.astype(np.float64))
    assert np.abs(out.cpu().numpy() - ref).max() <= D4_TOL
