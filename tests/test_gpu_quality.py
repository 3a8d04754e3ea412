"""GPU quality diagnostics (dwt_fuse_quality) against the oracle's sums, and
the DC-matched D4 study: on a synthetic scene whose MS bands are the 2x2
box average of a known full-resolution truth (plus noise), kappa = 2 brings
D4's fused bands back to the truth's mean level while kappa = 1 halves it.

Bars: sse and sum_ref within 1e-12 relative of the oracle's FP64 sums
(different summation order over float32 inputs converted exactly), the
GPU-formed RMSE and means likewise and the ERGAS-style score within 1e-9; the
fused-vs-truth RMSE of each kernel path within 1e-4 relative of the oracle's
(the fused values themselves differ by at most 1e-3)."""
import numpy as np
import pytest

from gpu_helpers import require_gpu, say, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


@pytest.mark.parametrize("B,H,W", [(1, 1, 1), (3, 17, 9), (2, 300, 1030), (4, 1024, 2048), (1, 5000, 3)])
def test_sums_match_oracle(dev, fz, oracle, B, H, W):
    rng = np.random.default_rng(B + H + W)
    f = rng.normal(100, 30, (B, H, W)).astype(np.float32)
    r = rng.normal(100, 30, (B, H, W)).astype(np.float32)
    say("quality", B, H, W)
    q = fz.quality(to_dev(f, dev), to_dev(r, dev))
    ref = oracle.quality(f.astype(np.float64), r.astype(np.float64))
    got_sse = q["sse"].cpu().numpy()
    got_sr = q["sum_ref"].cpu().numpy()
    assert np.allclose(got_sse, ref["sse"], rtol=1e-12, atol=0)
    assert np.allclose(got_sr, ref["sum_ref"], rtol=1e-12, atol=1e-9)
    # the scores are formed on the GPU (dwt_fuse_quality_scores) from its sums
    assert np.allclose(q["rmse"], ref["rmse"], rtol=1e-12, atol=0)
    assert np.allclose(q["mean"], ref["mean"], rtol=1e-12, atol=1e-12)
    assert abs(q["ergas"] - ref["ergas"]) <= 1e-9 * ref["ergas"]
    # fixed order: a second call gives the same bits
    q2 = fz.quality(to_dev(f, dev), to_dev(r, dev))
    assert torch.equal(q["sse"], q2["sse"]) and torch.equal(q["sum_ref"], q2["sum_ref"])


def test_score_zero_mean_band(dev, fz, oracle):
    """A reference band with mean 0 makes the ERGAS-style score +inf on the
    GPU as in the oracle; the other bands' RMSE and means stay finite."""
    rng = np.random.default_rng(5)
    f = rng.normal(10, 3, (2, 16, 24)).astype(np.float32)
    r = np.stack([rng.normal(10, 3, (16, 24)), np.zeros((16, 24))]).astype(np.float32)
    say("quality zero mean")
    q = fz.quality(to_dev(f, dev), to_dev(r, dev))
    with np.errstate(divide="ignore"):  # rmse / 0 in the oracle's score
        ref = oracle.quality(f.astype(np.float64), r.astype(np.float64))
    assert q["ergas"] == float("inf") and ref["ergas"] == float("inf")
    assert np.allclose(q["rmse"], ref["rmse"], rtol=1e-12) and q["mean"][1] == 0.0


@pytest.mark.parametrize("cols", [(5, 55, 1, 51), (4, 68, 8, 72)])
def test_pitched_inputs(dev, fz, oracle, cols):
    """Pitched views: odd offsets take the scalar loop, 16-byte aligned rows
    of a width divisible by 4 the vector loop."""
    rng = np.random.default_rng(3)
    big_f = to_dev(rng.normal(0, 1, (3, 40, 80)).astype(np.float32), dev)
    big_r = to_dev(rng.normal(0, 1, (3, 40, 80)).astype(np.float32), dev)
    f0, f1, r0, r1 = cols
    f, r = big_f[:, 4:34, f0:f1], big_r[:, 8:38, r0:r1]
    say("quality pitched", cols)
    q = fz.quality(f, r)
    ref = oracle.quality(f.cpu().numpy().astype(np.float64), r.cpu().numpy().astype(np.float64))
    assert np.allclose(q["sse"].cpu().numpy(), ref["sse"], rtol=1e-12)
    assert np.allclose(q["sum_ref"].cpu().numpy(), ref["sum_ref"], rtol=1e-12, atol=1e-9)


def test_dc_matched_d4(dev, fz, oracle):
    from paper_1803_00737_amd import synth

    H = W = 512
    B = 3
    seed = synth.seed_for(1, 77)
    pan, ms = synth.make_scene(H, W, B, seed)
    truth = synth.make_truth(pan, H, W, B, seed)
    p, m, t = to_dev(pan, dev), to_dev(ms, dev), to_dev(truth, dev)
    res = {}
    for name, w, kappa in [("d4_k1", "d4", 1.0), ("d4_k2", "d4", 2.0), ("haar", "haar", 1.0)]:
        say("dc matched", name)
        out = fz.fuse(p, m, w, kappa=kappa)
        q = fz.quality(out, t)
        ref = oracle.quality(oracle.fuse(w, pan, ms, kappa=kappa), truth)
        assert np.allclose(q["rmse"], ref["rmse"], rtol=1e-4)
        res[name] = q
    # kappa = 1 D4 loses half the mean level; kappa = 2 keeps it
    for b in range(B):
        assert res["d4_k2"]["rmse"][b] < 0.25 * res["d4_k1"]["rmse"][b]
    assert res["d4_k2"]["ergas"] < 0.25 * res["d4_k1"]["ergas"]
