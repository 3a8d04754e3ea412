"""Host-side parts of bench.py (no GPU): the refusal of a multi-GPU run, the
algorithmic byte counts behind `roofline.achieved`, the oracle baseline's
row-strip sample, and the lookup of the committed HBM counters behind
`roofline.traffic` (only for the library build and launch shape they were
taken on)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("H,W,B", [(15872, 14336, 6), (8192, 8192, 3), (512, 512, 1), (2048, 2048, 4)])
def test_algorithmic_bytes(H, W, B):
    # per output pixel 5 + 4/B bytes in float32 (PAN once, MS once, outputs once)
    assert bench.algo_bytes(H, W, B) == H * W * (4 + 5 * B)
    assert bench.algo_bytes(H, W, B) / (B * H * W) == pytest.approx(5 + 4 / B)
    # 8-bit: 1/B + 1/4 + 1 bytes per output pixel
    assert bench.u8_bytes(H, W, B) / (B * H * W) == pytest.approx(1 / B + 0.25 + 1)


def test_headline_bytes_match_the_roofline_figure():
    assert bench.algo_bytes(15872, 14336, 6) == 7736393728


@pytest.mark.parametrize("H", [15872, 8192, 2048])
def test_oracle_sample_strips(H):
    strips = bench._strip_rows(H, 8, 248)
    assert len(strips) == 8
    for (a, b), nxt in zip(strips, strips[1:] + [(H + 1, H + 1)]):
        assert a % 2 == 0 and b - a == 248 and 0 <= a and b <= H and b <= nxt[0]


def test_traffic_lookup(tmp_path, monkeypatch):
    from paper_1803_00737_amd.build import build_id

    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"build_id": build_id(), "tiles": {
        "2 4 2 7 4 0 2": {"traffic_bytes_per_launch": 7.8e9},
        "4 4 2 3 6 0 0": {"traffic_bytes_per_launch": 8.3e9}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.read_traffic("2 4 2 7 4 0 2") == 7.8e9
    assert bench.read_traffic("4 4 2 3 6 0 0") == 8.3e9
    assert bench.read_traffic("1 1 1 1 1 0 0") is None  # a shape without counters
    assert bench.read_traffic(None) is None
    path.write_text(json.dumps({"build_id": "another", "tiles": {"2 4 2 7 4 0 2": {"traffic_bytes_per_launch": 1.0}}}))
    assert bench.read_traffic("2 4 2 7 4 0 2") is None  # counters of another build
