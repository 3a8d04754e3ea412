"""Seeded synthetic PAN/MS scenes shaped like the paper's Landsat-7 workloads.

The paper fuses Landsat-7 scenes of the Donetsk region (section 4); those are
not available here, so every workload is synthetic.  This module only draws
inputs: it contains none of the wavelet arithmetic and is shared by the tests
and the benchmark.

Recipe (all counts and noise levels fixed; amplitudes are this project's
choice):

* PAN = clip(rint(110 + sum of 20 Gaussian blobs + sum of 10 rectangles +
  N(0, 3)), 0, 255), stored as float32 holding integers.
  - blob: amplitude U(-70, 110), sigma U(0.02, 0.12) * min(H, W), centre
    uniform over the image, separable exp(-dx^2/2s^2) * exp(-dy^2/2s^2);
  - rectangle: top-left uniform, height U(0.03, 0.25) * H, width
    U(0.03, 0.25) * W, additive level U(-60, 60) (sharp edges exercise the
    detail bands).
* MS band b = clip(rint(box2x2_mean(PAN) * a_b + o_b + N(0, 2)), 0, 255) with
  a_b ~ U(gain_lo, gain_hi) and o_b ~ U(off_lo, off_hi).
* rint is round-half-to-even.

``device=None`` draws everything with numpy's PCG64.  With a torch device the
scene parameters still come from PCG64 (identical blobs, rectangles, gains and
offsets) but the per-pixel noise is drawn on the device by torch's generator
seeded with the same seed -- the same distribution, a different noise sample;
this is what large scenes use, since drawing 10^8 normals on the host is slow.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

SEED_BASE = 180300737


def seed_for(config_index: int, scene_index: int = 0) -> int:
    """seed = 180300737 + 1000 * config_index + scene_index."""
    return SEED_BASE + 1000 * config_index + scene_index


@dataclass
class SceneParams:
    H: int
    W: int
    B: int
    seed: int
    blobs: np.ndarray  # (20, 4): amplitude, sigma, cy, cx
    rects: np.ndarray  # (10, 5): y0, x0, h, w, level
    band_gain: np.ndarray  # (B,)
    band_offset: np.ndarray  # (B,)


def draw_params(H: int, W: int, B: int, seed: int, gain=(0.6, 1.4), offset=(-10.0, 10.0)) -> SceneParams:
    rng = np.random.Generator(np.random.PCG64(seed))
    m = min(H, W)
    blobs = np.stack([
        rng.uniform(-70.0, 110.0, 20),
        rng.uniform(0.02, 0.12, 20) * m,
        rng.uniform(0.0, H, 20),
        rng.uniform(0.0, W, 20),
    ], axis=1)
    rh = np.maximum(1, np.rint(rng.uniform(0.03, 0.25, 10) * H)).astype(np.int64)
    rw = np.maximum(1, np.rint(rng.uniform(0.03, 0.25, 10) * W)).astype(np.int64)
    y0 = rng.integers(0, H, 10)
    x0 = rng.integers(0, W, 10)
    lvl = rng.uniform(-60.0, 60.0, 10)
    rects = np.stack([y0, x0, rh, rw, lvl], axis=1).astype(np.float64)
    bg = rng.uniform(gain[0], gain[1], B)
    bo = rng.uniform(offset[0], offset[1], B) if offset is not None else np.zeros(B)
    return SceneParams(H, W, B, seed, blobs, rects, bg, bo)


def _pan_field_numpy(p: SceneParams, rng) -> np.ndarray:
    H, W = p.H, p.W
    yy = np.arange(H, dtype=np.float64)
    xx = np.arange(W, dtype=np.float64)
    f = np.full((H, W), 110.0, dtype=np.float64)
    for amp, sig, cy, cx in p.blobs:
        gy = np.exp(-((yy - cy) ** 2) / (2.0 * sig * sig))
        gx = np.exp(-((xx - cx) ** 2) / (2.0 * sig * sig))
        f += amp * np.outer(gy, gx)
    for y0, x0, h, w, lvl in p.rects:
        y0, x0, h, w = int(y0), int(x0), int(h), int(w)
        f[y0:min(H, y0 + h), x0:min(W, x0 + w)] += lvl
    f += rng.normal(0.0, 3.0, (H, W))
    return np.clip(np.rint(f), 0, 255).astype(np.float32)


def _ms_numpy(p: SceneParams, pan: np.ndarray, rng) -> np.ndarray:
    H2, W2 = p.H // 2, p.W // 2
    box = pan.astype(np.float64).reshape(H2, 2, W2, 2).mean(axis=(1, 3))
    ms = np.empty((p.B, H2, W2), dtype=np.float32)
    for b in range(p.B):
        v = box * p.band_gain[b] + p.band_offset[b] + rng.normal(0.0, 2.0, (H2, W2))
        ms[b] = np.clip(np.rint(v), 0, 255)
    return ms


def _scene_torch(p: SceneParams, device):
    import torch

    H, W = p.H, p.W
    gen = torch.Generator(device=device)
    gen.manual_seed(p.seed)
    yy = torch.arange(H, dtype=torch.float32, device=device)
    xx = torch.arange(W, dtype=torch.float32, device=device)
    f = torch.full((H, W), 110.0, dtype=torch.float32, device=device)
    for amp, sig, cy, cx in p.blobs:
        gy = torch.exp(-((yy - float(cy)) ** 2) / (2.0 * float(sig) ** 2))
        gx = torch.exp(-((xx - float(cx)) ** 2) / (2.0 * float(sig) ** 2))
        f.addr_(gy, gx, alpha=float(amp))
    for y0, x0, h, w, lvl in p.rects:
        y0, x0, h, w = int(y0), int(x0), int(h), int(w)
        f[y0:min(H, y0 + h), x0:min(W, x0 + w)] += float(lvl)
    f += 3.0 * torch.randn((H, W), generator=gen, device=device, dtype=torch.float32)
    pan = torch.clamp(torch.round(f), 0, 255)
    del f
    H2, W2 = H // 2, W // 2
    box = pan.view(H2, 2, W2, 2).mean(dim=(1, 3))
    ms = torch.empty((p.B, H2, W2), dtype=torch.float32, device=device)
    for b in range(p.B):
        v = box * float(p.band_gain[b]) + float(p.band_offset[b])
        v += 2.0 * torch.randn((H2, W2), generator=gen, device=device, dtype=torch.float32)
        ms[b] = torch.clamp(torch.round(v), 0, 255)
    return pan, ms


def make_scene(H: int, W: int, B: int, seed: int, gain=(0.6, 1.4), offset=(-10.0, 10.0), device=None):
    """Return (pan (H, W), ms (B, H/2, W/2)) float32, numpy or torch on ``device``."""
    if H % 2 or W % 2 or H < 2 or W < 2:
        raise ValueError("PAN sides must be even and >= 2")
    p = draw_params(H, W, B, seed, gain, offset)
    if device is None:
        rng = np.random.Generator(np.random.PCG64(seed + 0x5EED))
        pan = _pan_field_numpy(p, rng)
        return pan, _ms_numpy(p, pan, rng)
    return _scene_torch(p, device)


def make_truth(pan, H: int, W: int, B: int, seed: int, gain=(0.6, 1.4), offset=(-10.0, 10.0)):
    """Full-resolution reference of each MS band of the scene drawn with the
    same arguments: clip(rint(PAN * a_b + o_b), 0, 255), what a sensor with
    that band's response would record at PAN resolution (noise-free).  The
    MS band itself is this reference box-averaged 2x2 plus noise, so it is the
    target a fused band should reproduce.  ``pan`` is the scene's PAN (numpy
    or torch); the result has the same type and device, float32."""
    p = draw_params(H, W, B, seed, gain, offset)
    if isinstance(pan, np.ndarray):
        t = np.empty((B, H, W), dtype=np.float32)
        for b in range(B):
            t[b] = np.clip(np.rint(pan.astype(np.float64) * p.band_gain[b] + p.band_offset[b]), 0, 255)
        return t
    import torch

    t = torch.empty((B, H, W), dtype=torch.float32, device=pan.device)
    for b in range(B):
        t[b] = torch.clamp(torch.round(pan * float(p.band_gain[b]) + float(p.band_offset[b])), 0, 255)
    return t


def band_gains(H: int, W: int, B: int, seed: int, gain=(0.6, 1.4), offset=(-10.0, 10.0)) -> np.ndarray:
    """The per-band response a_b the scene's MS bands were drawn with."""
    return draw_params(H, W, B, seed, gain, offset).band_gain.copy()


# ---- the five workloads -------------------------------------------------

@dataclass
class Workload:
    name: str
    wavelet: str
    H: int
    W: int
    B: int
    seed: int
    gain: tuple = (0.6, 1.4)
    offset: Optional[tuple] = (-10.0, 10.0)

    def make(self, device=None):
        return make_scene(self.H, self.W, self.B, self.seed, self.gain, self.offset, device)

    def truth(self, pan):
        return make_truth(pan, self.H, self.W, self.B, self.seed, self.gain, self.offset)

    def band_gains(self):
        return band_gains(self.H, self.W, self.B, self.seed, self.gain, self.offset)


def haar_512() -> Workload:
    """Haar, PAN 512x512, 1 MS band (gain U(0.7, 1.3), no offset)."""
    return Workload("haar_512x512_b1", "haar", 512, 512, 1, seed_for(0), (0.7, 1.3), None)


def d4_8192() -> Workload:
    """Daubechies-4, PAN 8192x8192, 3 MS bands."""
    return Workload("d4_8192x8192_b3", "d4", 8192, 8192, 3, seed_for(1))


def landsat(wavelet: str) -> Workload:
    """Landsat-7-shaped scene: PAN 15872 rows x 14336 columns, 6 MS bands."""
    return Workload("landsat_15872x14336_b6_" + wavelet, wavelet, 15872, 14336, 6, seed_for(2))


@dataclass
class BatchScene:
    wavelet: str
    H: int
    W: int
    B: int
    seed: int


def uneven_batch(n: int = 96, config_index: int = 3, lo: int = 256, hi: int = 4096) -> List[BatchScene]:
    """n independent scenes: even sides log-uniform in [lo, hi] drawn per side
    (non-square allowed), 3-6 bands, Haar for even i and D4 for odd i."""
    rng = np.random.Generator(np.random.PCG64(seed_for(config_index, 999)))
    out = []
    for i in range(n):
        H = int(2 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 2))
        W = int(2 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 2))
        B = int(rng.integers(3, 7))
        out.append(BatchScene("haar" if i % 2 == 0 else "d4", H, W, B, seed_for(config_index, i)))
    return out


def grad_targets(B: int, seed: int):
    """Per-band target gains U(0.8, 1.2) for the differentiation workload."""
    rng = np.random.Generator(np.random.PCG64(seed + 0x7A6))
    return rng.uniform(0.8, 1.2, B)
