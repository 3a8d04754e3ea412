"""Shared helpers for the GPU tests (not collected: no test_ prefix)."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

D4_TOL = 1e-3  # max-abs on the 0-255 scale


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1803_00737_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdwtfuse.so is not built")
    return torch.device("cuda:0")


def say(*a):
    """Name the case before each GPU step (flushed, so it survives a crash)."""
    print("[gpu-case]", *a, flush=True)


def int_scene(rng, H, W, B):
    pan = rng.integers(0, 256, (H, W)).astype(np.float32)
    ms = rng.integers(0, 256, (B, H // 2, W // 2)).astype(np.float32)
    return pan, ms


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def strided_view(a: np.ndarray, dev, pad_cols: int, offset: int):
    """Device view of ``a`` whose rows have pitch (cols + pad_cols) and whose
    first element sits ``offset`` floats into the allocation."""
    shape = a.shape
    rows = int(np.prod(shape[:-1]))
    cols = shape[-1]
    pitch = cols + pad_cols
    base = torch.full((offset + rows * pitch + 8,), float("nan"), dtype=torch.float32, device=dev)
    v = base[offset:offset + rows * pitch].view(rows, pitch)[:, :cols]
    v.copy_(torch.from_numpy(np.ascontiguousarray(a).reshape(rows, cols)).to(dev))
    return v.view(*shape) if len(shape) == 2 else v.unflatten(0, shape[:-1])


def ulp_diff(a: np.ndarray, b: np.ndarray) -> int:
    ai = a.astype(np.float32).view(np.int32).astype(np.int64)
    bi = b.astype(np.float32).view(np.int32).astype(np.int64)
    ai = np.where(ai < 0, -(ai & 0x7FFFFFFF), ai)
    bi = np.where(bi < 0, -(bi & 0x7FFFFFFF), bi)
    return int(np.abs(ai - bi).max()) if ai.size else 0
