"""Plain FP64 CPU oracle for DWT-replacement pan-sharpening.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_1803_00737_amd``) never imports, links or calls it, and the two share
no code.

The arithmetic lives in ``dwt_oracle.c`` (plain C, FP64, each function citing
the equation it follows); this module only builds that file with gcc and
marshals numpy arrays through ctypes.  Method: section 2 of the paper --
forward 2D DWT of PAN (rows, then columns), approximation quadrant replaced by
an MS band, inverse 2D DWT (columns, then rows); Haar per Eq. 1-2 / 11-12,
Daubechies-4 with periodic wrap per Eq. 3-10 / 13-16.

Every function here is pinned by the ``-m "not gpu"`` tests against closed
forms, invariants, brute-force matrices and an FFT-based evaluation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "dwt_oracle.c")
LIB_PATH = os.path.join(_HERE, "libdwt_oracle.so")

HAAR = 0
D4 = 1
_WAVELETS = {"haar": HAAR, "d4": D4, HAAR: HAAR, D4: D4}

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``dwt_oracle.c`` into ``libdwt_oracle.so`` (gcc, -O2, no fast-math)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        lib.oracle_filters.argtypes = [dp, dp, dp, dp]
        for name in ("oracle_dwt1_fwd", "oracle_dwt1_inv", "oracle_dwt1_fwd_T", "oracle_dwt1_inv_T"):
            getattr(lib, name).argtypes = [ci, i64, dp, dp]
            getattr(lib, name).restype = ci
        for name in ("oracle_dwt2_fwd", "oracle_dwt2_inv"):
            getattr(lib, name).argtypes = [ci, i64, i64, dp, dp]
            getattr(lib, name).restype = ci
        lib.oracle_fuse.argtypes = [ci, i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_fuse.restype = ci
        lib.oracle_fuse_kappa.argtypes = [ci, i64, i64, i64, dp, dp, dp, ctypes.c_double, dp]
        lib.oracle_fuse_kappa.restype = ci
        lib.oracle_fuse_rows.argtypes = [ci, i64, i64, i64, dp, dp, dp, ctypes.c_double, i64, i64, dp]
        lib.oracle_fuse_rows.restype = ci
        lib.oracle_quantize_u8.argtypes = [i64, dp, ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_quantize_u8.restype = ci
        lib.oracle_quality.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_quality.restype = ci
        lib.oracle_fuse_point.argtypes = [ci, i64, i64, dp, dp, ctypes.c_double, i64, i64]
        lib.oracle_fuse_point.restype = ctypes.c_double
        lib.oracle_fuse_backward.argtypes = [ci, i64, i64, i64, dp, dp, dp, dp, dp, dp]
        lib.oracle_fuse_backward.restype = ci
        _lib = lib
        return lib


def _wav(w) -> int:
    try:
        return _WAVELETS[w]
    except KeyError:
        raise ValueError("unknown wavelet %r" % (w,))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s: invalid arguments (rc=%d)" % (what, rc))


def filters():
    """Return dict with h (Eq. 7-8), g (Eq. 9-10 as read), t and u (after Eq. 16)."""
    lib = _load()
    out = {k: np.zeros(4) for k in "hgtu"}
    lib.oracle_filters(_ptr(out["h"]), _ptr(out["g"]), _ptr(out["t"]), _ptr(out["u"]))
    return out


def _vec_op(name, w, v):
    lib = _load()
    v = _f64(v)
    out = np.empty_like(v)
    _check(getattr(lib, name)(_wav(w), v.shape[0], _ptr(v), _ptr(out)), name)
    return out


def dwt1_fwd(w, s):
    """1D forward transform, output [a | d] (Eq. 1-2 Haar, Eq. 3-6 D4)."""
    return _vec_op("oracle_dwt1_fwd", w, s)


def dwt1_inv(w, c):
    """1D inverse transform (Eq. 11-12 Haar, Eq. 13-16 D4)."""
    return _vec_op("oracle_dwt1_inv", w, c)


def dwt1_fwd_T(w, y):
    """Transpose of the 1D forward map."""
    return _vec_op("oracle_dwt1_fwd_T", w, y)


def dwt1_inv_T(w, y):
    """Transpose of the 1D inverse map."""
    return _vec_op("oracle_dwt1_inv_T", w, y)


def dwt2_fwd(w, x):
    """2D forward transform: rows, then columns (section 2)."""
    lib = _load()
    x = _f64(x)
    out = np.empty_like(x)
    _check(lib.oracle_dwt2_fwd(_wav(w), x.shape[0], x.shape[1], _ptr(x), _ptr(out)), "dwt2_fwd")
    return out


def dwt2_inv(w, X):
    """2D inverse transform: columns, then rows (section 2)."""
    lib = _load()
    X = _f64(X)
    out = np.empty_like(X)
    _check(lib.oracle_dwt2_inv(_wav(w), X.shape[0], X.shape[1], _ptr(X), _ptr(out)), "dwt2_inv")
    return out


def _gain(gain, B):
    if gain is None:
        return None
    g = _f64(gain).reshape(-1)
    if g.shape[0] != B:
        raise ValueError("gain must have B=%d entries" % B)
    return g


def fuse(w, pan, ms, gain=None, kappa=1.0):
    """Fused images (B, H, W) float64 for PAN (H, W) and MS (B, H/2, W/2);
    the MS band replaces LL multiplied by ``kappa`` (1 = as printed)."""
    lib = _load()
    pan = _f64(pan)
    ms = _f64(ms)
    if ms.ndim == 2:
        ms = ms[None]
    H, W = pan.shape
    B = ms.shape[0]
    if ms.shape[1:] != (H // 2, W // 2):
        raise ValueError("ms must be (B, H/2, W/2)")
    g = _gain(gain, B)
    out = np.empty((B, H, W), dtype=np.float64)
    if kappa == 1.0:
        _check(lib.oracle_fuse(_wav(w), H, W, B, _ptr(pan), _ptr(ms), _ptr(g), _ptr(out)), "fuse")
    else:
        _check(lib.oracle_fuse_kappa(_wav(w), H, W, B, _ptr(pan), _ptr(ms), _ptr(g), float(kappa), _ptr(out)),
               "fuse_kappa")
    return out


def fuse_rows(w, pan, ms, row0, row1, gain=None, kappa=1.0):
    """Rows row0 .. row1-1 of ``fuse(w, pan, ms, gain, kappa)``, (B, row1-row0, W)
    float64, equal to those rows of the whole-image result bit for bit; only
    the rows they need are transformed."""
    lib = _load()
    pan = _f64(pan)
    ms = _f64(ms)
    if ms.ndim == 2:
        ms = ms[None]
    H, W = pan.shape
    B = ms.shape[0]
    if ms.shape[1:] != (H // 2, W // 2):
        raise ValueError("ms must be (B, H/2, W/2)")
    if not 0 <= row0 <= row1 <= H:
        raise ValueError("need 0 <= row0 <= row1 <= H")
    g = _gain(gain, B)
    out = np.empty((B, row1 - row0, W), dtype=np.float64)
    _check(lib.oracle_fuse_rows(_wav(w), H, W, B, _ptr(pan), _ptr(ms), _ptr(g), float(kappa), int(row0), int(row1),
                                _ptr(out)), "fuse_rows")
    return out


def dc_kappa(w) -> float:
    """kappa that matches the DC gain of the analysis LL, (sum of the
    low-pass taps)^2: 2 for D4 (the taps of Eq. 7-8 sum to sqrt 2), 1 for the
    divided-by-2 Haar of Eq. 1-2."""
    return 2.0 if _wav(w) == D4 else 1.0


def quality(fused, ref):
    """Per-band quality of fused (B, H, W) against ref (B, H, W): dict with
    sse, sum_ref (arrays of B), rmse, mean and the ERGAS-style score
    100 * (1/2) * sqrt(mean_b (rmse_b / mean_b)^2) (PAN pixels half the MS
    pixel size, section 2)."""
    lib = _load()
    f = _f64(fused)
    r = _f64(ref)
    if f.ndim == 2:
        f, r = f[None], r[None]
    if f.shape != r.shape:
        raise ValueError("fused and ref must have the same shape")
    B, H, W = f.shape
    sse = np.empty(B)
    sr = np.empty(B)
    _check(lib.oracle_quality(H, W, B, _ptr(f), _ptr(r), _ptr(sse), _ptr(sr)), "quality")
    n = float(H * W)
    rmse = np.sqrt(sse / n)
    mean = sr / n
    return {"sse": sse, "sum_ref": sr, "rmse": rmse, "mean": mean,
            "ergas": 100.0 * 0.5 * float(np.sqrt(np.mean((rmse / mean) ** 2)))}


def quantize_u8(v):
    """8-bit code of each value: nearest integer, ties to even, clamped to
    [0, 255], NaN -> 0 (section 3's 8-bit image representation)."""
    lib = _load()
    v = _f64(v)
    out = np.empty(v.shape, dtype=np.uint8)
    _check(lib.oracle_quantize_u8(v.size, _ptr(v), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
           "quantize_u8")
    return out


def fuse_point(w, pan, ms_band, gain, y, x):
    """One fused pixel (y, x) for one MS band, FP64."""
    lib = _load()
    pan = _f64(pan)
    ms_band = _f64(ms_band)
    H, W = pan.shape
    return lib.oracle_fuse_point(_wav(w), H, W, _ptr(pan), _ptr(ms_band), float(gain), int(y), int(x))


def fuse_points(w, pan, ms, gain, bands, ys, xs):
    """Fused pixels at (band, y, x) triples; pan/ms already float64 contiguous."""
    lib = _load()
    pan = _f64(pan)
    ms = _f64(ms)
    H, W = pan.shape
    H2, W2 = H // 2, W // 2
    wv = _wav(w)
    g = np.ones(ms.shape[0]) if gain is None else np.asarray(gain, dtype=np.float64)
    pp = _ptr(pan)
    out = np.empty(len(ys), dtype=np.float64)
    base = ms.ctypes.data
    dp = ctypes.POINTER(ctypes.c_double)
    for k, (b, y, x) in enumerate(zip(bands, ys, xs)):
        mptr = ctypes.cast(base + int(b) * H2 * W2 * 8, dp)
        out[k] = lib.oracle_fuse_point(wv, H, W, pp, mptr, float(g[int(b)]), int(y), int(x))
    return out


def fuse_backward(w, pan, gain, grad_out):
    """Transpose of the fusion map: (grad_pan, grad_ms, grad_gain), FP64."""
    lib = _load()
    pan = _f64(pan)
    go = _f64(grad_out)
    if go.ndim == 2:
        go = go[None]
    B, H, W = go.shape
    g = _gain(gain, B)
    gp = np.empty((H, W))
    gm = np.empty((B, H // 2, W // 2))
    gg = np.empty(B)
    _check(lib.oracle_fuse_backward(_wav(w), H, W, B, _ptr(pan), _ptr(g), _ptr(go),
                                    _ptr(gp), _ptr(gm), _ptr(gg)), "fuse_backward")
    return gp, gm, gg
