"""Python surface over the C ABI: ``fuse``, ``fuse_batched``, ``fuse_backward``
and ``DwtFuseFn`` (torch.autograd.Function).

Every step of the computation runs in the HIP library; this module only
checks tensor placement/dtype, allocates outputs with torch and passes
pointers, pitches and the current HIP stream.  Tensors must be float32 on a
GPU with unit stride along rows; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import threading
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import BwdItem, DwtFuseError, Item, wavelet_id


class Context:
    """One dwt_fuse_ctx (device + stream + workspace + tuning table)."""

    def __init__(self, device: int):
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self.lib.dwt_fuse_create(ctypes.byref(h), self.device, None)
        if st != 0:
            raise DwtFuseError(st, "dwt_fuse_create")
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.lib.dwt_fuse_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def check(self, st: int, where: str):
        if st != 0:
            detail = self.lib.dwt_fuse_last_error(self.handle) or b""
            raise DwtFuseError(st, where, detail.decode(errors="replace"))

    def bind_stream(self, stream: Optional[torch.cuda.Stream] = None):
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.check(self.lib.dwt_fuse_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)),
                   "dwt_fuse_set_stream")

    def set_tuning(self, enable: bool = True):
        self.check(self.lib.dwt_fuse_set_tuning(self.handle, 1 if enable else 0), "dwt_fuse_set_tuning")

    def force_tile(self, seg_rows: int = 0, waves_per_block: int = 0, cols_per_lane: int = 0, variant: int = 0):
        """Force the launch shape (0 = automatic); variant 1 = rolling, 2 = one-shot."""
        self.check(self.lib.dwt_fuse_force_tile(self.handle, seg_rows, waves_per_block, cols_per_lane, variant),
                   "dwt_fuse_force_tile")

    def force_band_split(self, bands_per_unit: int = 0):
        """LDS-staged D4: bands per work unit (0 = automatic)."""
        self.check(self.lib.dwt_fuse_force_band_split(self.handle, bands_per_unit), "dwt_fuse_force_band_split")

    def force_order(self, order: int = -1):
        """Unit order of forward and adjoint launches (-1 = automatic): bit 0
        row bands (else column strips), bit 1 dispatch order (else per-XCD runs)."""
        self.check(self.lib.dwt_fuse_force_order(self.handle, order), "dwt_fuse_force_order")

    def tune_save(self, path: str):
        self.check(self.lib.dwt_fuse_tune_save(self.handle, path.encode()), "dwt_fuse_tune_save")

    def tune_load(self, path: str):
        self.check(self.lib.dwt_fuse_tune_load(self.handle, path.encode()), "dwt_fuse_tune_load")


_ctx_lock = threading.Lock()
_contexts = {}


def context(device=None) -> Context:
    """The shared context of a device (created on first use)."""
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    with _ctx_lock:
        c = _contexts.get(device)
        if c is None:
            c = _contexts[device] = Context(device)
        return c


_FORMATS = {torch.float32: _lib.F32, torch.uint8: _lib.U8}


def _require(t: torch.Tensor, name: str, ndim: int, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on a GPU (there is no CPU path)" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.dim() != ndim:
        raise ValueError("%s must have %d dimensions, got shape %s" % (name, ndim, tuple(t.shape)))


def _rows_unit(t: torch.Tensor) -> torch.Tensor:
    """Tensor with unit stride along its last dimension (pitches may be anything)."""
    if t.stride(-1) != 1 or any(s < 0 for s in t.stride()):
        t = t.contiguous()
    return t


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _pitch(t: torch.Tensor, dim: int) -> int:
    # A size-1 dimension may report any stride; use the dense value then.
    if t.shape[dim] == 1:
        n = 1
        for s in t.shape[dim + 1:]:
            n *= s
        return max(n, t.stride(dim))
    return t.stride(dim)


def _prep_scene(pan, ms, gain, out, out_dtype=torch.float32, allow_u8=False):
    u8 = allow_u8 and isinstance(pan, torch.Tensor) and pan.dtype == torch.uint8
    in_dtype = torch.uint8 if u8 else torch.float32
    _require(pan, "pan", 2, in_dtype)
    if ms.dim() == 2:
        ms = ms.unsqueeze(0)
    _require(ms, "ms", 3, in_dtype)
    pan = _rows_unit(pan)
    ms = _rows_unit(ms)
    H, W = pan.shape
    B = ms.shape[0]
    if tuple(ms.shape[1:]) != (H // 2, W // 2):
        raise ValueError("ms must be (B, H/2, W/2) = (B, %d, %d), got %s" % (H // 2, W // 2, tuple(ms.shape)))
    if ms.device != pan.device:
        raise ValueError("pan and ms must be on the same device")
    if gain is not None:
        _require(gain, "gain", 1)
        gain = gain.contiguous()
        if gain.shape[0] != B:
            raise ValueError("gain must have B=%d entries" % B)
        if gain.device != pan.device:
            raise ValueError("gain must be on the device of pan")
    if out is None:
        out = torch.empty((B, H, W), dtype=out_dtype, device=pan.device)
    else:
        _require(out, "out", 3, out_dtype)
        if tuple(out.shape) != (B, H, W):
            raise ValueError("out must be (B, H, W)")
        if out.device != pan.device:
            raise ValueError("out must be on the device of pan")
        if out.stride(-1) != 1:
            raise ValueError("out must have unit stride along rows")
    return pan, ms, gain, out, H, W, B


def fuse(pan: torch.Tensor, ms: torch.Tensor, wavelet="d4", gain: Optional[torch.Tensor] = None,
         out: Optional[torch.Tensor] = None, out_dtype=None, kappa: float = 1.0) -> torch.Tensor:
    """Fused bands (B, H, W) for PAN (H, W) and MS (B, H/2, W/2) (or (H/2, W/2)).

    Section 2 of the paper: forward 2D DWT of PAN, LL quadrant replaced by each
    MS band, inverse 2D DWT (Haar Eq. 1-2/11-12 or D4 Eq. 3-16 with wrap).
    ``gain`` (B,) scales the PAN detail quadrants per band (None = 1).

    pan/ms may be float32 or uint8 (8-bit pixels); ``out_dtype`` float32 or
    uint8 (nearest integer, ties to even, clamped to [0, 255]; default: the
    dtype of ``out`` if given, else float32).  ``kappa`` scales the MS band where
    it replaces LL (1 = as printed, 2 = DC-matched D4)."""
    if out_dtype is None:
        out_dtype = out.dtype if isinstance(out, torch.Tensor) else torch.float32
    if out_dtype not in _FORMATS:
        raise TypeError("out_dtype must be float32 or uint8, got %s" % (out_dtype,))
    pan, ms, gain, out, H, W, B = _prep_scene(pan, ms, gain, out, out_dtype, allow_u8=True)
    c = context(pan.device)
    c.bind_stream()
    if pan.dtype == torch.float32 and out_dtype == torch.float32 and float(kappa) == 1.0:
        st = c.lib.dwt_fuse_run(c.handle, wavelet_id(wavelet), H, W, B,
                                _ptr(pan), _pitch(pan, 0), _ptr(ms), _pitch(ms, 1), _pitch(ms, 0),
                                _ptr(gain), _ptr(out), _pitch(out, 1), _pitch(out, 0))
        c.check(st, "dwt_fuse_run")
        return out
    opts = _lib.Opts(_FORMATS[pan.dtype], _FORMATS[out_dtype], float(kappa))
    st = c.lib.dwt_fuse_run_ex(c.handle, wavelet_id(wavelet), H, W, B,
                               _ptr(pan), _pitch(pan, 0), _ptr(ms), _pitch(ms, 1), _pitch(ms, 0),
                               _ptr(gain), _ptr(out), _pitch(out, 1), _pitch(out, 0), ctypes.byref(opts))
    c.check(st, "dwt_fuse_run_ex")
    return out


def quality(fused: torch.Tensor, ref: torch.Tensor) -> dict:
    """Quality of fused bands (B, H, W) against reference bands of the same
    shape (e.g. a synthetic full-resolution truth), float32 on the GPU.

    The per-band sums (squared error, reference) are reduced on the GPU in
    FP64 and the scores formed from them there (dwt_fuse_quality_scores);
    returns dict with ``sse``, ``sum_ref`` (float64 tensors of B, on the
    device), ``rmse`` and ``mean`` (lists), and ``ergas`` =
    100 * (1/2) * sqrt(mean_b (rmse_b / mean_b)^2) for the 1:2 PAN:MS pixel
    size of section 2."""
    if fused.dim() == 2:
        fused = fused.unsqueeze(0)
    if ref.dim() == 2:
        ref = ref.unsqueeze(0)
    _require(fused, "fused", 3)
    _require(ref, "ref", 3)
    if fused.shape != ref.shape:
        raise ValueError("fused and ref must have the same shape, got %s and %s"
                         % (tuple(fused.shape), tuple(ref.shape)))
    fused, ref = _rows_unit(fused), _rows_unit(ref)
    B, H, W = fused.shape
    out = torch.empty(4 * B + 1, dtype=torch.float64, device=fused.device)
    c = context(fused.device)
    c.bind_stream()
    st = c.lib.dwt_fuse_quality_scores(c.handle, H, W, B, _ptr(fused), _pitch(fused, 1), _pitch(fused, 0),
                                       _ptr(ref), _pitch(ref, 1), _pitch(ref, 0), _ptr(out))
    c.check(st, "dwt_fuse_quality_scores")
    host = out.cpu().tolist()
    return {"sse": out[:B], "sum_ref": out[B:2 * B], "rmse": host[2 * B:3 * B], "mean": host[3 * B:4 * B],
            "ergas": host[4 * B]}


def fuse_multipass(pan: torch.Tensor, ms: torch.Tensor, wavelet="d4", out: Optional[torch.Tensor] = None):
    """The paper's per-channel multi-pass GPU pipeline (section 3), as a
    comparator for ``fuse``: same result, one full-image pass per step."""
    pan, ms, _, out, H, W, B = _prep_scene(pan, ms, None, out)
    c = context(pan.device)
    c.bind_stream()
    st = c.lib.dwt_fuse_run_multipass(c.handle, wavelet_id(wavelet), H, W, B, _ptr(pan), _pitch(pan, 0),
                                      _ptr(ms), _pitch(ms, 1), _pitch(ms, 0), _ptr(out), _pitch(out, 1),
                                      _pitch(out, 0))
    c.check(st, "dwt_fuse_run_multipass")
    return out


def _check_batch_device(device, scene_device):
    """A batch runs on its scenes' device; an explicit `device` must be it."""
    if device is None:
        return
    if isinstance(device, int):
        idx = device
    else:
        d = torch.device(device)
        if d.type != "cuda":
            raise ValueError("device %s is not a GPU" % (device,))
        idx = d.index if d.index is not None else torch.cuda.current_device()
    if idx != scene_device.index:
        raise ValueError("device %s differs from the scenes' device %s" % (device, scene_device))


def make_items(scenes: Sequence[dict]):
    """Prepare dwt_fuse_item descriptors; each scene is a dict with keys pan,
    ms, wavelet and optionally gain, out.  Returns (items array, outs, keep)."""
    n = len(scenes)
    arr = (Item * max(n, 1))()
    outs, keep = [], []
    for i, s in enumerate(scenes):
        if s["pan"].device != scenes[0]["pan"].device:
            raise ValueError("scene %d is on %s, scene 0 on %s: one batch runs on one device"
                             % (i, s["pan"].device, scenes[0]["pan"].device))
        pan, ms, gain, out, H, W, B = _prep_scene(s["pan"], s["ms"], s.get("gain"), s.get("out"))
        keep.extend([pan, ms, gain, out])
        outs.append(out)
        it = arr[i]
        it.wavelet = wavelet_id(s.get("wavelet", "d4"))
        it.B = B
        it.H = H
        it.W = W
        it.pan = pan.data_ptr()
        it.ms = ms.data_ptr()
        it.gain = gain.data_ptr() if gain is not None else None
        it.out = out.data_ptr()
        it.pan_ld = _pitch(pan, 0)
        it.ms_ld = _pitch(ms, 1)
        it.ms_band_stride = _pitch(ms, 0)
        it.out_ld = _pitch(out, 1)
        it.out_band_stride = _pitch(out, 0)
    return arr, outs, keep


def fuse_batched(scenes: Sequence[dict], graph: bool = False, device=None) -> List[torch.Tensor]:
    """Fuse many independent scenes of any sizes, band counts and wavelets in
    one kernel launch (optionally captured into / replayed from a hipGraph).
    Returns the list of outputs."""
    if len(scenes) == 0:
        return []
    arr, outs, keep = make_items(scenes)
    _check_batch_device(device, scenes[0]["pan"].device)
    c = context(scenes[0]["pan"].device)
    c.bind_stream()
    st = c.lib.dwt_fuse_run_batched(c.handle, arr, len(scenes), _lib.GRAPH if graph else 0)
    c.check(st, "dwt_fuse_run_batched")
    return outs


def _prep_backward(pan, grad_out, gain, need_pan, need_ms, need_gain):
    _require(pan, "pan", 2)
    if grad_out.dim() == 2:
        grad_out = grad_out.unsqueeze(0)
    _require(grad_out, "grad_out", 3)
    pan = _rows_unit(pan)
    grad_out = _rows_unit(grad_out)
    H, W = pan.shape
    B = grad_out.shape[0]
    if tuple(grad_out.shape[1:]) != (H, W):
        raise ValueError("grad_out must be (B, H, W)")
    if gain is not None:
        _require(gain, "gain", 1)
        gain = gain.contiguous()
        if gain.shape[0] != B:
            raise ValueError("gain must have B=%d entries" % B)
        if gain.device != pan.device:
            raise ValueError("gain must be on the device of pan")
    if grad_out.device != pan.device:
        raise ValueError("pan and grad_out must be on the same device")
    dev = pan.device
    gp = torch.empty((H, W), dtype=torch.float32, device=dev) if need_pan else None
    gm = torch.empty((B, H // 2, W // 2), dtype=torch.float32, device=dev) if need_ms else None
    gg = torch.empty((B,), dtype=torch.float32, device=dev) if need_gain else None
    return pan, grad_out, gain, gp, gm, gg, H, W, B


def fuse_backward(pan: torch.Tensor, grad_out: torch.Tensor, wavelet="d4", gain: Optional[torch.Tensor] = None,
                  need_pan: bool = True, need_ms: bool = True, need_gain: bool = True):
    """Transpose of ``fuse``: (grad_pan (H,W), grad_ms (B,H/2,W/2), grad_gain (B,))
    for dLoss/d(out) = grad_out (B, H, W).  Entries not requested are None."""
    pan, grad_out, gain, gp, gm, gg, H, W, B = _prep_backward(pan, grad_out, gain, need_pan, need_ms, need_gain)
    c = context(pan.device)
    c.bind_stream()
    st = c.lib.dwt_fuse_backward(c.handle, wavelet_id(wavelet), H, W, B, _ptr(pan), _pitch(pan, 0), _ptr(gain),
                                 _ptr(grad_out), _pitch(grad_out, 1), _pitch(grad_out, 0),
                                 _ptr(gp), _ptr(gm), _ptr(gg))
    c.check(st, "dwt_fuse_backward")
    return gp, gm, gg


def fuse_backward_noalloc(pan: torch.Tensor, grad_out: torch.Tensor, grad_pan: Optional[torch.Tensor],
                          grad_ms: Optional[torch.Tensor], grad_gain: Optional[torch.Tensor], wavelet="d4",
                          gain: Optional[torch.Tensor] = None):
    """``fuse_backward`` into caller-provided outputs through
    dwt_fuse_backward_noalloc: neither this call nor the library allocates
    device memory (the grad_gain reduction uses the library's static scratch,
    so calls overlapping on one GPU race).  pan (H, W) and grad_out (B, H, W)
    need unit stride along rows; grad_pan (H, W), grad_ms (B, H/2, W/2) and
    grad_gain (B,) must be contiguous float32 on the same GPU, or None."""
    _require(pan, "pan", 2)
    _require(grad_out, "grad_out", 3)
    for t, name in ((pan, "pan"), (grad_out, "grad_out")):
        if t.stride(-1) != 1 or any(s < 0 for s in t.stride()):
            raise ValueError("%s needs unit stride along its rows (no copy is made)" % name)
    H, W = pan.shape
    B = grad_out.shape[0]
    if tuple(grad_out.shape[1:]) != (H, W):
        raise ValueError("grad_out must be (B, H, W)")
    for t, name, shape in ((grad_pan, "grad_pan", (H, W)), (grad_ms, "grad_ms", (B, H // 2, W // 2)),
                           (grad_gain, "grad_gain", (B,)), (gain, "gain", (B,))):
        if t is None:
            continue
        _require(t, name, len(shape))
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor" % (name, shape))
        if t.device != pan.device:
            raise ValueError("%s must be on the device of pan" % name)
    if grad_out.device != pan.device:
        raise ValueError("pan and grad_out must be on the same device")
    c = context(pan.device)
    c.bind_stream()
    st = c.lib.dwt_fuse_backward_noalloc(c.handle, wavelet_id(wavelet), H, W, B, _ptr(pan), _pitch(pan, 0),
                                         _ptr(gain), _ptr(grad_out), _pitch(grad_out, 1), _pitch(grad_out, 0),
                                         _ptr(grad_pan), _ptr(grad_ms), _ptr(grad_gain))
    c.check(st, "dwt_fuse_backward_noalloc")
    return grad_pan, grad_ms, grad_gain


def make_bwd_items(scenes: Sequence[dict]):
    """Prepare dwt_fuse_bwd_item descriptors; each scene is a dict with keys
    pan, grad_out, wavelet and optionally gain, need_pan, need_ms, need_gain
    (default True).  Returns (items array, [(grad_pan, grad_ms, grad_gain)],
    keep)."""
    n = len(scenes)
    arr = (BwdItem * max(n, 1))()
    outs, keep = [], []
    for i, s in enumerate(scenes):
        if s["pan"].device != scenes[0]["pan"].device:
            raise ValueError("scene %d is on %s, scene 0 on %s: one batch runs on one device"
                             % (i, s["pan"].device, scenes[0]["pan"].device))
        pan, go, gain, gp, gm, gg, H, W, B = _prep_backward(s["pan"], s["grad_out"], s.get("gain"),
                                                           s.get("need_pan", True), s.get("need_ms", True),
                                                           s.get("need_gain", True))
        keep.extend([pan, go, gain])
        outs.append((gp, gm, gg))
        it = arr[i]
        it.wavelet = wavelet_id(s.get("wavelet", "d4"))
        it.B = B
        it.H = H
        it.W = W
        it.pan = pan.data_ptr()
        it.gain = gain.data_ptr() if gain is not None else None
        it.grad_out = go.data_ptr()
        it.grad_pan = gp.data_ptr() if gp is not None else None
        it.grad_ms = gm.data_ptr() if gm is not None else None
        it.grad_gain = gg.data_ptr() if gg is not None else None
        it.pan_ld = _pitch(pan, 0)
        it.go_ld = _pitch(go, 1)
        it.go_band_stride = _pitch(go, 0)
    return arr, outs, keep


def fuse_backward_batched(scenes: Sequence[dict], device=None):
    """``fuse_backward`` of many independent scenes (dicts as in
    ``make_bwd_items``) with one launch per adjoint kernel variant (scenes on
    the LDS-staged adjoint, D4 with 5 or more bands, a launch each); results
    equal per-scene ``fuse_backward`` calls bit for bit.  Returns
    [(grad_pan, grad_ms, grad_gain)] per scene; entries not requested are
    None."""
    if len(scenes) == 0:
        return []
    arr, outs, keep = make_bwd_items(scenes)
    _check_batch_device(device, scenes[0]["pan"].device)
    c = context(scenes[0]["pan"].device)
    c.bind_stream()
    c.check(c.lib.dwt_fuse_backward_batched(c.handle, arr, len(scenes)), "dwt_fuse_backward_batched")
    return outs


class DwtFuseFn(torch.autograd.Function):
    """Differentiable fusion: ``DwtFuseFn.apply(pan, ms, gain, wavelet)``.

    Forward runs the fused kernel; backward runs the hand-written adjoint
    kernel (gradients w.r.t. PAN, MS and the per-band detail gain)."""

    @staticmethod
    def forward(ctx, pan, ms, gain, wavelet="d4"):
        ctx.wavelet = wavelet
        ctx.squeeze = ms.dim() == 2
        ctx.save_for_backward(pan, gain)
        return fuse(pan, ms, wavelet, gain)

    @staticmethod
    def backward(ctx, grad_out):
        pan, gain = ctx.saved_tensors
        need_pan, need_ms, need_gain = ctx.needs_input_grad[:3]
        gp, gm, gg = fuse_backward(pan, grad_out, ctx.wavelet, gain, need_pan, need_ms,
                                   need_gain and gain is not None)
        if gm is not None and ctx.squeeze:
            gm = gm[0]
        return gp, gm, gg, None
