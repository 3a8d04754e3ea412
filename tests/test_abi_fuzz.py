"""Property-based checks of the host-side argument validation (no GPU): for
random sizes, pitches, band strides and fake device addresses, every
dwt_fuse_check_* entry point returns one of the documented status codes and
never crashes; OK is returned only when the byte ranges neither overflow nor
overlap, recomputed here in Python integers."""
import ctypes
import os

import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from paper_1803_00737_amd import _lib  # noqa: E402

STATUSES = set(range(10))
I64 = 2 ** 63 - 1


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1803_00737_amd import build

        build.build()
    return _lib.load(require_torch=False)


def span(ptr, nb, rows, cols, ld, bs, esize):
    """Byte range [lo, hi) of nb bands of rows x cols (pointers as unsigned
    64-bit addresses), or None when the size or the address range overflows."""
    if nb < 1 or rows < 1 or cols < 1:
        return None
    e = (nb - 1) * bs + (rows - 1) * ld + cols
    if e > I64 // 4:
        return None
    lo = ptr % 2 ** 64
    if lo + e * esize > 2 ** 64 - 1:
        return None
    return (lo, lo + e * esize)


def overlap(a, b):
    return a[0] < b[1] and b[0] < a[1]


sizes = st.integers(min_value=-4, max_value=70000)
pitch_extra = st.integers(min_value=-3, max_value=1 << 20)
addr = st.integers(min_value=1, max_value=1 << 44)


@settings(max_examples=400, deadline=None)
@given(H=sizes, W=sizes, B=st.integers(-2, 40), pe=pitch_extra, me=pitch_extra, oe=pitch_extra,
       pan=addr, ms=addr, out=addr, wav=st.integers(-1, 2), big=st.booleans())
def test_check_run_never_crashes(lib, H, W, B, pe, me, oe, pan, ms, out, wav, big):
    if big:
        H, W = H * 40000, W * 30000
    pan_ld = max(W, 0) + pe
    ms_ld = max(W // 2, 0) + me
    out_ld = max(W, 0) + oe
    ms_bs = (max(H, 0) // 2) * ms_ld
    out_bs = max(H, 0) * out_ld
    st_ = lib.dwt_fuse_check_run(wav, H, W, B, pan, pan_ld, ms, ms_ld, ms_bs, None, out, out_ld, out_bs)
    assert st_ in STATUSES
    if st_ == 0:
        assert H >= 2 and W >= 2 and H % 2 == 0 and W % 2 == 0 and B >= 1 and wav in (0, 1)
        sp = span(pan, 1, H, W, pan_ld, 0, 4)
        sm = span(ms, B, H // 2, W // 2, ms_ld, ms_bs, 4)
        so = span(out, B, H, W, out_ld, out_bs, 4)
        assert sp and sm and so
        assert not overlap(so, sp) and not overlap(so, sm)


@settings(max_examples=300, deadline=None)
@given(H=st.integers(-2, 5000), W=st.integers(-2, 5000), B=st.integers(-1, 12), fin=st.integers(-1, 2),
       fout=st.integers(-1, 2), pan=addr, gap=st.integers(-(1 << 26), 1 << 26))
def test_check_run_ex_never_crashes(lib, H, W, B, fin, fout, pan, gap):
    es = {0: 4, 1: 1}
    ms = pan + (1 << 30)
    out = pan + gap
    o = _lib.Opts(fin, fout, 1.0)
    st_ = lib.dwt_fuse_check_run_ex(1, H, W, B, pan, W, ms, W // 2, (H // 2) * (W // 2), None, out, W, H * W,
                                    ctypes.byref(o))
    assert st_ in STATUSES
    if st_ == 0:
        assert fin in es and fout in es
        sp = span(pan, 1, H, W, W, 0, es[fin])
        so = span(out, B, H, W, W, H * W, es[fout])
        assert sp and so and not overlap(sp, so)


@settings(max_examples=200, deadline=None)
@given(n=st.integers(-3, 6), H=st.integers(0, 300), W=st.integers(0, 300), B=st.integers(0, 5),
       stride=st.integers(0, 1 << 22))
def test_check_batched_never_crashes(lib, n, H, W, B, stride):
    k = max(n, 0)
    items = (_lib.Item * max(k, 1))()
    for i in range(k):
        it = items[i]
        it.wavelet, it.B, it.H, it.W = i % 2, B, H, W
        base = (1 << 40) + i * stride
        it.pan, it.ms, it.out, it.gain = base, base + (1 << 30), base + (1 << 31), None
        it.pan_ld, it.ms_ld, it.out_ld = W, W // 2, W
        it.ms_band_stride, it.out_band_stride = (H // 2) * (W // 2), H * W
    st_ = lib.dwt_fuse_check_batched(items if n >= 0 else items, n)
    assert st_ in STATUSES
    if n < 0:
        assert st_ != 0


@settings(max_examples=300, deadline=None)
@given(n=st.integers(-2, 5), H=st.integers(-2, 300), W=st.integers(-2, 300), B=st.integers(-1, 10),
       stride=st.integers(0, 1 << 24), shift=st.integers(-(1 << 22), 1 << 22), which=st.integers(0, 5),
       outs=st.integers(0, 7))
def test_check_backward_batched_never_crashes(lib, n, H, W, B, stride, shift, which, outs):
    """Random batches of backward descriptors, one field of the last item
    moved by `shift` bytes: OK only when every item is valid on its own, no
    output overlaps another output and no output overlaps any input."""
    k = max(n, 0)
    items = (_lib.BwdItem * max(k, 1))()
    for i in range(k):
        it = items[i]
        it.wavelet, it.B, it.H, it.W = i % 2, B, H, W
        base = (1 << 40) + i * stride
        it.pan, it.grad_out, it.gain = base, base + (1 << 30), base + (3 << 30)
        it.grad_pan = base + (1 << 31) if outs & 1 else None
        it.grad_ms = base + (5 << 29) if outs & 2 else None
        it.grad_gain = base + (7 << 29) if outs & 4 else None
        it.pan_ld, it.go_ld, it.go_band_stride = W, W, H * W
    if k > 0:
        f = ["pan", "grad_out", "gain", "grad_pan", "grad_ms", "grad_gain"][which]
        if getattr(items[k - 1], f) is not None:
            setattr(items[k - 1], f, max(1, getattr(items[k - 1], f) + shift))
    st_ = lib.dwt_fuse_check_backward_batched(items, n)
    assert st_ in STATUSES
    if n < 0:
        assert st_ != 0
    if st_ != 0 or k == 0:
        return
    assert H >= 2 and W >= 2 and H % 2 == 0 and W % 2 == 0 and B >= 1
    ins, outs_ = [], []
    for i in range(k):
        it = items[i]
        ins.append(span(it.pan, 1, H, W, W, 0, 4))
        ins.append(span(it.grad_out, B, H, W, W, H * W, 4))
        ins.append(span(it.gain, 1, 1, B, B, 0, 4))
        for ptr, nb, rows, cols in ((it.grad_pan, 1, H, W), (it.grad_ms, B, H // 2, W // 2), (it.grad_gain, 1, 1, B)):
            if ptr is not None:
                outs_.append(span(ptr, nb, rows, cols, cols, rows * cols, 4))
    assert all(s is not None for s in ins + outs_)
    for a in range(len(outs_)):
        for b in range(a + 1, len(outs_)):
            assert not overlap(outs_[a], outs_[b])
        for s in ins:
            assert not overlap(outs_[a], s)
