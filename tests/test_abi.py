"""The C-ABI library loads, exports every symbol include/dwt_fuse.h declares,
and rejects every invalid argument combination on the host (validation runs
before any HIP call, so no GPU is needed here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwt_fuse.h")

from paper_1803_00737_amd import _lib  # noqa: E402

OK, E_NULL, E_SHAPE, E_WAVELET, E_STRIDE, E_ALIAS = 0, 1, 2, 3, 4, 5
P = 0x100000000  # fake device addresses: the checks never dereference them


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1803_00737_amd import build

        build.build()
    return _lib.load(require_torch=False)


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(dwt_fuse_[a-z_]+)\s*\(", text))


def test_exports_every_declared_symbol(lib):
    decl = declared_symbols()
    assert len(decl) >= 15
    assert decl == set(_lib.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name


def run_check(lib, w=1, H=8, W=8, B=2, pan=P, pan_ld=None, ms=P + 10**6, ms_ld=None, ms_bs=None, gain=None,
              out=P + 2 * 10**6, out_ld=None, out_bs=None):
    pan_ld = W if pan_ld is None else pan_ld
    ms_ld = W // 2 if ms_ld is None else ms_ld
    ms_bs = (H // 2) * ms_ld if ms_bs is None else ms_bs
    out_ld = W if out_ld is None else out_ld
    out_bs = H * out_ld if out_bs is None else out_bs
    return lib.dwt_fuse_check_run(w, H, W, B, pan, pan_ld, ms, ms_ld, ms_bs, gain, out, out_ld, out_bs)


def test_valid_arguments(lib):
    assert run_check(lib) == OK
    assert run_check(lib, w=0) == OK
    assert run_check(lib, H=2, W=2, B=1) == OK
    assert run_check(lib, B=1, ms_bs=0, out_bs=0) == OK  # band stride unused with one band
    assert run_check(lib, pan=P + 4, pan_ld=13) == OK  # unaligned pointer / odd pitch are allowed
    assert run_check(lib, gain=P + 5 * 10**6) == OK


def test_null_pointers(lib):
    assert run_check(lib, pan=None) == E_NULL
    assert run_check(lib, ms=None) == E_NULL
    assert run_check(lib, out=None) == E_NULL


@pytest.mark.parametrize("H,W,B", [(7, 8, 1), (8, 7, 1), (0, 8, 1), (8, 0, 1), (2, 1, 1), (8, 8, 0),
                                   (8, 8, -3), (-2, 8, 1), (2 ** 31, 8, 1)])
def test_bad_shapes(lib, H, W, B):
    assert run_check(lib, H=H, W=W, B=B, pan_ld=max(W, 1), ms_ld=max(W // 2, 1), ms_bs=10**9,
                     out_ld=max(W, 1), out_bs=10**10) == E_SHAPE


def test_overflowing_size(lib):
    big = 2 ** 30
    assert run_check(lib, H=big, W=big, B=2 ** 19) == E_SHAPE


@pytest.mark.parametrize("w", [2, -1, 99])
def test_bad_wavelet(lib, w):
    assert run_check(lib, w=w) == E_WAVELET


def test_bad_strides(lib):
    assert run_check(lib, pan_ld=7) == E_STRIDE
    assert run_check(lib, ms_ld=3) == E_STRIDE
    assert run_check(lib, out_ld=6) == E_STRIDE
    assert run_check(lib, ms_bs=15) == E_STRIDE  # < (H/2) * ms_ld = 16
    assert run_check(lib, out_bs=63) == E_STRIDE
    assert run_check(lib, pan_ld=-8) == E_STRIDE


def test_aliasing(lib):
    assert run_check(lib, out=P) == E_ALIAS  # out == pan
    # out band 1 overlaps the last bytes of ms
    ms = P + 10**6
    ms_bytes = 2 * 16 * 4
    assert run_check(lib, out=ms + ms_bytes - 4) == E_ALIAS
    assert run_check(lib, out=ms + ms_bytes) == OK  # touching, not overlapping
    out = P + 2 * 10**6
    assert run_check(lib, gain=out + 8) == E_ALIAS
    assert run_check(lib, pan=out + 2 * 64 * 4 - 4) == E_ALIAS


def item(w=1, H=8, W=8, B=2, base=P):
    it = _lib.Item()
    it.wavelet, it.B, it.H, it.W = w, B, H, W
    it.pan, it.ms, it.gain, it.out = base, base + 10**6, None, base + 2 * 10**6
    it.pan_ld, it.ms_ld, it.ms_band_stride = W, W // 2, (H // 2) * (W // 2)
    it.out_ld, it.out_band_stride = W, H * W
    return it


def batch(*items):
    arr = (_lib.Item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def test_batched_validation(lib):
    assert lib.dwt_fuse_check_batched(None, 0) == OK
    assert lib.dwt_fuse_check_batched(None, 3) == E_NULL
    assert lib.dwt_fuse_check_batched(batch(item()), -1) == E_SHAPE
    assert lib.dwt_fuse_check_batched(batch(item(), item(base=P + 10**7)), 2) == OK
    assert lib.dwt_fuse_check_batched(batch(item(), item(H=7, base=P + 10**7)), 2) == E_SHAPE
    assert lib.dwt_fuse_check_batched(batch(item(), item(w=5, base=P + 10**7)), 2) == E_WAVELET
    # two items writing the same output
    a, b = item(), item(base=P + 10**7)
    b.out = a.out + 64
    assert lib.dwt_fuse_check_batched(batch(a, b), 2) == E_ALIAS
    # item 1's output overlaps item 0's MS
    b = item(base=P + 10**7)
    b.out = a.ms + 8
    assert lib.dwt_fuse_check_batched(batch(a, b), 2) == E_ALIAS
    # items may share inputs (one PAN, several MS sets)
    b = item(base=P + 10**7)
    b.pan = a.pan
    assert lib.dwt_fuse_check_batched(batch(a, b), 2) == OK


def bwd_check(lib, w=1, H=8, W=8, B=2, pan=P, gain=None, gy=P + 10**6, gp=P + 2 * 10**6, gm=P + 3 * 10**6,
              gg=P + 4 * 10**6, gy_ld=None, gy_bs=None):
    gy_ld = W if gy_ld is None else gy_ld
    gy_bs = H * gy_ld if gy_bs is None else gy_bs
    return lib.dwt_fuse_check_backward(w, H, W, B, pan, W, gain, gy, gy_ld, gy_bs, gp, gm, gg)


def test_backward_validation(lib):
    assert bwd_check(lib) == OK
    assert bwd_check(lib, gp=None, gm=None, gg=None) == OK
    assert bwd_check(lib, pan=None) == E_NULL
    assert bwd_check(lib, gy=None) == E_NULL
    assert bwd_check(lib, H=5) == E_SHAPE
    assert bwd_check(lib, w=3) == E_WAVELET
    assert bwd_check(lib, gy_ld=4) == E_STRIDE
    assert bwd_check(lib, gp=P + 10**6 + 16) == E_ALIAS  # grad_pan over grad_out
    assert bwd_check(lib, gm=P + 2 * 10**6 + 8) == E_ALIAS  # grad_ms over grad_pan
    assert bwd_check(lib, gg=P + 4) == E_ALIAS  # grad_gain over pan


def bwd_item(w=1, H=8, W=8, B=2, base=P, gain=False, outs=(True, True, True)):
    it = _lib.BwdItem()
    it.wavelet, it.B, it.H, it.W = w, B, H, W
    it.pan = base
    it.grad_out = base + 10**6
    it.gain = base + 5 * 10**6 if gain else None
    it.grad_pan = base + 2 * 10**6 if outs[0] else None
    it.grad_ms = base + 3 * 10**6 if outs[1] else None
    it.grad_gain = base + 4 * 10**6 if outs[2] else None
    it.pan_ld, it.go_ld, it.go_band_stride = W, W, H * W
    return it


def bwd_batch(*items):
    arr = (_lib.BwdItem * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def test_backward_batched_validation(lib):
    chk = lib.dwt_fuse_check_backward_batched
    assert chk(None, 0) == OK
    assert chk(None, 2) == E_NULL
    assert chk(bwd_batch(bwd_item()), -1) == E_SHAPE
    a = bwd_item()
    assert chk(bwd_batch(a, bwd_item(base=P + 10**7, gain=True)), 2) == OK
    # per-item rules, reported for the first failing item
    assert chk(bwd_batch(a, bwd_item(H=6, W=5, base=P + 10**7)), 2) == E_SHAPE
    assert chk(bwd_batch(a, bwd_item(w=4, base=P + 10**7)), 2) == E_WAVELET
    b = bwd_item(base=P + 10**7)
    b.pan = None
    assert chk(bwd_batch(a, b), 2) == E_NULL
    b = bwd_item(base=P + 10**7)
    b.go_ld = 4
    assert chk(bwd_batch(a, b), 2) == E_STRIDE
    # item 1's grad_ms over item 0's grad_pan
    b = bwd_item(base=P + 10**7)
    b.grad_ms = a.grad_pan + 8
    assert chk(bwd_batch(a, b), 2) == E_ALIAS
    # item 1's grad_gain over item 0's grad_out
    b = bwd_item(base=P + 10**7)
    b.grad_gain = a.grad_out + 4
    assert chk(bwd_batch(a, b), 2) == E_ALIAS
    # item 0's grad_pan over item 1's gain
    b = bwd_item(base=P + 10**7, gain=True)
    b.gain = a.grad_pan + 16
    assert chk(bwd_batch(a, b), 2) == E_ALIAS
    # inputs may be shared (one PAN, several upstream gradients); absent outputs never alias
    b = bwd_item(base=P + 10**7, outs=(False, True, False))
    b.pan = a.pan
    assert chk(bwd_batch(a, b), 2) == OK
    assert chk(bwd_batch(bwd_item(outs=(False, False, False)), bwd_item(outs=(False, False, False))), 2) == OK
    assert lib.dwt_fuse_backward_batched(None, None, 0) == E_NULL


def test_status_strings(lib):
    for s in range(9):
        assert lib.dwt_fuse_status_str(s)
    assert lib.dwt_fuse_status_str(42) == b"unknown status"
    assert lib.dwt_fuse_last_error(None) == b""


def test_null_context_entry_points(lib):
    assert lib.dwt_fuse_run(None, 1, 8, 8, 1, P, 8, P + 10**6, 4, 16, None, P + 2 * 10**6, 8, 64) == E_NULL
    assert lib.dwt_fuse_run_batched(None, None, 0, 0) == E_NULL
    assert lib.dwt_fuse_backward(None, 1, 8, 8, 1, P, 8, None, P, 8, 64, None, None, None) == E_NULL
    assert lib.dwt_fuse_set_stream(None, None) == E_NULL
    assert lib.dwt_fuse_set_tuning(None, 1) == E_NULL
    assert lib.dwt_fuse_force_tile(None, 1, 1, 1, 0) == E_NULL
    assert lib.dwt_fuse_force_band_split(None, 1) == E_NULL
    assert lib.dwt_fuse_force_order(None, 3) == E_NULL
    assert lib.dwt_fuse_quality_scores(None, 8, 8, 1, P, 8, 64, P + 10**6, 8, 64, P + 2 * 10**6) == E_NULL
    assert lib.dwt_fuse_backward_noalloc(None, 1, 8, 8, 1, P, 8, None, P, 8, 64, None, None, None) == E_NULL
    assert lib.dwt_fuse_run_multipass(None, 1, 8, 8, 1, P, 8, P + 10**6, 4, 16, P + 2 * 10**6, 8, 64) == E_NULL
    lib.dwt_fuse_destroy(None)  # NULL-safe
    assert lib.dwt_fuse_create(None, 0, None) == E_NULL


def test_cpu_tensors_rejected_by_binding():
    torch = pytest.importorskip("torch")
    from paper_1803_00737_amd import api

    with pytest.raises(ValueError, match="GPU"):
        api.fuse(torch.zeros(8, 8), torch.zeros(1, 4, 4), "haar")
    with pytest.raises(ValueError, match="GPU"):
        api.fuse_backward(torch.zeros(8, 8), torch.zeros(1, 8, 8), "d4")
    with pytest.raises(ValueError, match="GPU"):
        api.fuse_backward_batched([dict(pan=torch.zeros(8, 8), grad_out=torch.zeros(1, 8, 8))])
    with pytest.raises(ValueError, match="GPU"):
        api.fuse_batched([dict(pan=torch.zeros(8, 8), ms=torch.zeros(1, 4, 4))])


def test_batch_device_argument_checked():
    torch = pytest.importorskip("torch")
    from paper_1803_00737_amd import api

    cuda0 = torch.device("cuda", 0)
    api._check_batch_device(None, cuda0)
    api._check_batch_device(0, cuda0)
    api._check_batch_device("cuda:0", cuda0)
    with pytest.raises(ValueError, match="differs"):
        api._check_batch_device(1, cuda0)
    with pytest.raises(ValueError, match="not a GPU"):
        api._check_batch_device("cpu", cuda0)


def test_no_oracle_in_product():
    """The product package never references the oracle."""
    pkg = os.path.join(ROOT, "paper_1803_00737_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)


def ex_check(lib, fin=1, fout=1, kappa=1.0, w=1, H=8, W=8, B=2, pan=P, pan_ld=None, ms=P + 10**6, ms_ld=None,
             ms_bs=None, gain=None, out=P + 2 * 10**6, out_ld=None, out_bs=None, opts=True):
    pan_ld = W if pan_ld is None else pan_ld
    ms_ld = W // 2 if ms_ld is None else ms_ld
    ms_bs = (H // 2) * ms_ld if ms_bs is None else ms_bs
    out_ld = W if out_ld is None else out_ld
    out_bs = H * out_ld if out_bs is None else out_bs
    o = ctypes.byref(_lib.Opts(fin, fout, kappa)) if opts else None
    return lib.dwt_fuse_check_run_ex(w, H, W, B, pan, pan_ld, ms, ms_ld, ms_bs, gain, out, out_ld, out_bs, o)


def test_run_ex_validation(lib):
    E_FORMAT = 9
    assert ex_check(lib) == OK
    assert ex_check(lib, opts=False) == OK  # NULL opts = float32 in and out, kappa 1
    assert ex_check(lib, fin=0, fout=1, kappa=2.0) == OK
    assert ex_check(lib, fin=2) == E_FORMAT
    assert ex_check(lib, fout=-1) == E_FORMAT
    assert ex_check(lib, pan=None) == E_NULL
    assert ex_check(lib, w=5) == E_WAVELET
    assert ex_check(lib, H=7) == E_SHAPE
    assert ex_check(lib, pan_ld=7) == E_STRIDE
    assert ex_check(lib, pan=P + 1, pan_ld=9) == OK  # byte pitches need no alignment
    # byte ranges follow each buffer's element size: 8-bit PAN of 8 x 8 ends
    # 64 bytes after its start, a float one 256 bytes after
    assert ex_check(lib, out=P + 64, B=1) == OK
    assert ex_check(lib, out=P + 63, B=1) == E_ALIAS
    assert ex_check(lib, fin=0, fout=0, out=P + 64, B=1) == E_ALIAS
    assert ex_check(lib, fin=0, fout=0, out=P + 256, B=1) == OK
    # 8-bit out of 2 bands x 8 x 8 spans 128 bytes
    assert ex_check(lib, out=P - 128, B=2) == OK
    assert ex_check(lib, out=P - 127, B=2) == E_ALIAS
    assert lib.dwt_fuse_status_str(E_FORMAT) == b"unknown element format"


def test_only_the_header_is_exported(lib):
    """The library exports exactly the C ABI the header declares (internal
    C++ symbols have hidden visibility)."""
    import shutil
    import subprocess

    nm = shutil.which("nm")
    if not nm:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.split()[1:2] == ["T"]}
    assert exported == declared_symbols()
