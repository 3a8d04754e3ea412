"""GPU parity of the fused forward kernels against the FP64 oracle, through
the C ABI (via the thin binding).

Bars: Haar bit-exact on integer-valued inputs (the oracle's values are
multiples of 1/4 and exactly representable in float32); D4 max-abs <= 1e-3 on
the 0-255 scale.  Sizes span several work units and ragged tails (odd W/2,
widths not a multiple of the 256/512-column strip), all three load paths
(128-bit, 64-bit, scalar), pitched views, and the full-size workloads
(sampled outputs checked one by one with the single-pixel oracle).
"""
import numpy as np
import pytest

from gpu_helpers import D4_TOL, int_scene, require_gpu, say, strided_view, to_dev, torch, ulp_diff

pytestmark = pytest.mark.gpu

SHAPES = [(2, 2), (2, 6), (4, 10), (6, 2), (34, 70), (130, 258), (64, 4070), (200, 1030), (66, 514),
          (258, 1026), (512, 512)]


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


def oracle_out(oracle, wavelet, pan, ms, gain=None):
    return oracle.fuse(wavelet, pan.astype(np.float64), ms.astype(np.float64), gain)


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("B", [1, 3])
def test_haar_bit_exact(dev, fz, oracle, H, W, B):
    rng = np.random.default_rng(H * 1000 + W + B)
    pan, ms = int_scene(rng, H, W, B)
    say("haar", H, W, B)
    out = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "haar").cpu().numpy()
    ref = oracle_out(oracle, "haar", pan, ms).astype(np.float32)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("B", [1, 3])
def test_d4_within_tolerance(dev, fz, oracle, H, W, B):
    rng = np.random.default_rng(H * 1000 + W + B + 7)
    pan, ms = int_scene(rng, H, W, B)
    say("d4", H, W, B)
    out = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "d4").cpu().numpy()
    ref = oracle_out(oracle, "d4", pan, ms)
    assert np.abs(out - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(2, 1 << 20), (1 << 20, 2), (4, (1 << 19) + 6), ((1 << 18) + 2, 6)])
def test_extreme_aspect_ratios(dev, fz, oracle, wavelet, H, W):
    """One-row-pair and one-column-pair images a million pixels long (every
    D4 tap wraps along the short side; strips or tiles by the thousand along
    the long one), in the default and the tuned launch shapes, forward and
    adjoint, against the oracle over the whole image."""
    rng = np.random.default_rng(H + W)
    pan, ms = int_scene(rng, H, W, 2)
    say("aspect", wavelet, H, W)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    ref = oracle_out(oracle, wavelet, pan, ms)
    ctx = fz.context(dev)
    for tuned in (False, True):
        ctx.set_tuning(tuned)
        try:
            out = fz.fuse(p, m, wavelet).cpu().numpy()
        finally:
            ctx.set_tuning(False)
        if wavelet == "haar":
            assert np.array_equal(out, ref.astype(np.float32))
        else:
            assert np.abs(out - ref).max() <= D4_TOL
    gy = rng.normal(size=(2, H, W)).astype(np.float32)
    gp, gm, _ = fz.fuse_backward(p, to_dev(gy, dev), wavelet, need_gain=False)
    rp, rm, _ = oracle.fuse_backward(wavelet, pan.astype(np.float64), None, gy.astype(np.float64))
    assert np.abs(gp.cpu().numpy() - rp).max() <= 16e-5 * max(1.0, np.abs(rp).max())
    assert np.abs(gm.cpu().numpy() - rm).max() <= 16e-5 * max(1.0, np.abs(rm).max())


def test_haar_workload_512(dev, fz, oracle):
    from paper_1803_00737_amd import synth

    wl = synth.haar_512()
    pan, ms = wl.make()
    say("haar 512 workload")
    out = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "haar").cpu().numpy()
    assert np.array_equal(out, oracle_out(oracle, "haar", pan, ms).astype(np.float32))


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_gains(dev, fz, oracle, wavelet):
    rng = np.random.default_rng(21)
    pan, ms = int_scene(rng, 66, 130, 4)
    for gain in ([1.0, 0.5, 2.0, 0.0], [0.7, 1.3, 1.05, 0.91]):
        say(wavelet, "gain", gain)
        g = torch.tensor(gain, dtype=torch.float32, device=dev)
        out = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet, g).cpu().numpy()
        ref = oracle_out(oracle, wavelet, pan, ms, np.array(gain, np.float32).astype(np.float64))
        if wavelet == "d4":
            assert np.abs(out - ref).max() <= D4_TOL
        elif gain[3] == 0.0:  # powers of two: still exact
            assert np.array_equal(out, ref.astype(np.float32))
        else:  # one rounding (fused multiply-add) against the rounded FP64 value
            assert ulp_diff(out, ref.astype(np.float32)) <= 1


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("pad,offset", [(0, 0), (6, 0), (4, 2), (1, 1), (3, 3)])
@pytest.mark.parametrize("H,W", [(34, 70), (66, 1030)])
def test_paths_and_pitches(dev, fz, oracle, wavelet, pad, offset, H, W):
    """Pitched and misaligned views take the 64-bit or scalar paths; results
    must be identical to the contiguous (128-bit) call."""
    rng = np.random.default_rng(pad * 10 + offset + H)
    pan, ms = int_scene(rng, H, W, 3)
    say(wavelet, "pitch", pad, offset, H, W)
    pv = strided_view(pan, dev, pad, offset)
    mv = strided_view(ms, dev, pad, offset)
    ov = strided_view(np.zeros((3, H, W), np.float32), dev, pad, offset)
    fz.fuse(pv, mv, wavelet, out=ov)
    got = ov.cpu().numpy()
    base = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    assert np.array_equal(got, base)
    ref = oracle_out(oracle, wavelet, pan, ms)
    if wavelet == "haar":
        assert np.array_equal(got, ref.astype(np.float32))
    else:
        assert np.abs(got - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(8, 8), (34, 136), (66, 516), (34, 134), (130, 1288), (10, 1290)])
@pytest.mark.parametrize("pad,off", [(8, 4), (6, 2), (5, 1)])
def test_forward_writes_stay_inside(dev, fz, wavelet, H, W, pad, off):
    """Every forward variant writes only its output: the output is a window
    (rows 1..H, columns off..off+W-1) of a larger buffer whose other elements
    hold a sentinel, with pitches and offsets that select the 128-bit, 64-bit
    and scalar paths; the sentinels must survive every forced launch shape,
    float and 8-bit output alike, and the window must match the plain call."""
    rng = np.random.default_rng(H * W + pad)
    B = 3
    pan, ms = int_scene(rng, H, W, B)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    ref = fz.fuse(p, m, wavelet)
    ref8 = fz.fuse(p.to(torch.uint8), m.to(torch.uint8), wavelet, out_dtype=torch.uint8)
    sentinel = 12345.0
    ctx = fz.context(dev)
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (16, 4, 2, 1), (3, 2, 1, 1), (1, 4, 2, 2), (2, 2, 1, 2),
                                  (2, 4, 2, 3), (1, 2, 2, 3), (4, 1, 2, 3)]:
            say(wavelet, "sentinel", H, W, pad, off, seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            big = torch.full((B, H + 2, W + pad), sentinel, device=dev)
            out = big[:, 1:H + 1, off:off + W]
            fz.fuse(p, m, wavelet, out=out)
            inside = torch.zeros_like(big, dtype=torch.bool)
            inside[:, 1:H + 1, off:off + W] = True
            assert bool((big[~inside] == sentinel).all()), ("float output escaped its window", seg, wpb, nc, var)
            assert torch.equal(out, ref), ("float window differs", seg, wpb, nc, var)
            big8 = torch.full((B, H + 2, W + pad), 77, dtype=torch.uint8, device=dev)
            out8 = big8[:, 1:H + 1, off:off + W]
            fz.fuse(p.to(torch.uint8), m.to(torch.uint8), wavelet, out=out8, out_dtype=torch.uint8)
            assert bool((big8[~inside] == 77).all()), ("8-bit output escaped its window", seg, wpb, nc, var)
            assert torch.equal(out8, ref8), ("8-bit window differs", seg, wpb, nc, var)
    finally:
        ctx.force_tile(0, 0, 0, 0)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(250, 1034), (250, 1288), (18, 8)])
def test_tile_shapes_give_identical_results(dev, fz, wavelet, H, W):
    """Every output pixel is evaluated in the same order whatever unit holds
    it, so forced launch shapes (rolling, one-shot and LDS-staged variants,
    staged units split into band groups of 1 or 2 bands) must agree bit for
    bit.  1288 = 5 full 256-column strips + a partial one
    on the 128-bit path; H/2 = 125 leaves partial tiles."""
    rng = np.random.default_rng(5)
    pan, ms = int_scene(rng, H, W, 3)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    ctx = fz.context(dev)
    outs = []
    try:
        for seg, wpb, nc, var, split in [(0, 0, 0, 0, 0), (1, 1, 1, 1, 0), (3, 2, 2, 1, 0), (7, 4, 1, 1, 0),
                                         (64, 1, 2, 1, 0), (200, 4, 2, 1, 0), (1, 1, 2, 2, 0), (2, 4, 2, 2, 0),
                                         (1, 2, 1, 2, 0), (2, 1, 1, 2, 0), (1, 4, 2, 3, 0), (2, 2, 2, 3, 0),
                                         (4, 1, 2, 3, 0), (2, 4, 2, 3, 0), (4, 4, 2, 3, 0), (2, 4, 2, 3, 1),
                                         (1, 2, 2, 3, 2), (4, 1, 2, 3, 1)]:
            say(wavelet, "tile", seg, wpb, nc, var, "split", split)
            ctx.force_tile(seg, wpb, nc, var)
            ctx.force_band_split(split)
            outs.append(fz.fuse(p, m, wavelet).cpu().numpy())
    finally:
        ctx.force_tile(0, 0, 0, 0)
        ctx.force_band_split(0)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(250, 1288), (66, 1030), (18, 8), (130, 2824), (34, 4104), (300, 3320)])
def test_unit_orders_give_identical_results(dev, fz, oracle, wavelet, H, W):
    """Every unit order (column strips or row bands, per-XCD runs or dispatch
    order, XCD slabs for the LDS-staged tiles: 1, 5, 6, 12, 14 and 18 overlapped
    strips of 128 coefficient columns over 2-38 row bands, so some XCDs' chunks are
    empty or shorter and rotate from band to band) of
    every variant gives the same output bit for bit, and the oracle's; 8-bit
    output too.  Outputs start as NaN (8-bit: alternately 0 and 255), so a
    unit that an order skips shows."""
    rng = np.random.default_rng(17)
    pan, ms = int_scene(rng, H, W, 3)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    ref = oracle_out(oracle, wavelet, pan, ms)
    ctx = fz.context(dev)
    base = None
    fill8 = 0
    try:
        for order in (0, 1, 2, 3, 4, 5, 6, 7):
            ctx.force_order(order)
            for seg, wpb, nc, var in [(0, 0, 0, 0), (16, 4, 2, 1), (1, 2, 1, 2), (2, 4, 2, 2), (2, 4, 2, 3),
                                      (1, 4, 2, 3), (4, 2, 2, 3)]:
                say(wavelet, "order", order, H, W, "tile", seg, wpb, nc, var)
                ctx.force_tile(seg, wpb, nc, var)
                o = torch.full((3, H, W), float("nan"), device=dev)
                o8 = torch.full((3, H, W), fill8, dtype=torch.uint8, device=dev)
                fill8 = 255 - fill8
                out = fz.fuse(p, m, wavelet, out=o).cpu().numpy()
                out8 = fz.fuse(p.to(torch.uint8), m.to(torch.uint8), wavelet, out=o8).cpu().numpy()
                if base is None:
                    base = (out, out8)
                    if wavelet == "haar":
                        assert np.array_equal(out, ref.astype(np.float32))
                    else:
                        assert np.abs(out - ref).max() <= D4_TOL
                assert np.array_equal(out, base[0]), (order, seg, wpb, nc, var)
                assert np.array_equal(out8, base[1]), (order, seg, wpb, nc, var)
    finally:
        ctx.force_tile(0, 0, 0, 0)
        ctx.force_order(-1)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(66, 1032), (34, 70), (10, 516)])
@pytest.mark.parametrize("ms_pad,ms_off", [(0, 0), (1, 1), (2, 2)])
def test_tile_shapes_on_8_byte_rows(dev, fz, oracle, wavelet, H, W, ms_pad, ms_off):
    """PAN/out rows with an even pitch that is not a multiple of 4 floats are
    8-byte aligned, every other one also 16-byte aligned; the first row here
    starts 8 bytes past a 16-byte boundary.  Two coefficient columns per lane
    then take 16-byte accesses on the aligned rows and 8-byte ones on the
    others, and MS rows 8-byte pairs where their alignment allows.  Every
    forced shape must equal the contiguous call bit for bit."""
    rng = np.random.default_rng(H + W + ms_pad)
    pan, ms = int_scene(rng, H, W, 3)
    base = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    pad = 2 if W % 4 == 0 else 0  # pitch = 2 (mod 4)
    pv = strided_view(pan, dev, pad, 2)
    mv = strided_view(ms, dev, ms_pad, ms_off)
    ctx = fz.context(dev)
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (1, 1, 2, 1), (3, 2, 2, 1), (5, 4, 1, 1), (1, 1, 2, 2),
                                  (2, 4, 2, 2), (2, 4, 1, 2), (2, 4, 2, 3)]:
            say(wavelet, "8-byte rows", H, W, "ms", ms_pad, ms_off, "tile", seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            ov = strided_view(np.zeros((3, H, W), np.float32), dev, pad, 2)
            fz.fuse(pv, mv, wavelet, out=ov)
            assert np.array_equal(ov.cpu().numpy(), base)
    finally:
        ctx.force_tile(0, 0, 0, 0)
    if wavelet == "haar":
        assert np.array_equal(base, oracle_out(oracle, "haar", pan, ms).astype(np.float32))
    else:
        assert np.abs(base - oracle_out(oracle, "d4", pan, ms)).max() <= D4_TOL


def padded(a: np.ndarray, dev, pitch: int):
    """Device view of ``a`` inside a NaN-filled buffer whose rows have
    ``pitch`` floats (the first row at the start of the allocation).
    Returns (view, buffer)."""
    buf = torch.full(a.shape[:-1] + (pitch,), float("nan"), dtype=torch.float32, device=dev)
    v = buf[..., :a.shape[-1]]
    v.copy_(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    return v, buf


W2MOD4_SHAPES = [(2, 2), (34, 70), (66, 1030), (64, 4070)]
W2MOD4_TILES = [(0, 0, 0, 0), (16, 4, 2, 1), (1, 4, 2, 2), (2, 1, 2, 2), (2, 4, 2, 3), (1, 2, 2, 3),
                (4, 1, 2, 3), (4, 4, 2, 3)]


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", W2MOD4_SHAPES)
def test_16_byte_rows_with_w_2_mod_4(dev, fz, oracle, wavelet, H, W):
    """W = 2 (mod 4) with PAN and output rows padded to a multiple of 4
    floats and MS rows to an even pitch: every row is 16-byte aligned, so the
    128-bit path runs although W/2 is odd.  The last coefficient column's D4
    row filter wraps to pixels 0, 1 (Eq. 5-6) where the row padding (NaN
    here) follows pixel W-1 in memory.  Every forced shape (rolling, one-shot,
    LDS-staged) must match the oracle, equal the contiguous call bit for bit,
    and leave the output padding untouched."""
    B = 3
    rng = np.random.default_rng(H * 7 + W)
    pan, ms = int_scene(rng, H, W, B)
    base = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    ref = oracle_out(oracle, wavelet, pan, ms)
    pitch = W + 2
    pv, _ = padded(pan, dev, pitch)
    mv, _ = padded(ms, dev, W // 2 + 1)
    ctx = fz.context(dev)
    try:
        for seg, wpb, nc, var in W2MOD4_TILES:
            say(wavelet, "16-byte rows, W = 2 mod 4", H, W, "tile", seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            ov, obuf = padded(np.zeros((B, H, W), np.float32), dev, pitch)
            fz.fuse(pv, mv, wavelet, out=ov)
            got = ov.cpu().numpy()
            assert bool(torch.isnan(obuf[..., W:]).all()), ("output padding written", seg, wpb, nc, var)
            if wavelet == "haar":
                assert np.array_equal(got, ref.astype(np.float32)), (seg, wpb, nc, var)
            else:
                assert np.abs(got - ref).max() <= D4_TOL, (seg, wpb, nc, var)
            assert np.array_equal(got, base), (seg, wpb, nc, var)
    finally:
        ctx.force_tile(0, 0, 0, 0)


@pytest.mark.parametrize("variant", [0, 3])
def test_16_byte_rows_with_w_2_mod_4_batched(dev, fz, oracle, variant):
    """The same padded layouts as one batch (default form and the forced flat
    grid, whose D4 scenes on 16-byte rows run the LDS-staged tile): each
    output equals its contiguous per-image call bit for bit and the oracle."""
    rng = np.random.default_rng(31 + variant)
    scenes, host, bufs = [], [], []
    for i, (H, W) in enumerate(W2MOD4_SHAPES * 2):
        w = "d4" if i < len(W2MOD4_SHAPES) else "haar"
        B = 3 + i % 3
        pan, ms = int_scene(rng, H, W, B)
        pv, _ = padded(pan, dev, W + 2)
        mv, _ = padded(ms, dev, W // 2 + 1)
        ov, obuf = padded(np.zeros((B, H, W), np.float32), dev, W + 2)
        scenes.append(dict(pan=pv, ms=mv, out=ov, wavelet=w))
        host.append((w, pan, ms))
        bufs.append(obuf)
    ctx = fz.context(dev)
    say("16-byte rows, W = 2 mod 4, batched variant", variant)
    try:
        ctx.force_tile(0, 0, 0, variant)
        outs = fz.fuse_batched(scenes)
    finally:
        ctx.force_tile(0, 0, 0, 0)
    for o, obuf, (w, pan, ms) in zip(outs, bufs, host):
        W = pan.shape[1]
        assert bool(torch.isnan(obuf[..., W:]).all())
        got = o.cpu().numpy()
        assert np.array_equal(got, fz.fuse(to_dev(pan, dev), to_dev(ms, dev), w).cpu().numpy())
        ref = oracle_out(oracle, w, pan, ms)
        if w == "haar":
            assert np.array_equal(got, ref.astype(np.float32))
        else:
            assert np.abs(got - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_cyclic_shift_equivariance(dev, fz, wavelet):
    """Shifting PAN by (2r, 2c) and MS by (r, c) shifts the output by (2r, 2c):
    pins the periodic wrap without the oracle."""
    rng = np.random.default_rng(77)
    pan, ms = int_scene(rng, 96, 520, 2)
    say(wavelet, "shift")
    out = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    for r, c in [(1, 0), (0, 1), (5, 131), (47, 259)]:
        o2 = fz.fuse(to_dev(np.roll(pan, (2 * r, 2 * c), (0, 1)), dev),
                     to_dev(np.roll(ms, (r, c), (1, 2)), dev), wavelet).cpu().numpy()
        assert np.array_equal(o2, np.roll(out, (2 * r, 2 * c), (1, 2)))


def test_ms_equal_to_ll_reproduces_pan(dev, fz, oracle):
    rng = np.random.default_rng(3)
    pan, _ = int_scene(rng, 130, 258, 1)
    for w in ("haar", "d4"):
        ll = oracle.dwt2_fwd(w, pan.astype(np.float64))[:65, :129].astype(np.float32)
        say(w, "ms=LL(pan)")
        out = fz.fuse(to_dev(pan, dev), to_dev(ll[None], dev), w).cpu().numpy()[0]
        tol = 0 if w == "haar" else D4_TOL
        assert np.abs(out - pan).max() <= tol


def test_errors_surface_as_exceptions(dev, fz):
    from paper_1803_00737_amd._lib import DwtFuseError

    pan = torch.zeros(8, 8, device=dev)
    ms = torch.zeros(1, 4, 4, device=dev)
    with pytest.raises(DwtFuseError, match="E_ALIAS"):
        fz.fuse(pan, ms, "d4", out=pan.view(1, 8, 8))
    # zero bands: an empty tensor has a NULL data pointer, which the library
    # reports first (E_NULL); either way nothing is launched
    with pytest.raises(DwtFuseError, match="E_NULL|E_SHAPE"):
        fz.fuse(pan, torch.zeros(0, 4, 4, device=dev), "d4")
    with pytest.raises(DwtFuseError, match="E_SHAPE"):  # odd H: rejected by the library
        fz.fuse(torch.zeros(7, 8, device=dev), torch.zeros(1, 3, 4, device=dev), "d4")
    with pytest.raises(ValueError):  # MS shape does not match PAN: rejected by the binding
        fz.fuse(torch.zeros(8, 8, device=dev), torch.zeros(1, 3, 4, device=dev), "d4")
    with pytest.raises(ValueError):
        fz.fuse(pan, ms, "db8")
    # backward: gain of the wrong length is rejected by the binding
    with pytest.raises(ValueError):
        fz.fuse_backward(pan, torch.zeros(2, 8, 8, device=dev), "d4", torch.ones(3, device=dev))
    with pytest.raises(DwtFuseError, match="E_ALIAS"):  # gradient output aliasing an input
        from paper_1803_00737_amd.api import context, _ptr
        c = context(dev)
        gy = torch.zeros(1, 8, 8, device=dev)
        c.check(c.lib.dwt_fuse_backward(c.handle, 1, 8, 8, 1, _ptr(pan), 8, None, _ptr(gy), 8, 64, _ptr(gy), None,
                                        None), "dwt_fuse_backward")


def test_nan_propagates(dev, fz):
    pan = torch.full((16, 16), 10.0, device=dev)
    pan[5, 7] = float("nan")
    ms = torch.ones(1, 8, 8, device=dev)
    out = fz.fuse(pan, ms, "d4")
    assert torch.isnan(out).any() and not torch.isnan(out).all()
    out = fz.fuse(pan, ms, "haar")
    assert int(torch.isnan(out).sum()) == 4  # only the 2x2 block holding the NaN


# ---- full-size workloads, sampled --------------------------------------

def sample_points(H, W, B, seg_rows_hint, n, rng):
    ys = [0, 1, 2, H - 1, H - 2, H // 2, H // 2 + 1]
    xs = [0, 1, 2, 3, W - 1, W - 2, W - 3, W // 2]
    # unit and strip seams
    for k in (1, 2, 3):
        ys += [min(H - 1, 2 * seg_rows_hint * k), min(H - 1, 2 * seg_rows_hint * k - 1)]
    for k in (1, 2, 5):
        xs += [min(W - 1, 256 * k), min(W - 1, 256 * k - 1), min(W - 1, 512 * k - 1)]
    pts = [(b, y, x) for b in range(B) for y in ys for x in xs[:6]]
    pts += [(int(rng.integers(B)), int(rng.integers(H)), int(rng.integers(W))) for _ in range(n)]
    return pts


def check_full_size(dev, fz, oracle, wl, n=600):
    """Sampled parity at a full workload size, in the launch configuration the
    benchmark times (tuner on: the shape it picks for this size class)."""
    say("full size", wl.name, "generate")
    pan_d, ms_d = wl.make(device=dev)
    torch.cuda.synchronize()
    say("full size", wl.name, "fuse (tuned)")
    ctx = fz.context(dev)
    ctx.set_tuning(True)
    try:
        out_d = fz.fuse(pan_d, ms_d, wl.wavelet)
    finally:
        ctx.set_tuning(False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    pts = sample_points(wl.H, wl.W, wl.B, 16, n, rng)
    b, y, x = map(np.array, zip(*pts))
    got = out_d[torch.from_numpy(b).to(dev), torch.from_numpy(y).to(dev), torch.from_numpy(x).to(dev)].cpu().numpy()
    pan = pan_d.cpu().numpy().astype(np.float64)
    ms = ms_d.cpu().numpy().astype(np.float64)
    ref = oracle.fuse_points(wl.wavelet, pan, ms, None, b, y, x)
    del out_d, pan_d, ms_d
    torch.cuda.empty_cache()
    return got, ref


def test_full_size_d4_8192(dev, fz, oracle):
    from paper_1803_00737_amd import synth

    got, ref = check_full_size(dev, fz, oracle, synth.d4_8192())
    assert np.abs(got - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_full_size_landsat(dev, fz, oracle, wavelet):
    from paper_1803_00737_amd import synth

    got, ref = check_full_size(dev, fz, oracle, synth.landsat(wavelet), n=400)
    if wavelet == "haar":
        assert np.array_equal(got, ref.astype(np.float32))
    else:
        assert np.abs(got - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_full_width_landsat_rows(dev, fz, oracle, wavelet):
    """Whole rows of the Landsat-shaped scene (15872 x 14336, 6 bands) in the
    launch configuration the benchmark times (tuner on): the top and bottom
    64 rows, whose D4 taps wrap to the opposite border (Eq. 5-6, 13-14), and
    an interior strip across tile and unit seams, every column of every band
    element by element against the row-strip oracle."""
    from paper_1803_00737_amd import synth

    wl = synth.landsat(wavelet)
    say("full width", wl.name, "generate")
    pan_d, ms_d = wl.make(device=dev)
    ctx = fz.context(dev)
    ctx.set_tuning(True)
    try:
        say("full width", wl.name, "fuse (tuned)")
        out_d = fz.fuse(pan_d, ms_d, wavelet)
    finally:
        ctx.set_tuning(False)
    torch.cuda.synchronize()
    strips = [(0, 64), (4000, 4064), (wl.H - 64, wl.H)]
    got = [out_d[:, a:b].cpu().numpy() for a, b in strips]
    pan = pan_d.cpu().numpy().astype(np.float64)
    ms = ms_d.cpu().numpy().astype(np.float64)
    del out_d, pan_d, ms_d
    torch.cuda.empty_cache()
    for (a, b), g in zip(strips, got):
        say("full width", wl.name, "oracle rows", a, b)
        ref = oracle.fuse_rows(wavelet, pan, ms, a, b)
        if wavelet == "haar":
            assert np.array_equal(g, ref.astype(np.float32)), (a, b)
        else:
            assert np.abs(g - ref).max() <= D4_TOL, (a, b)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_output_beyond_2_pow_31_elements(dev, fz, oracle, wavelet):
    """PAN 8192 x 8192 with 33 bands: the output holds 2.2e9 float32 elements
    (8.9 GB), more than a 32-bit index can address, so every band offset must
    be formed in 64-bit arithmetic.  Sampled pixels of the first and last
    bands against the single-pixel oracle, in the tuned launch shape."""
    H = W = 8192
    B = 33
    rng = np.random.default_rng(33)
    say("beyond 2^31", wavelet, "generate")
    pan_d = torch.randint(0, 256, (H, W), device=dev).float()
    ms1 = torch.randint(0, 256, (1, H // 2, W // 2), device=dev).float()
    ms_d = ms1.expand(B, H // 2, W // 2).contiguous()
    ms_d[B - 1] = torch.flip(ms1[0], dims=[0])  # a last band that differs from the others
    ctx = fz.context(dev)
    ctx.set_tuning(True)
    try:
        say("beyond 2^31", wavelet, "fuse")
        out = fz.fuse(pan_d, ms_d, wavelet)
    finally:
        ctx.set_tuning(False)
    torch.cuda.synchronize()
    assert out.numel() > 2 ** 31
    pts = [(b, int(y), int(x)) for b in (0, 1, B - 2, B - 1) for y, x in
           zip(rng.integers(0, H, 24), rng.integers(0, W, 24))] + [(B - 1, H - 1, W - 1), (B - 1, 0, 0)]
    b, y, x = map(np.array, zip(*pts))
    got = out[torch.from_numpy(b).to(dev), torch.from_numpy(y).to(dev), torch.from_numpy(x).to(dev)].cpu().numpy()
    pan = pan_d.cpu().numpy().astype(np.float64)
    ms_small = np.stack([ms_d[k].cpu().numpy() for k in (0, B - 1)]).astype(np.float64)
    del out, ms_d, pan_d
    torch.cuda.empty_cache()
    bi = np.where(b == B - 1, 1, 0)
    ref = oracle.fuse_points(wavelet, pan, ms_small, None, bi, y, x)
    if wavelet == "haar":
        assert np.array_equal(got, ref.astype(np.float32))
    else:
        assert np.abs(got - ref).max() <= D4_TOL
