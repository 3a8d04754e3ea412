"""Adjoint kernel: gradients w.r.t. PAN, MS and the per-band detail gain,
against the FP64 oracle's transpose, a dot-product test, FP64 central finite
differences of an MSE loss on 32x32 crops, and autograd end to end.

Tolerances (float32 sums of at most 16 terms per gradient pixel; gain
gradients are sums over the whole image, accumulated in float32 per lane
and across the wavefront for each coefficient row of a strip, then in FP64
across those (row, strip) slots):
  grad_pan, grad_ms: max-abs <= 1e-5 * max(1, max|reference|) * 16
  grad_gain:         |err| <= 1e-5 * sum|y_b * D| + 1e-6
"""
import numpy as np
import pytest

from gpu_helpers import int_scene, require_gpu, say, strided_view, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


def detail_part(oracle, w, pan):
    """PAN minus its LL-only reconstruction (FP64, via the oracle)."""
    ms_ll = oracle.dwt2_fwd(w, pan)[: pan.shape[0] // 2, : pan.shape[1] // 2]
    return pan - oracle.fuse(w, pan, ms_ll[None], [0.0])[0]


def check_grads(oracle, w, pan, gy, gain, got):
    gp, gm, gg = got
    rp, rm, rg = oracle.fuse_backward(w, pan.astype(np.float64), None if gain is None else gain.astype(np.float64),
                                      gy.astype(np.float64))
    tol_p = 16e-5 * max(1.0, np.abs(rp).max())
    tol_m = 16e-5 * max(1.0, np.abs(rm).max())
    assert np.abs(gp - rp).max() <= tol_p
    assert np.abs(gm - rm).max() <= tol_m
    D = detail_part(oracle, w, pan.astype(np.float64))
    for b in range(gy.shape[0]):
        bound = 1e-5 * np.abs(gy[b] * D).sum() + 1e-6
        assert abs(gg[b] - rg[b]) <= bound, (b, gg[b], rg[b], bound)


# widths = 2 mod 4 take the 64-bit path, multiples of 4 the 128-bit one
# (1288 = 5 full 256-column strips + a partial one; odd H/2 = partial units)
SHAPES = [(2, 2), (4, 6), (34, 70), (66, 1030), (130, 258), (64, 4070), (8, 8), (34, 136), (130, 1288),
          (66, 516), (2, 4)]


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("B", [1, 4, 10])
def test_adjoint_matches_oracle(dev, fz, oracle, wavelet, H, W, B):
    rng = np.random.default_rng(H + W + B)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    say("adjoint", wavelet, H, W, B)
    got = fz.fuse_backward(to_dev(pan, dev), to_dev(gy, dev), wavelet, to_dev(gain, dev))
    check_grads(oracle, wavelet, pan, gy, gain, [t.cpu().numpy() for t in got])


@pytest.mark.parametrize("H,W,B,wavelet", [(1030, 2050, 3, "d4"), (1024, 1024, 6, "d4"), (514, 2048, 2, "haar"),
                                            (258, 1030, 9, "d4")])
def test_adjoint_tuner_keeps_results(dev, fz, oracle, H, W, B, wavelet):
    """The adjoint tuner (rolling units, one-shot and LDS-staged tiles, unit
    orders, timed on the call's own buffers) picks a shape whose gradients
    equal the default shape's bit for bit (every candidate keeps the path's
    strip width, so grad_gain keeps its slot layout; above 8 bands grad_pan
    within rounding) and meet the oracle's bound; a second call replays the
    tuned shape."""
    rng = np.random.default_rng(H + W + B)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    p, y, g = to_dev(pan, dev), to_dev(gy, dev), to_dev(gain, dev)
    say("adjoint tuner", H, W, B, wavelet)
    ref = [t.cpu().numpy() for t in fz.fuse_backward(p, y, wavelet, g)]
    ctx = fz.Context(dev.index or 0)  # a context of its own: empty tuning table
    ctx.bind_stream()
    ctx.set_tuning(True)
    from paper_1803_00737_amd import _lib

    def run():
        gp = torch.empty((H, W), device=dev)
        gm = torch.empty((B, H // 2, W // 2), device=dev)
        gg = torch.empty(B, device=dev)
        wid = _lib.wavelet_id(wavelet)
        ctx.check(ctx.lib.dwt_fuse_backward(ctx.handle, wid, H, W, B, p.data_ptr(), W, g.data_ptr(), y.data_ptr(), W,
                                            H * W, gp.data_ptr(), gm.data_ptr(), gg.data_ptr()), "backward")
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in (gp, gm, gg)]

    for rep in range(2):
        got = run()
        for k, (r, q) in enumerate(zip(ref, got)):
            if k == 0 and B > 8:
                # above 8 bands the staged adjoint sums the bands in one pass, the
                # rolling one in groups of 8: grad_pan rounds differently
                assert np.abs(r - q).max() <= 16e-5 * max(1.0, np.abs(r).max())
            else:
                assert np.array_equal(r, q), (rep, k)
    check_grads(oracle, wavelet, pan, gy, gain, got)


@pytest.mark.parametrize("H,W,B", [(130, 1030, 3), (66, 516, 6)])
def test_adjoint_unit_orders(dev, fz, H, W, B):
    """Every unit order of the rolling, one-shot and LDS-staged adjoints gives
    the gradients of the default order bit for bit."""
    rng = np.random.default_rng(H + W + B)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    p, y, g = to_dev(pan, dev), to_dev(gy, dev), to_dev(gain, dev)
    ctx = fz.context(dev)
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (16, 4, 2, 0), (4, 2, 2, 1), (2, 4, 2, 2), (2, 4, 2, 3)]:
            ctx.force_tile(seg, wpb, nc, var)
            ctx.force_order(-1)
            ref = [t.cpu().numpy() for t in fz.fuse_backward(p, y, "d4", g)]
            for order in (0, 1, 2, 3):
                say("adjoint order", order, H, W, B, seg, wpb, nc, var)
                ctx.force_order(order)
                got = [t.cpu().numpy() for t in fz.fuse_backward(p, y, "d4", g)]
                for r, q in zip(ref, got):
                    assert np.array_equal(r, q), (order, seg, wpb, nc, var)
    finally:
        ctx.force_tile(0, 0, 0, 0)
        ctx.force_order(-1)


@pytest.mark.parametrize("H,W", [(8, 8), (34, 136), (130, 1288), (66, 516), (2, 4), (66, 1030)])
@pytest.mark.parametrize("B", [1, 4, 6, 10])
def test_forced_adjoint_shapes(dev, fz, oracle, H, W, B):
    """Forced launch shapes of the adjoint: rolling wavefronts with several
    rows per unit / waves per workgroup / columns per lane (variant 0: the
    band loop unrolled for up to 4 bands; variant 1: a dynamic band loop),
    one-shot tiles of
    1 or 2 rows (variant 2), and the LDS-staged D4 adjoint (variant 3, 1 or 2
    rows per wavefront; upstream gradients staged a group of bands at a time,
    or with 1 column per lane requested, band after band in two buffers).  Every shape must meet the oracle's tolerance; all
    of them form every per-pixel gradient with the same fma chains in the same
    order, so grad_pan and grad_ms also agree bit for bit.  The gain products
    are summed per (coefficient row, strip) whatever the unit length, so
    grad_gain agrees bit for bit between shapes with the same strip width
    (128 columns: two columns per lane, on 16- or 8-byte rows, and the staged
    kernel; 64 columns: one column per lane)."""
    rng = np.random.default_rng(7 * H + W + B)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    p, y, g = to_dev(pan, dev), to_dev(gy, dev), to_dev(gain, dev)
    ctx = fz.context(dev)
    outs = []
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (1, 1, 1, 1), (3, 2, 2, 1), (16, 4, 2, 1), (200, 1, 1, 1),
                                  (1, 1, 1, 0), (3, 2, 2, 0), (16, 4, 2, 0), (200, 1, 1, 0),
                                  (1, 4, 2, 2), (2, 2, 2, 2), (2, 1, 1, 2), (1, 2, 1, 2),
                                  (1, 4, 2, 3), (2, 2, 2, 3), (1, 1, 2, 3), (2, 4, 2, 3), (1, 4, 1, 3),
                                  (2, 2, 1, 3)]:
            say("adjoint forced", H, W, B, seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            got = [t.cpu().numpy() for t in fz.fuse_backward(p, y, "d4", g)]
            check_grads(oracle, "d4", pan, gy, gain, got)
            outs.append((seg, wpb, nc, var, got))
    finally:
        ctx.force_tile(0, 0, 0, 0)

    def strip_cols(seg, wpb, nc, var):
        if (seg, wpb, nc, var) == (0, 0, 0, 0):  # default: staged from 5 bands on 16-byte rows, else 2 columns
            return 128
        return 128 if var == 3 or nc != 1 else 64

    def staged(seg, wpb, nc, var):  # contiguous rows: 16- or 8-byte aligned, both staged
        return var == 3 or ((seg, wpb, nc, var) == (0, 0, 0, 0) and B >= 5)

    for r in outs:
        ref = next(q for q in outs if strip_cols(*q[:4]) == strip_cols(*r[:4]))
        assert np.array_equal(r[4][2], ref[4][2]), ("grad_gain differs", r[:4], ref[:4])
        # Above 8 bands the rolling and one-shot kernels sum grad_pan over
        # groups of 8 bands and add the groups; the staged kernel sums all
        # bands in one pass, so only kernels of the same kind agree bit for bit.
        ref = next(q for q in outs if B <= 8 or staged(*q[:4]) == staged(*r[:4]))
        assert np.array_equal(r[4][0], ref[4][0]), ("grad_pan differs", r[:4], ref[:4])
        assert np.array_equal(r[4][1], outs[0][4][1]), ("grad_ms differs", r[:4])


@pytest.mark.parametrize("H,W", [(8, 8), (34, 136), (130, 1288), (66, 516), (34, 134), (66, 1030), (2, 2)])
@pytest.mark.parametrize("B", [1, 3, 4, 6])
def test_haar_adjoint_band_loop_forms(dev, fz, oracle, H, W, B):
    """Haar adjoint: the band loop unrolled (default up to 4 bands) and the
    dynamic band loop in groups of 4 bands (forced variant 1; the default
    above 4 bands), at several unit lengths, take the same fma chains, so all
    three gradients agree bit for bit, and meet the oracle's tolerance."""
    rng = np.random.default_rng(11 * H + W + B)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    p, y, g = to_dev(pan, dev), to_dev(gy, dev), to_dev(gain, dev)
    ctx = fz.context(dev)
    outs = []
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (1, 1, 1, 1), (7, 2, 2, 1), (32, 4, 2, 1), (3, 4, 2, 0),
                                  (1, 1, 1, 0), (64, 1, 2, 0)]:
            say("haar adjoint", H, W, B, seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            got = [t.cpu().numpy() for t in fz.fuse_backward(p, y, "haar", g)]
            check_grads(oracle, "haar", pan, gy, gain, got)
            outs.append(((seg, wpb, nc, var), got))
    finally:
        ctx.force_tile(0, 0, 0, 0)
    def strip_cols(seg, wpb, nc, var):
        return 128 if nc != 1 else 64

    for shape, o in outs[1:]:
        assert np.array_equal(o[0], outs[0][1][0]), ("grad_pan differs", shape)
        assert np.array_equal(o[1], outs[0][1][1]), ("grad_ms differs", shape)
        ref = next(q for q in outs if strip_cols(*q[0]) == strip_cols(*shape))
        assert np.array_equal(o[2], ref[1][2]), ("grad_gain differs", shape, ref[0])


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(8, 8), (34, 136), (66, 516), (10, 1292), (34, 134), (10, 1290), (6, 6)])
def test_adjoint_writes_stay_inside(dev, fz, wavelet, H, W):
    """Lanes past the last coefficient column of a strip (W/2 not a multiple
    of the strip width; on 8-byte rows W/2 is odd, so one lane holds a valid
    and an invalid column) store nothing: grad_pan and grad_ms are views into
    larger buffers whose other elements hold a sentinel, and every forced
    adjoint shape must leave the sentinels alone."""
    import ctypes

    B = 3
    rng = np.random.default_rng(H * W)
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    p, y = to_dev(pan, dev), to_dev(gy, dev)
    gain = torch.ones(B, device=dev)
    npan, nms = H * W, B * (H // 2) * (W // 2)
    sentinel = 12345.0
    ctx = fz.context(dev)
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (1, 1, 1, 1), (16, 4, 2, 1), (3, 2, 2, 0), (1, 4, 2, 2),
                                  (2, 2, 2, 2), (1, 4, 2, 3), (2, 2, 1, 3)]:
            say("adjoint sentinel", wavelet, H, W, seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            gp = torch.full((npan + 4096,), sentinel, device=dev)
            gm = torch.full((nms + 4096,), sentinel, device=dev)
            gg = torch.full((B + 64,), sentinel, device=dev)
            ctx.check(ctx.lib.dwt_fuse_backward(ctx.handle, 0 if wavelet == "haar" else 1, H, W, B,
                                                ctypes.c_void_p(p.data_ptr()), W, ctypes.c_void_p(gain.data_ptr()),
                                                ctypes.c_void_p(y.data_ptr()), W, H * W,
                                                ctypes.c_void_p(gp.data_ptr()), ctypes.c_void_p(gm.data_ptr()),
                                                ctypes.c_void_p(gg.data_ptr())), "dwt_fuse_backward")
            torch.cuda.synchronize(dev)
            assert bool((gp[npan:] == sentinel).all()), ("grad_pan tail written", seg, wpb, nc, var)
            assert bool((gm[nms:] == sentinel).all()), ("grad_ms tail written", seg, wpb, nc, var)
            assert bool((gg[B:] == sentinel).all()), ("grad_gain tail written", seg, wpb, nc, var)
            assert bool(torch.isfinite(gp[:npan]).all()) and bool(torch.isfinite(gm[:nms]).all())
    finally:
        ctx.force_tile(0, 0, 0, 0)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("pad,offset", [(4, 0), (2, 2), (1, 1)])
def test_adjoint_paths(dev, fz, oracle, wavelet, pad, offset):
    rng = np.random.default_rng(pad + offset)
    H, W, B = 34, 134, 3
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    say("adjoint paths", wavelet, pad, offset)
    got = fz.fuse_backward(strided_view(pan, dev, pad, offset), strided_view(gy, dev, pad, offset), wavelet)
    check_grads(oracle, wavelet, pan, gy, None, [t.cpu().numpy() for t in got])


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_dot_product(dev, fz, wavelet):
    """<J x, y> = <x, J^T y> for the map (pan, ms) -> out at fixed gains."""
    rng = np.random.default_rng(11)
    H, W, B = 66, 264, 3
    pan = to_dev(rng.normal(size=(H, W)).astype(np.float32), dev)
    ms = to_dev(rng.normal(size=(B, H // 2, W // 2)).astype(np.float32), dev)
    y = to_dev(rng.normal(size=(B, H, W)).astype(np.float32), dev)
    gain = to_dev(rng.uniform(0.5, 1.5, B).astype(np.float32), dev)
    say("dot product", wavelet)
    out = fz.fuse(pan, ms, wavelet, gain)
    gp, gm, _ = fz.fuse_backward(pan, y, wavelet, gain, need_gain=False)
    lhs = (out.double() * y.double()).sum().item()
    rhs = (pan.double() * gp.double()).sum().item() + (ms.double() * gm.double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs)) + 1e-3


def _adjoint_identities(fz, pan, ms, y, gain, wavelet, grads):
    """At any size: <F(pan, ms), y> = <pan, grad_pan> + <ms, grad_ms> (the map
    is linear in (pan, ms) at fixed gains), and grad_gain_b = <y_b, D_b> with
    D_b = F(gain 1)_b - F(gain 0)_b = PAN - P PAN.  Sums in FP64.  The bounds
    scale with the sums of absolute products: float32 rounding of each output
    and gradient element is unbiased and independent, so the sums drift by
    about sqrt(n) roundings, some 10^-11 of the scale here; 10^-8 (10^-7 for
    grad_gain, summed in float32 along rows of 512 products) leaves a margin
    of over 20x, while a wrong row of gradients would move the sums by an
    estimated ~10^-6 of the scale."""
    gp, gm, gg = grads
    out = fz.fuse(pan, ms, wavelet, gain)
    prod = out.double() * y.double()
    lhs = prod.sum().item()
    scale = prod.abs().sum().item()
    del prod, out
    rhs = (pan.double() * gp.double()).sum().item() + (ms.double() * gm.double()).sum().item()
    assert abs(lhs - rhs) <= 1e-8 * scale + 1e-3, (lhs, rhs, scale)
    B = y.shape[0]
    one = torch.ones(B, device=pan.device)
    d = fz.fuse(pan, ms, wavelet, one) - fz.fuse(pan, ms, wavelet, torch.zeros(B, device=pan.device))
    for b in range(B):
        prod = d[b].double() * y[b].double()
        ref = prod.sum().item()
        bound = 1e-7 * prod.abs().sum().item() + 1e-3
        assert abs(float(gg[b]) - ref) <= bound, (b, float(gg[b]), ref, bound)
    del d


@pytest.mark.parametrize("H,W,B", [(8192, 8192, 3), (8192, 8190, 6)])
def test_full_size_adjoint_identities(dev, fz, H, W, B):
    """Full-size adjoint in the configuration the benchmark times (D4 8192^2
    with 3 bands: band-unrolled rolling units; 8-byte rows with 6 bands: the
    LDS-staged adjoint), checked through identities that hold at any size."""
    from paper_1803_00737_amd import synth

    say("full-size adjoint identities", H, W, B)
    pan, ms = synth.make_scene(H, W, B, synth.seed_for(2, 0), device=dev)
    y = torch.randn((B, H, W), device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    gain = torch.linspace(0.5, 1.5, B, device=dev)
    grads = fz.fuse_backward(pan, y, "d4", gain)
    _adjoint_identities(fz, pan, ms, y, gain, "d4", grads)
    torch.cuda.empty_cache()


def test_full_size_batched_adjoint_identities(dev, fz):
    """The differentiation workload's adjoint (16 scenes of 2048^2 with 4
    bands in one batched call, 64-row units) satisfies the same identities
    scene by scene."""
    from paper_1803_00737_amd import synth

    H = W = 2048
    B = 4
    gain = torch.ones(B, device=dev)
    scenes, inputs = [], []
    for s in range(16):
        pan, ms = synth.make_scene(H, W, B, synth.seed_for(4, s), device=dev)
        y = torch.randn((B, H, W), device=dev, generator=torch.Generator(device=dev).manual_seed(100 + s))
        scenes.append(dict(pan=pan, grad_out=y, wavelet="d4", gain=gain))
        inputs.append((pan, ms, y))
    say("full-size batched adjoint identities")
    got = fz.fuse_backward_batched(scenes)
    for (pan, ms, y), g in zip(inputs, got):
        _adjoint_identities(fz, pan, ms, y, gain, "d4", g)


@pytest.mark.parametrize("wavelet", ["d4", "haar"])
def test_autograd_vs_fp64_finite_differences(dev, fz, oracle, wavelet):
    """MSE(fused, target) on a 32x32 crop (4 bands, gain initialised to 1):
    autograd through the fused kernel and the adjoint kernel vs FP64 central
    differences through the oracle (exact up to rounding: the loss is
    quadratic in every input)."""
    rng = np.random.default_rng(32)
    H = W = 32
    B = 4
    pan, ms = int_scene(rng, H, W, B)
    tgt_gain = rng.uniform(0.8, 1.2, B)
    target = (pan[None].astype(np.float64) * tgt_gain[:, None, None])
    p = to_dev(pan, dev).requires_grad_(True)
    m = to_dev(ms, dev).requires_grad_(True)
    g = torch.ones(B, device=dev, requires_grad=True)
    say("autograd", wavelet)
    out = fz.DwtFuseFn.apply(p, m, g, wavelet)
    loss = ((out - to_dev(target.astype(np.float32), dev)) ** 2).mean()
    loss.backward()
    count = B * H * W

    def L(pp, mm, gg):
        return ((oracle.fuse(wavelet, pp, mm, gg) - target) ** 2).sum() / count

    pan64, ms64, g64 = pan.astype(np.float64), ms.astype(np.float64), np.ones(B)
    eps = 0.5
    gp, gm, gg = p.grad.cpu().numpy(), m.grad.cpu().numpy(), g.grad.cpu().numpy()
    for _ in range(8):
        y, x = rng.integers(0, H, 2)
        d = np.zeros_like(pan64)
        d[y, x] = eps
        fd = (L(pan64 + d, ms64, g64) - L(pan64 - d, ms64, g64)) / (2 * eps)
        assert abs(fd - gp[y, x]) <= 1e-4 * max(1.0, abs(fd))
        b, i, j = rng.integers(0, B), rng.integers(0, 16), rng.integers(0, 16)
        d = np.zeros_like(ms64)
        d[b, i, j] = eps
        fd = (L(pan64, ms64 + d, g64) - L(pan64, ms64 - d, g64)) / (2 * eps)
        assert abs(fd - gm[b, i, j]) <= 1e-4 * max(1.0, abs(fd))
    for b in range(B):
        e = np.zeros(B)
        e[b] = 1e-3
        fd = (L(pan64, ms64, g64 + e) - L(pan64, ms64, g64 - e)) / 2e-3
        assert abs(fd - gg[b]) <= 1e-3 * max(1.0, abs(fd))


def test_differentiation_workload_finite_differences(dev, fz, oracle):
    """Scene 0 of the 16 x 2048^2 (4 bands, D4) differentiation workload:
    autograd through DwtFuseFn on the whole scene against FP64 central
    differences of the whole-scene MSE, for PAN pixels and MS coefficients in
    32 x 32 (16 x 16) windows in the interior and at the wrap seams (corners
    and edges), and for every band's gain.  A PAN or MS perturbation changes
    only a few output rows (D4 support), so the loss difference is evaluated
    with the row-strip oracle over the rows it can change (wrapped), exactly
    as over the whole scene; the loss is quadratic, so central differences
    are exact up to rounding."""
    from paper_1803_00737_amd import synth

    H = W = 2048
    B = 4
    seed = synth.seed_for(4, 0)
    pan_d, ms_d = synth.make_scene(H, W, B, seed, device=dev)
    tg = synth.grad_targets(B, seed)
    p = pan_d.clone().requires_grad_(True)
    m = ms_d.clone().requires_grad_(True)
    g = torch.ones(B, device=dev, requires_grad=True)
    say("differentiation FD windows: autograd")
    out = fz.DwtFuseFn.apply(p, m, g, "d4")
    target_d = pan_d[None] * torch.tensor(tg, dtype=torch.float32, device=dev)[:, None, None]
    ((out - target_d) ** 2).mean().backward()
    gp, gm, gg = p.grad.cpu().numpy(), m.grad.cpu().numpy(), g.grad.cpu().numpy()
    pan = pan_d.cpu().numpy().astype(np.float64)
    ms = ms_d.cpu().numpy().astype(np.float64)
    target = pan[None] * tg[:, None, None]  # a constant: computed from the unperturbed PAN
    count = B * H * W

    def row_ranges(lo, hi):  # output rows lo .. hi-1, wrapped, as contiguous ranges
        rows = [(lo + k) % H for k in range(hi - lo)]
        out_r, start = [], rows[0]
        for a, b in zip(rows, rows[1:] + [None]):
            if b is None or b != a + 1:
                out_r.append((start, a + 1))
                start = b
        return out_r

    def local_loss(pp, mm, gain, rows):
        total = 0.0
        for a, b in rows:
            f = oracle.fuse_rows("d4", pp, mm, a, b, gain)
            total += ((f - target[:, a:b]) ** 2).sum()
        return total / count

    ones = np.ones(B)
    eps = 0.5
    fd_p, got_p, fd_m, got_m = [], [], [], []
    rng = np.random.default_rng(11)
    for (y0, x0) in [(1000, 1000), (0, 0), (H - 32, W - 32), (0, W // 2), (H // 2, W - 32)]:
        say("differentiation FD windows: window", y0, x0)
        for _ in range(3):
            y, x = y0 + int(rng.integers(0, 32)), x0 + int(rng.integers(0, 32))
            rows = row_ranges(y - 6, y + 7)
            d = np.zeros_like(pan)
            d[y, x] = eps
            fd_p.append((local_loss(pan + d, ms, ones, rows) - local_loss(pan - d, ms, ones, rows)) / (2 * eps))
            got_p.append(gp[y, x])
            b, i, j = int(rng.integers(0, B)), y0 // 2 + int(rng.integers(0, 16)), x0 // 2 + int(rng.integers(0, 16))
            rows = row_ranges(2 * i - 4, 2 * i + 8)
            d = np.zeros_like(ms)
            d[b, i, j] = eps
            fd_m.append((local_loss(pan, ms + d, ones, rows) - local_loss(pan, ms - d, ones, rows)) / (2 * eps))
            got_m.append(gm[b, i, j])
    fd_p, got_p, fd_m, got_m = map(np.array, (fd_p, got_p, fd_m, got_m))
    assert np.abs(fd_p - got_p).max() <= 1e-3 * np.abs(fd_p).max()
    assert np.abs(fd_m - got_m).max() <= 1e-3 * np.abs(fd_m).max()
    say("differentiation FD windows: gains")
    # The gain derivative is 2 <out_b - target_b, D> / count with D = PAN - L^T L PAN
    # (the fused output with a zero MS band), a sum over the whole band with
    # much cancellation, so the GPU's float32 forward error e_b (max-abs,
    # measured here against the oracle) enters it by up to
    # 2 e_b sum|D| / count (Hoelder), on top of the adjoint's own rounding.
    D = oracle.fuse("d4", pan, np.zeros((1, H // 2, W // 2)), [1.0])[0]
    out_h = out.detach().cpu().numpy()
    for b in range(B):
        def band_loss(gb):
            f = oracle.fuse("d4", pan, ms[b:b + 1], [gb])[0]
            return ((f - target[b]) ** 2).sum() / count
        f1 = oracle.fuse("d4", pan, ms[b:b + 1], [1.0])[0]
        e_b = np.abs(out_h[b] - f1).max()
        assert e_b <= 1e-3
        fd = (band_loss(1.0 + 1e-3) - band_loss(1.0 - 1e-3)) / 2e-3
        bound = 2 * e_b * np.abs(D).sum() / count + 1e-5 * np.abs(2 * (f1 - target[b]) * D).sum() / count + 1e-9
        assert abs(fd - gg[b]) <= bound, (b, fd, gg[b], bound)


def test_differentiation_workload(dev, fz, oracle):
    """16 scenes of 2048x2048, 4 bands, D4, gain 1, MSE to PAN x U(0.8, 1.2):
    forward + adjoint on every scene; the first two scenes are checked in
    full against the oracle's gradients."""
    from paper_1803_00737_amd import synth

    for s in range(16):
        seed = synth.seed_for(4, s)
        pan, ms = synth.make_scene(2048, 2048, 4, seed, device=dev)
        tg = torch.tensor(synth.grad_targets(4, seed), dtype=torch.float32, device=dev)
        p = pan.clone().requires_grad_(True)
        m = ms.clone().requires_grad_(True)
        g = torch.ones(4, device=dev, requires_grad=True)
        say("differentiation scene", s)
        out = fz.DwtFuseFn.apply(p, m, g, "d4")
        target = pan[None] * tg[:, None, None]
        loss = ((out - target) ** 2).mean()
        loss.backward()
        assert torch.isfinite(p.grad).all() and torch.isfinite(m.grad).all() and torch.isfinite(g.grad).all()
        if s < 2:
            gy = (2.0 / out.numel()) * (out.detach() - target)
            check_grads(oracle, "d4", pan.cpu().numpy(), gy.cpu().numpy(), np.ones(4, np.float32),
                        [p.grad.cpu().numpy(), m.grad.cpu().numpy(), g.grad.cpu().numpy()])


def _bwd_scene(rng, dev, wavelet, H, W, B, pad=0, offset=0, gain=True, need=(True, True, True)):
    pan, _ = int_scene(rng, H, W, 1)
    gy = rng.normal(size=(B, H, W)).astype(np.float32)
    g = rng.uniform(0.5, 1.5, B).astype(np.float32) if gain else None
    p = strided_view(pan, dev, pad, offset) if pad or offset else to_dev(pan, dev)
    y = strided_view(gy, dev, pad, offset) if pad or offset else to_dev(gy, dev)
    return dict(pan=p, grad_out=y, wavelet=wavelet, gain=None if g is None else to_dev(g, dev),
                need_pan=need[0], need_ms=need[1], need_gain=need[2] and gain,
                host=(pan, gy, g))


def _single(fz, s):
    return fz.fuse_backward(s["pan"], s["grad_out"], s["wavelet"], s["gain"], s["need_pan"], s["need_ms"],
                            s["need_gain"])


def _same(a, b):
    for x, y in zip(a, b):
        assert (x is None) == (y is None)
        if x is not None:
            assert torch.equal(x, y)


# (wavelet, H, W, B, pad, offset, gain, need): every adjoint variant and load
# path -- D4 and Haar with <= 4 bands (band loop unrolled), D4 from 5 bands on
# 16- and 8-byte rows (the LDS-staged adjoint, a launch per scene), Haar with
# 6 and 9 bands (groups of 4; two band groups, the second adding into
# grad_pan), 16-byte, 8-byte and 4-byte rows, scenes without grad_gain or
# without any output.
BWD_BATCH = [("d4", 66, 516, 4, 0, 0, True, (True, True, True)),
             ("d4", 34, 70, 3, 0, 0, True, (True, True, True)),
             ("haar", 130, 258, 2, 0, 0, True, (True, True, True)),
             ("d4", 130, 1288, 9, 0, 0, True, (True, True, True)),
             ("haar", 34, 136, 9, 0, 0, False, (True, True, False)),
             ("d4", 34, 134, 3, 2, 2, True, (True, False, True)),
             ("d4", 34, 134, 1, 1, 1, True, (False, True, True)),
             ("haar", 34, 134, 5, 1, 1, True, (True, True, True)),
             ("d4", 8, 8, 2, 0, 0, True, (False, False, False)),
             ("d4", 2, 4, 1, 0, 0, True, (True, True, True)),
             ("d4", 66, 516, 4, 0, 0, False, (True, True, False)),
             ("d4", 66, 1030, 6, 0, 0, True, (True, True, True)),
             ("d4", 34, 134, 9, 0, 0, True, (True, True, True)),
             ("haar", 66, 1030, 6, 0, 0, True, (True, True, True))]


def test_backward_batched_matches_single_calls(dev, fz, oracle):
    """One batched call equals a dwt_fuse_backward call per scene bit for bit
    (same kernel variant per scene, same fma chains, same fixed-order gain sums),
    and meets the oracle's tolerance."""
    rng = np.random.default_rng(99)
    scenes = [_bwd_scene(rng, dev, *c) for c in BWD_BATCH]
    say("backward batched", len(scenes), "scenes")
    got = fz.fuse_backward_batched(scenes)
    for i, (s, g) in enumerate(zip(scenes, got)):
        say("backward batched scene", i, BWD_BATCH[i])
        _same(g, _single(fz, s))
        pan, gy, gain = s["host"]
        if g[0] is not None and g[1] is not None and g[2] is not None:
            check_grads(oracle, s["wavelet"], pan, gy, gain, [t.cpu().numpy() for t in g])


@pytest.mark.parametrize("seg,wpb,nc,var", [(1, 1, 1, 1), (16, 4, 2, 1), (1, 4, 2, 2), (2, 2, 1, 2), (3, 2, 2, 0)])
def test_backward_batched_forced_shapes(dev, fz, seg, wpb, nc, var):
    """Forced adjoint shapes (rolling with a dynamic band loop, one-shot tiles,
    other unit lengths) apply to every scene of a batch as to a single call."""
    rng = np.random.default_rng(seg * 10 + var)
    scenes = [_bwd_scene(rng, dev, *c) for c in BWD_BATCH[:6]]
    ctx = fz.context(dev)
    try:
        ctx.force_tile(seg, wpb, nc, var)
        say("backward batched forced", seg, wpb, nc, var)
        got = fz.fuse_backward_batched(scenes)
        for s, g in zip(scenes, got):
            _same(g, _single(fz, s))
    finally:
        ctx.force_tile(0, 0, 0, 0)


def test_backward_batched_joint_unit_length(dev, fz):
    """Eight 1024^2 D4 scenes with 4 bands: together they fill the GPU with
    units twice as long as one scene alone takes, and the results still equal
    the single calls bit for bit (grad_gain included: its products are kept
    per coefficient row, not per unit)."""
    rng = np.random.default_rng(17)
    scenes = [_bwd_scene(rng, dev, "d4", 1024, 1024, 4) for _ in range(8)]
    say("backward batched joint unit length")
    got = fz.fuse_backward_batched(scenes)
    for s, g in zip(scenes, got):
        _same(g, _single(fz, s))


def test_backward_batched_twice_and_empty(dev, fz):
    """Consecutive batched calls reuse the context's tables (the second call,
    with a smaller batch, must not see the first one's scenes); n = 0 is a
    no-op."""
    rng = np.random.default_rng(5)
    big = [_bwd_scene(rng, dev, *c) for c in BWD_BATCH]
    small = [_bwd_scene(rng, dev, *c) for c in BWD_BATCH[2:4]]
    say("backward batched twice")
    g1 = fz.fuse_backward_batched(big)
    g2 = fz.fuse_backward_batched(small)
    for s, g in zip(big, g1):
        _same(g, _single(fz, s))
    for s, g in zip(small, g2):
        _same(g, _single(fz, s))
    assert fz.fuse_backward_batched([]) == []


def test_backward_batched_rejects_aliasing(dev, fz):
    rng = np.random.default_rng(6)
    a = _bwd_scene(rng, dev, "d4", 34, 70, 2)
    b = _bwd_scene(rng, dev, "d4", 34, 70, 2)
    arr, outs, keep = fz.make_bwd_items([a, b])
    arr[1].grad_pan = arr[0].grad_pan  # two scenes writing one grad_pan
    ctx = fz.context(dev)
    ctx.bind_stream()
    from paper_1803_00737_amd import _lib

    assert ctx.lib.dwt_fuse_backward_batched(ctx.handle, arr, 2) == _lib.E_ALIAS
    arr, outs, keep = fz.make_bwd_items([a, b])
    arr[1].grad_ms = arr[0].grad_out  # a gradient over another scene's upstream gradient
    assert ctx.lib.dwt_fuse_backward_batched(ctx.handle, arr, 2) == _lib.E_ALIAS


def test_differentiation_workload_batched(dev, fz, oracle):
    """The 16 x 2048^2, 4-band D4 step as two batched calls (forward of all
    scenes, then the adjoint of all scenes): gradients equal the per-scene
    calls bit for bit; scene 0 is checked against the oracle."""
    from paper_1803_00737_amd import synth

    scenes, bwd = [], []
    for s in range(16):
        seed = synth.seed_for(4, s)
        pan, ms = synth.make_scene(2048, 2048, 4, seed, device=dev)
        tg = torch.tensor(synth.grad_targets(4, seed), dtype=torch.float32, device=dev)
        scenes.append(dict(pan=pan, ms=ms, wavelet="d4", gain=torch.ones(4, device=dev), tg=tg))
    say("differentiation batched: forward")
    outs = fz.fuse_batched([{k: v for k, v in s.items() if k != "tg"} for s in scenes])
    for s, out in zip(scenes, outs):
        target = s["pan"][None] * s["tg"][:, None, None]
        gy = (2.0 / (16 * out.numel())) * (out - target)
        bwd.append(dict(pan=s["pan"], grad_out=gy, wavelet="d4", gain=s["gain"]))
    say("differentiation batched: adjoint")
    got = fz.fuse_backward_batched(bwd)
    for i, (b, g) in enumerate(zip(bwd, got)):
        _same(g, fz.fuse_backward(b["pan"], b["grad_out"], "d4", b["gain"]))
        if i == 0:
            check_grads(oracle, "d4", b["pan"].cpu().numpy(), b["grad_out"].cpu().numpy(), np.ones(4, np.float32),
                        [t.cpu().numpy() for t in g])


def test_adjoint_beyond_2_31_elements(dev, fz):
    """D4 adjoint of 8192 x 8192 with 33 bands: the upstream gradient holds
    2.2e9 elements (8.9 GB), more than a 32-bit index can address, so band
    offsets must be formed in 64-bit arithmetic (the bands run in groups
    that accumulate into grad_pan).  Checked through the identities of
    _adjoint_identities, summed band by band in FP64: <F, y> = <PAN,
    grad_pan> + <MS, grad_ms>, and grad_gain_b = <y_b, PAN - P PAN>."""
    H = W = 8192
    B = 33
    say("adjoint beyond 2^31", "generate")
    g = torch.Generator(device=dev).manual_seed(33)
    pan = torch.randint(0, 256, (H, W), device=dev, generator=g).float()
    ms = torch.randint(0, 256, (B, H // 2, W // 2), device=dev, generator=g).float()
    y = torch.randn((B, H, W), device=dev, generator=g)
    assert y.numel() > 2 ** 31
    gain = torch.linspace(0.5, 1.5, B, device=dev)
    say("adjoint beyond 2^31", "backward")
    gp, gm, gg = fz.fuse_backward(pan, y, "d4", gain)
    say("adjoint beyond 2^31", "forward and sums")
    out = fz.fuse(pan, ms, "d4", gain)
    lhs = scale = 0.0
    rhs = float((pan.double() * gp.double()).sum())
    rscale = float((pan.double() * gp.double()).abs().sum())
    for b in range(B):
        prod = out[b].double() * y[b].double()
        lhs += float(prod.sum())
        scale += float(prod.abs().sum())
        mprod = ms[b].double() * gm[b].double()
        rhs += float(mprod.sum())
        rscale += float(mprod.abs().sum())
    assert abs(lhs - rhs) <= 1e-8 * max(scale, rscale), (lhs, rhs, scale)
    del out
    one, zero = torch.ones(1, device=dev), torch.zeros(1, device=dev)
    d = (fz.fuse(pan, ms[:1], "d4", one) - fz.fuse(pan, ms[:1], "d4", zero))[0].double()  # PAN - P PAN
    for b in range(B):
        prod = y[b].double() * d
        ref = float(prod.sum())
        bound = 1e-7 * float(prod.abs().sum()) + 1e-3
        assert abs(float(gg[b]) - ref) <= bound, (b, float(gg[b]), ref, bound)
    del y, gp, gm, d
    torch.cuda.empty_cache()
