"""GPU parity of the format variants (dwt_fuse_run_ex): 8-bit or float32
PAN/MS in, 8-bit or float32 out, and the kappa scale of the inserted MS band.

Bars:
  * float32 output from 8-bit input equals the float32 path on the same
    (exactly converted) values bit for bit, and so meets that path's bars
    against the oracle (Haar exact, D4 within 1e-3);
  * 8-bit output equals the oracle's 8-bit code of its FP64 value (nearest
    integer, ties to even, clamp to [0, 255]) exactly for Haar on integer
    inputs (every value is a multiple of 1/4, so float32 is exact); for D4 the
    rounding is decided on the kernel's float32 value, which is within 1e-3
    of the FP64 one, so where the FP64 value lies within 1e-3 of a rounding
    boundary either neighbouring code is accepted and everywhere else the
    code must match exactly;
  * kappa: Haar with kappa in {2, 1/2} stays exact (kappa * m is exact),
    other kappas and D4 within 1e-3 of the oracle's kappa fusion.
"""
import numpy as np
import pytest

from gpu_helpers import D4_TOL, int_scene, require_gpu, say, to_dev, torch

pytestmark = pytest.mark.gpu

SHAPES = [(2, 2), (4, 6), (34, 70), (66, 1030), (130, 258), (64, 4070), (8, 8), (34, 136), (130, 1288),
          (66, 516), (256, 2064), (18, 4098)]


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def fz():
    from paper_1803_00737_amd import api

    return api


def u8_scene(rng, H, W, B):
    pan, ms = int_scene(rng, H, W, B)
    return pan.astype(np.uint8), ms.astype(np.uint8)


def check_u8(oracle, got, ref64, exact):
    want = oracle.quantize_u8(ref64)
    if exact:
        assert np.array_equal(got, want)
        return
    near = np.abs(ref64 - np.floor(ref64) - 0.5) <= D4_TOL
    lo = oracle.quantize_u8(np.floor(ref64))
    hi = oracle.quantize_u8(np.ceil(ref64))
    ok = (got == want) | (near & ((got == lo) | (got == hi)))
    assert ok.all(), (np.argwhere(~ok)[:5], got[~ok][:5], ref64[~ok][:5])


def self_code(f32):
    """8-bit code of the kernel's own float32 values (a property check, not a
    reference: rint is ties-to-even)."""
    return np.clip(np.rint(f32.astype(np.float64)), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("B", [1, 3, 9])
def test_u8_input(dev, fz, oracle, wavelet, H, W, B):
    rng = np.random.default_rng(H * 7 + W + B)
    pan, ms = u8_scene(rng, H, W, B)
    p8, m8 = to_dev(pan, dev), to_dev(ms, dev)
    say("u8 in", wavelet, H, W, B)
    f32 = fz.fuse(p8, m8, wavelet).cpu().numpy()
    base = fz.fuse(to_dev(pan.astype(np.float32), dev), to_dev(ms.astype(np.float32), dev), wavelet).cpu().numpy()
    assert np.array_equal(f32, base)
    say("u8 in u8 out", wavelet, H, W, B)
    q = fz.fuse(p8, m8, wavelet, out_dtype=torch.uint8)
    assert q.dtype == torch.uint8
    q = q.cpu().numpy()
    assert np.array_equal(q, self_code(f32))
    ref = oracle.fuse(wavelet, pan.astype(np.float64), ms.astype(np.float64))
    check_u8(oracle, q, ref, exact=(wavelet == "haar"))
    if wavelet == "haar":
        assert np.array_equal(f32, ref.astype(np.float32))
    else:
        assert np.abs(f32 - ref).max() <= D4_TOL


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W,B", [(66, 1030, 3), (130, 1288, 4), (8, 8, 1)])
def test_f32_input_u8_output(dev, fz, oracle, wavelet, H, W, B):
    rng = np.random.default_rng(H + W)
    pan, ms = int_scene(rng, H, W, B)
    gain = rng.uniform(0.5, 1.5, B).astype(np.float32)
    p, m, g = to_dev(pan, dev), to_dev(ms, dev), to_dev(gain, dev)
    say("f32 in u8 out", wavelet, H, W, B)
    f32 = fz.fuse(p, m, wavelet, g).cpu().numpy()
    q = fz.fuse(p, m, wavelet, g, out_dtype=torch.uint8).cpu().numpy()
    assert np.array_equal(q, self_code(f32))
    ref = oracle.fuse(wavelet, pan.astype(np.float64), ms.astype(np.float64), gain.astype(np.float64))
    check_u8(oracle, q, ref, exact=False)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("kappa", [2.0, 0.5, 1.7])
@pytest.mark.parametrize("H,W,B", [(34, 70, 3), (130, 1288, 2), (66, 516, 5)])
def test_kappa(dev, fz, oracle, wavelet, kappa, H, W, B):
    rng = np.random.default_rng(int(kappa * 10) + H)
    pan, ms = int_scene(rng, H, W, B)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    say("kappa", wavelet, kappa, H, W, B)
    got = fz.fuse(p, m, wavelet, kappa=kappa).cpu().numpy()
    ref = oracle.fuse(wavelet, pan.astype(np.float64), ms.astype(np.float64), kappa=kappa)
    if wavelet == "haar" and kappa in (2.0, 0.5):
        assert np.array_equal(got, ref.astype(np.float32))
    else:
        assert np.abs(got - ref).max() <= D4_TOL
    if kappa == 0.5:  # exact scaling: same as the float path on pre-scaled MS
        base = fz.fuse(p, m * 0.5, wavelet).cpu().numpy()
        assert np.array_equal(got, base)
    say("kappa u8", wavelet, kappa, H, W, B)
    q = fz.fuse(p.to(torch.uint8), m.to(torch.uint8), wavelet, out_dtype=torch.uint8, kappa=kappa).cpu().numpy()
    check_u8(oracle, q, ref, exact=(wavelet == "haar" and kappa in (2.0, 0.5)))


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("H,W", [(250, 1034), (250, 4104), (18, 8)])
def test_forced_shapes_identical(dev, fz, wavelet, H, W):
    """Every shape of the format kernels (one-shot tiles of 1 or 2 rows,
    rolling D4 units of any length (variant 1), LDS-staged D4 workgroups
    (variant 3), waves, columns) evaluates each pixel with the same
    operations, so all agree bit for bit."""
    rng = np.random.default_rng(9)
    pan, ms = u8_scene(rng, H, W, 3)
    p, m = to_dev(pan, dev), to_dev(ms, dev)
    ctx = fz.context(dev)
    outs = []
    try:
        for seg, wpb, nc, var in [(0, 0, 0, 0), (1, 1, 1, 0), (2, 4, 1, 0), (1, 2, 2, 0), (2, 1, 2, 0), (2, 4, 2, 0),
                                  (1, 4, 2, 0), (3, 2, 1, 1), (16, 4, 2, 1), (64, 1, 1, 1), (1, 4, 2, 1),
                                  (1, 4, 0, 3), (2, 4, 0, 3), (2, 2, 0, 3), (1, 1, 0, 3), (2, 1, 0, 3)]:
            say("codec shape", wavelet, H, W, seg, wpb, nc, var)
            ctx.force_tile(seg, wpb, nc, var)
            outs.append((fz.fuse(p, m, wavelet).cpu().numpy(),
                         fz.fuse(p, m, wavelet, out_dtype=torch.uint8).cpu().numpy()))
    finally:
        ctx.force_tile(0, 0, 0, 0)
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])


def strided_u8(a, dev, pad, offset):
    rows = int(np.prod(a.shape[:-1]))
    cols = a.shape[-1]
    pitch = cols + pad
    base = torch.full((offset + rows * pitch + 16,), 77, dtype=torch.uint8, device=dev)
    v = base[offset:offset + rows * pitch].view(rows, pitch)[:, :cols]
    v.copy_(torch.from_numpy(np.ascontiguousarray(a).reshape(rows, cols)).to(dev))
    return v.view(*a.shape) if a.ndim == 2 else v.unflatten(0, a.shape[:-1])


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
@pytest.mark.parametrize("pad,offset", [(16, 0), (1, 0), (0, 3), (5, 7)])
def test_pitches_and_offsets(dev, fz, wavelet, pad, offset):
    """Odd pitches and byte offsets take the scalar path; same results."""
    rng = np.random.default_rng(pad * 10 + offset)
    H, W, B = 34, 1030, 3
    pan, ms = u8_scene(rng, H, W, B)
    ref = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet, out_dtype=torch.uint8).cpu().numpy()
    reff = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), wavelet).cpu().numpy()
    say("codec pitches", wavelet, pad, offset)
    p, m = strided_u8(pan, dev, pad, offset), strided_u8(ms, dev, pad, offset)
    out = strided_u8(np.zeros((B, H, W), np.uint8), dev, pad, offset)
    fz.fuse(p, m, wavelet, out=out)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(fz.fuse(p, m, wavelet).cpu().numpy(), reff)


@pytest.mark.parametrize("pad,offset", [(16, 0), (1, 0), (0, 3), (5, 7), (2, 2)])
@pytest.mark.parametrize("B", [1, 3, 9])
def test_staged_u8_pitches_offsets_bands(dev, fz, pad, offset, B):
    """LDS-staged 8-bit D4 workgroups on pitched and offset views (rows not
    4-byte aligned take byte loads and stores) and with more bands than one
    LDS band group holds: identical to the contiguous call."""
    rng = np.random.default_rng(pad * 7 + offset + B)
    H, W = 66, 1290
    pan, ms = u8_scene(rng, H, W, B)
    ref = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "d4", out_dtype=torch.uint8).cpu().numpy()
    reff = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "d4").cpu().numpy()
    p, m = strided_u8(pan, dev, pad, offset), strided_u8(ms, dev, pad, offset)
    out = strided_u8(np.zeros((B, H, W), np.uint8), dev, pad, offset)
    ctx = fz.context(dev)
    try:
        for seg, wpb in ((2, 4), (1, 2)):
            say("codec staged pitches", pad, offset, B, seg, wpb)
            ctx.force_tile(seg, wpb, 0, 3)
            fz.fuse(p, m, "d4", out=out)
            assert np.array_equal(out.cpu().numpy(), ref)
            assert np.array_equal(fz.fuse(p, m, "d4").cpu().numpy(), reff)
    finally:
        ctx.force_tile(0, 0, 0, 0)


def test_nan_gain_gives_zero_code(dev, fz):
    rng = np.random.default_rng(4)
    pan, ms = u8_scene(rng, 18, 40, 2)
    g = torch.tensor([float("nan"), 1.0], device=dev)
    say("codec nan gain")
    q = fz.fuse(to_dev(pan, dev), to_dev(ms, dev), "d4", g, out_dtype=torch.uint8).cpu().numpy()
    assert (q[0] == 0).all()
    assert q[1].any()


def test_bad_dtypes(dev, fz):
    p = torch.zeros((8, 8), dtype=torch.uint8, device=dev)
    m = torch.zeros((1, 4, 4), dtype=torch.float32, device=dev)
    with pytest.raises(TypeError):
        fz.fuse(p, m, "d4")
    with pytest.raises(TypeError):
        fz.fuse(p, m.to(torch.uint8), "d4", out_dtype=torch.float16)


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_full_size_landsat_u8(dev, fz, oracle, wavelet):
    """15872 x 14336, 6 bands, 8-bit in and out, in the launch configuration
    the benchmark times (tuner on); sampled pixels against the single-pixel
    oracle."""
    from paper_1803_00737_amd import synth
    from test_gpu_parity import sample_points

    wl = synth.landsat(wavelet)
    say("full size u8", wl.name, "generate")
    pan_d, ms_d = wl.make(device=dev)
    p8, m8 = pan_d.to(torch.uint8), ms_d.to(torch.uint8)
    assert torch.equal(p8.float(), pan_d) and torch.equal(m8.float(), ms_d)
    del pan_d, ms_d
    ctx = fz.context(dev)
    ctx.set_tuning(True)
    try:
        say("full size u8", wl.name, "fuse (tuned)")
        q = fz.fuse(p8, m8, wavelet, out_dtype=torch.uint8)
    finally:
        ctx.set_tuning(False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    pts = sample_points(wl.H, wl.W, wl.B, 16, 400, rng)
    b, y, x = map(np.array, zip(*pts))
    idx = [torch.from_numpy(v).to(dev) for v in (b, y, x)]
    got = q[idx[0], idx[1], idx[2]].cpu().numpy()
    pan = p8.cpu().numpy().astype(np.float64)
    ms = m8.cpu().numpy().astype(np.float64)
    del q, p8, m8
    torch.cuda.empty_cache()
    ref = oracle.fuse_points(wavelet, pan, ms, None, b, y, x)
    check_u8(oracle, got, ref, exact=(wavelet == "haar"))


@pytest.mark.parametrize("wavelet", ["haar", "d4"])
def test_u8_beyond_2_31_bytes(dev, fz, oracle, wavelet):
    """8-bit in and out, 8192 x 8192 with 33 bands: the output holds 2.2e9
    bytes, more than a 32-bit index can address, so every band offset of the
    8-bit kernels must be formed in 64-bit arithmetic.  Sampled pixels of the
    first and last bands against the single-pixel oracle, in the tuned launch
    shape."""
    H = W = 8192
    B = 33
    rng = np.random.default_rng(34)
    say("u8 beyond 2^31", wavelet, "generate")
    p8 = torch.randint(0, 256, (H, W), device=dev, dtype=torch.uint8)
    ms1 = torch.randint(0, 256, (1, H // 2, W // 2), device=dev, dtype=torch.uint8)
    m8 = ms1.expand(B, H // 2, W // 2).contiguous()
    m8[B - 1] = torch.flip(ms1[0], dims=[1])  # a last band that differs from the others
    ctx = fz.context(dev)
    ctx.set_tuning(True)
    try:
        say("u8 beyond 2^31", wavelet, "fuse")
        q = fz.fuse(p8, m8, wavelet, out_dtype=torch.uint8)
    finally:
        ctx.set_tuning(False)
    torch.cuda.synchronize()
    assert q.numel() > 2 ** 31
    pts = [(b, int(y), int(x)) for b in (0, 1, B - 2, B - 1) for y, x in
           zip(rng.integers(0, H, 24), rng.integers(0, W, 24))] + [(B - 1, H - 1, W - 1), (B - 1, 0, 0)]
    b, y, x = map(np.array, zip(*pts))
    got = q[torch.from_numpy(b).to(dev), torch.from_numpy(y).to(dev), torch.from_numpy(x).to(dev)].cpu().numpy()
    pan = p8.cpu().numpy().astype(np.float64)
    ms_small = np.stack([m8[k].cpu().numpy() for k in (0, B - 1)]).astype(np.float64)
    del q, m8, p8
    torch.cuda.empty_cache()
    bi = np.where(b == B - 1, 1, 0)
    ref = oracle.fuse_points(wavelet, pan, ms_small, None, bi, y, x)
    check_u8(oracle, got, ref, exact=(wavelet == "haar"))
