"""GPU (gfx950) library vs the CPU oracle, through the C ABI.

Bar: the blob (header, code lengths, tile/chunk tables, exception list,
bitstream) and the decompressed field are bit-exact; the float64 Eq. 4
statistics agree to 1e-9 relative.  Every case prints its name first so a
failing run names it.
"""
import numpy as np
import pytest

from paper_1805_07384_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_07384_amd import fpsz
    return fpsz.Context(0)


def _bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def _gpu_compress(ctx, x: np.ndarray, psnr: float, domain: int):
    from paper_1805_07384_amd import fpsz
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ws = torch.empty(fpsz.compress_workspace_bytes(x.shape, xt.dtype), dtype=torch.uint8,
                     device="cuda")
    ws.fill_(0xA5)  # garbage: the library must not rely on a clean workspace
    cap = fpsz.compress_bound(x.shape, xt.dtype)
    blob = torch.full((cap,), 0x5A, dtype=torch.uint8, device="cuda")
    st, nb, info = ctx.compress_into(xt, psnr, ws, blob, domain)
    torch.cuda.synchronize()
    return st, blob[:nb], info.as_dict(), ws, xt


def _diagnose(ctx, orc, x, psnr, domain, ws, gblob: bytes, oblob: bytes):
    """Localise a blob mismatch through the workspace intermediates."""
    from paper_1805_07384_amd import fpsz
    _, t = orc.compress(x, psnr, domain=domain, trace=True)
    msgs = []
    hg, ho = orc.header(gblob) if len(gblob) >= 256 else {}, orc.header(oblob)
    for k in ho:
        if hg.get(k) != ho[k]:
            msgs.append("header %s: gpu %r oracle %r" % (k, hg.get(k), ho[k]))
    wsn = ws.cpu().numpy()
    o = fpsz.workspace_offset(x.shape, torch.float32 if x.dtype == np.float32 else torch.float64, 1)
    hist = wsn[o:o + 4 * 1036].view(np.uint32)
    if not np.array_equal(hist, t["hist"]):
        d = np.nonzero(hist != t["hist"])[0]
        msgs.append("histogram differs at %d bins, first %s" % (len(d), d[:5]))
    o = fpsz.workspace_offset(x.shape, torch.float32 if x.dtype == np.float32 else torch.float64, 2)
    ln = wsn[o:o + 1036]
    if not np.array_equal(ln, t["code_len"]):
        msgs.append("code lengths differ")
    o = fpsz.workspace_offset(x.shape, torch.float32 if x.dtype == np.float32 else torch.float64, 4)
    c16 = wsn[o:o + 2 * x.size].view(np.int16)
    if not np.array_equal(c16, t["code16"]):
        d = np.nonzero(c16 != t["code16"])[0]
        msgs.append("residual codes differ at %d positions, first %s gpu %s oracle %s"
                    % (len(d), d[:5], c16[d[:5]], t["code16"][d[:5]]))
    n = min(len(gblob), len(oblob))
    gb = np.frombuffer(gblob[:n], np.uint8)
    ob = np.frombuffer(oblob[:n], np.uint8)
    d = np.nonzero(gb != ob)[0]
    if len(d):
        msgs.append("first differing byte %d (of %d / %d)" % (d[0], len(gblob), len(oblob)))
    return "; ".join(msgs)


def _parity(ctx, orc, x, psnr, domain=0, check_stats=True):
    print("case shape=%s dtype=%s psnr=%s domain=%d" % (x.shape, x.dtype, psnr, domain), flush=True)
    ob, ot = orc.compress(x, psnr, domain=domain, trace=True)
    st, blob, info, ws, xt = _gpu_compress(ctx, x, psnr, domain)
    assert st == 0, "gpu compress status %d" % st
    gb = blob.cpu().numpy().tobytes()
    if gb != ob:
        pytest.fail("blob mismatch: " + _diagnose(ctx, orc, x, psnr, domain, ws, gb, ob))
    assert info["blob_bytes"] == len(ob)
    assert info["n_patches"] == ot["n_patches"] and info["n_outliers"] == ot["n_outliers"]
    assert info["eb"] == ot["eb"] and info["vr"] == ot["vr"]
    y = ctx.decompress(blob)
    oy = orc.decompress(ob)
    yn = y.cpu().numpy()
    assert yn.shape == x.shape
    assert np.array_equal(_bits(yn), _bits(oy)), "decompressed field differs"
    if check_stats:
        gs = ctx.verify(xt, y, info["vr"], info["eb"])
        os_ = orc.stats(x, oy, ot["vr"], ot["eb"])
        assert gs["n_over_eb"] == 0 == os_["n_over_eb"]
        assert gs["max_abs_err"] == os_["max_abs_err"]
        if os_["sse"] > 0:
            assert abs(gs["sse"] - os_["sse"]) <= 1e-9 * os_["sse"]
            assert abs(gs["psnr"] - os_["psnr"]) <= 1e-9 * abs(os_["psnr"])
    return info, y


SHAPES = [(20000,), (8192,), (8193,), (3, 5), (150, 300), (64, 128), (65, 129), (129, 257),
          (16, 16, 32), (17, 17, 33), (40, 37, 70), (1, 5, 8200), (2, 3, 4), (33, 17, 65)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_parity_shapes(ctx, orc, shape, dt):
    x = (synth.grf_numpy(shape, -3.0, 5) * 7.0 + 2.0).astype(dt)
    for domain in (0, 1):
        _parity(ctx, orc, x, 80.0, domain)


@pytest.mark.parametrize("psnr", [20.0, 40.0, 60.0, 100.0, 120.0])
def test_parity_psnr_sweep(ctx, orc, psnr):
    x = synth.field_3d_lognormal(shape=(48, 40, 70), seed=2)
    for domain in (0, 1):
        _parity(ctx, orc, x, psnr, domain)
        _parity(ctx, orc, x.astype(np.float64), psnr, domain)


def test_parity_outliers_and_patches(ctx, orc):
    x = synth.field_3d_spiky_f64(shape=(40, 64, 64), seed=5)
    info, _ = _parity(ctx, orc, x, 100.0, 0)
    assert info["n_outliers"] > 0
    info, _ = _parity(ctx, orc, x, 100.0, 1)
    xf = synth.field_2d_grf(300, 200, seed=3)
    info, _ = _parity(ctx, orc, xf, 120.0, 0)
    assert info["n_patches"] > 0
    # float64 at 150 dB: deep escape classes and many outliers (no patches:
    # the float64 patch path has its own case below)
    _parity(ctx, orc, xf.astype(np.float64) * 1.0001, 150.0, 0)


@pytest.mark.parametrize("case", ["outliers_f32", "patches_f64"])
def test_parity_tile_fused_exceptions(ctx, orc, case):
    # TILE-domain blobs whose tiles average at most ~2000 code words, on
    # fields of at least 2048 tiles (two workgroups of four tiles per CU),
    # are decoded and reconstructed in one launch; exception records in that
    # path, next to ragged tiles (z and y) and a last group of one tile
    # (19 x 17 x 7 = 2261 tiles).
    # outliers: a smooth field of tiny amplitude with sparse spikes of the
    # full range at 120 dB (spike residuals beyond 2^15 bins); patches:
    # float64 values within ulps of bin edges at 60 dB
    import patchfield as pf
    shape = (289, 257, 224)
    if case == "outliers_f32":
        rng = np.random.default_rng(21)
        x = synth.grf_numpy(shape, -3.0, 21) * 1e-5
        spikes = rng.random(shape) < 0.002
        x = np.where(spikes, rng.choice([-1.0, 1.0], size=shape), x).astype(np.float32)
        psnr = 120.0
    else:
        x = pf.f64_patch_field(shape=shape, psnr=60.0)
        psnr = 60.0
    h = orc.header(orc.compress(x, psnr, domain=1)[0])
    assert h["n_words"] / h["n_tiles"] <= 2048  # the one-launch path
    info, _ = _parity(ctx, orc, x, psnr, 1)
    if case == "outliers_f32":
        assert info["n_outliers"] > 0
    else:
        assert info["n_patches"] > 0


@pytest.mark.parametrize("shape", [(17, 33, 70), (33, 48, 96)])
def test_parity_f64_patches(ctx, orc, shape):
    # float64 values within three ulps of bin edges: two-record patches in a
    # full tile, in edge-clipped tiles, in a tile with more records than its
    # 64-record staging slot and beside outliers in one 32-point segment;
    # both Lorenzo domains, the separate and the fused check
    import patchfield as pf
    x = pf.f64_patch_field(shape=shape)
    _, ot = orc.compress(x, pf.PSNR, trace=True)
    assert ot["n_patches"] > 100 and ot["n_outliers"] > 0
    info, y = _parity(ctx, orc, x, pf.PSNR, 0)
    assert info["n_patches"] == ot["n_patches"]
    _parity(ctx, orc, x, pf.PSNR, 1)
    ob = orc.compress(x, pf.PSNR)[0]
    oy = orc.decompress(ob)
    blob = torch.from_numpy(np.frombuffer(ob, dtype=np.uint8).copy()).cuda()
    y2, st = ctx.decompress_verify(blob, torch.from_numpy(x).cuda())
    assert np.array_equal(_bits(y2.cpu().numpy()), _bits(oy))
    os_ = orc.stats(x, oy, ot["vr"], ot["eb"])
    assert st["n_over_eb"] == 0 and st["max_abs_err"] == os_["max_abs_err"]
    assert abs(st["sse"] - os_["sse"]) <= 1e-9 * os_["sse"]


def test_parity_config1_full_size(ctx, orc):
    # 2D float32 512 x 512, spectrum k^-3, range [-50, 50], 80 dB
    x = synth.field_2d_grf(512, 512, seed=1)
    info, _ = _parity(ctx, orc, x, 80.0, 0)
    assert abs(info["eb"] - 100 * orc.eb_rel(80.0)) < 1e-12


def _fibonacci_walk(n_sym=30, seed=4):
    """1D random walk whose Lorenzo residuals take n_sym values with
    Fibonacci counts, at the PSNR where 2 eb = 1: the unlimited Huffman tree
    is n_sym - 1 deep, so the 18-bit limit rebalances many levels."""
    fib = [1, 1]
    while len(fib) < n_sym:
        fib.append(fib[-1] + fib[-2])
    vals = [0]
    for k in range(1, n_sym):
        vals += [k, -k]
    steps = np.repeat(np.array(vals[:n_sym]), fib[::-1])
    np.random.default_rng(seed).shuffle(steps)
    s = np.cumsum(steps)
    r = float(s.max() - s.min())
    return s.astype(np.float32), float(-20 * np.log10((1 / (2 * r)) / np.sqrt(3)))


def test_parity_length_limit(ctx, orc):
    x, psnr = _fibonacci_walk()
    _, t = orc.compress(x, psnr, trace=True)
    h = t["hist"]
    assert orc.huffman_unlimited(h[h > 0]).max() >= 28 and t["code_len"].max() == 18
    _parity(ctx, orc, x, psnr, 0)
    # fewer symbols: a shallower overflow (only the last levels rebalanced)
    x, psnr = _fibonacci_walk(21, seed=5)
    _parity(ctx, orc, x, psnr, 1)


@pytest.fixture(scope="module")
def lognormal512():
    return synth.field_3d_lognormal(shape=(512, 512, 512), seed=2)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("domain", [1, 0])
@pytest.mark.parametrize("psnr", [40.0, 60.0, 80.0, 100.0, 120.0])
def test_parity_config2_full_size(ctx, orc, lognormal512, psnr, domain):
    # 3D float32 512^3 lognormal field, the benchmark workload at every
    # target of its sweep, in both Lorenzo domains: whole blob and whole
    # reconstruction compared (at 120 dB: escapes, outliers, tiles past their
    # staging slot, patches and chunks decoded from the global tail)
    info, _ = _parity(ctx, orc, lognormal512, psnr, domain)
    assert info["bits_per_value"] > 0
    if psnr == 120.0:
        assert info["n_outliers"] > 0 and info["n_patches"] > 0


@pytest.mark.timeout(400)
def test_parity_config5_slab(ctx, orc):
    # one GPU's share of the 1024^3 float64 field when it is split over 8
    # GPUs along z: a 128 x 1024 x 1024 slab of the same recipe (GRF k^-3
    # plus 1 % spikes of 1000 sigma) at 100 dB, blob and reconstruction
    # compared with the oracle
    x = synth.field_3d_spiky_f64(shape=(128, 1024, 1024), seed=5)
    info, _ = _parity(ctx, orc, x, 100.0, 0, check_stats=True)
    assert info["n_outliers"] > 0 or info["n_patches"] > 0


def _lorenzo3d_slab(q: "torch.Tensor", qprev: "torch.Tensor") -> "torch.Tensor":
    """3D Lorenzo residual (Eq. 1 with zeros outside the field) of the planes
    q, given the plane before them (zeros before the field)."""
    F = torch.nn.functional
    a = F.pad(torch.cat([qprev[None], q]), (1, 0, 1, 0))  # zero row / column in front
    return (a[1:, 1:, 1:] - a[:-1, 1:, 1:] - a[1:, :-1, 1:] - a[1:, 1:, :-1]
            + a[:-1, :-1, 1:] + a[:-1, 1:, :-1] + a[1:, :-1, :-1] - a[:-1, :-1, :-1])


def _lorenzo3d_tiles(q: "torch.Tensor") -> "torch.Tensor":
    """3D Lorenzo residual inside 16 x 16 x 32 tiles (TILE domain: zeros
    outside each tile) of planes q whose z, y and x extents are multiples of
    the tile's; returned tile-major, which does not matter for counts."""
    F = torch.nn.functional
    Z, Y, X = q.shape
    t = q.reshape(Z // 16, 16, Y // 16, 16, X // 32, 32).permute(0, 2, 4, 1, 3, 5)
    a = F.pad(t, (1, 0, 1, 0, 1, 0))
    return (a[..., 1:, 1:, 1:] - a[..., :-1, 1:, 1:] - a[..., 1:, :-1, 1:] - a[..., 1:, 1:, :-1]
            + a[..., :-1, :-1, 1:] + a[..., :-1, 1:, :-1] + a[..., 1:, :-1, :-1]
            - a[..., :-1, :-1, :-1])


@pytest.mark.timeout(400)
@pytest.mark.parametrize("domain", [0, 1])
def test_config5_full_size_f64(ctx, orc, domain):
    # 3D float64 1024^3 GRF k^-3 with 1 % spikes of 1000 sigma at 100 dB,
    # device-resident compress and fused decompress + Eq. 4 check at full
    # size, in both Lorenzo domains (TILE takes the one-launch decompression).  The whole-field oracle would take too long here, so the result is
    # held to what the method fixes at every point: vr and eb (Eq. 7),
    # x' = 2eb * rint(x / 2eb) unless |x - x'| > eb, where x' = x (a patch),
    # the outlier count (|Lorenzo residual| >= 2^15, residuals from a plain
    # torch stencil), the statistics, and the blob checksum by the oracle.
    from paper_1805_07384_amd import fpsz
    psnr, shape = 100.0, (1024, 1024, 1024)
    print("case config5 shape=%s float64 psnr=%s domain=%d" % (shape, psnr, domain), flush=True)
    x = synth.field_3d_spiky_f64(shape=shape, seed=5, backend="torch", device="cuda").contiguous()
    torch.cuda.synchronize()
    ws = torch.empty(fpsz.compress_workspace_bytes(shape, x.dtype), dtype=torch.uint8, device="cuda")
    cap = x.numel() * 8 + x.numel() // 8 + (1 << 20)  # the raw size and then some
    blob = torch.empty(cap, dtype=torch.uint8, device="cuda")
    print("compress", flush=True)
    st, nb, info = ctx.compress_into(x, psnr, ws, blob, domain)
    assert st == 0, "gpu compress status %d" % st
    info = info.as_dict()
    # the code lengths in the blob are the oracle's Huffman lengths of the
    # device histogram
    o = fpsz.workspace_offset(shape, x.dtype, 1)
    hist = ws[o:o + 4 * 1036].cpu().numpy().view(np.uint32)
    assert int(hist.sum()) == x.numel()
    lens = blob[256:256 + 1036].cpu().numpy()
    assert np.array_equal(lens, orc.code_lengths(hist))
    del ws
    vr = float(x.max().item()) - float(x.min().item())
    assert info["vr"] == vr
    assert info["eb"] == vr * orc.eb_rel(psnr)
    eb = info["eb"]
    e2, r = 2.0 * eb, 1.0 / (2.0 * eb)
    print("decompress + check", flush=True)
    out = torch.empty_like(x)
    wsd = torch.empty(fpsz.decompress_workspace_bytes(shape, x.dtype), dtype=torch.uint8,
                      device="cuda")
    st, stats = ctx.decompress_verify_into(blob, nb, wsd, out, x)
    assert st == 0, "gpu decompress status %d" % st
    stats = stats.as_dict()
    del wsd
    print("point-wise checks", flush=True)
    n_out = n_pat = 0
    sse = 0.0
    mx = 0.0
    qprev = torch.zeros(shape[1:], dtype=torch.int64, device="cuda")
    for z0 in range(0, shape[0], 64):
        xs = x[z0:z0 + 64]
        q = torch.round(xs * r).to(torch.int64)  # round half to even, as rint
        xq = q.to(torch.float64) * e2
        patch = (xs - xq).abs() > eb
        want = torch.where(patch, xs, xq)
        ys = out[z0:z0 + 64]
        assert torch.equal(ys.view(torch.int64), want.view(torch.int64)), "planes %d.." % z0
        n_pat += int(patch.sum().item())
        res = _lorenzo3d_slab(q, qprev) if domain == 0 else _lorenzo3d_tiles(q)
        n_out += int((res.abs() >= 32768).sum().item())
        del res
        d = xs - ys
        sse += float((d * d).sum().item())
        mx = max(mx, float(d.abs().max().item()))
        qprev = q[-1]
    assert info["n_patches"] == n_pat and info["n_outliers"] == n_out
    assert stats["n_over_eb"] == 0 and stats["max_abs_err"] == mx <= eb
    assert abs(stats["sse"] - sse) <= 1e-9 * sse
    psnr_t = -20.0 * np.log10(np.sqrt(sse / x.numel()) / vr)
    assert abs(stats["psnr"] - psnr_t) <= 1e-9 * abs(psnr_t)
    print("blob checksum", flush=True)
    b = blob[:nb].cpu().numpy().tobytes()
    h = orc.header(b)
    assert h["n"] == x.numel() and h["bytes"] == nb
    assert h["n_outliers"] == n_out and h["n_patches"] == n_pat
    assert h["checksum"] == orc.checksum(b[:200] + b"\0" * 8 + b[208:])


def test_constant_and_tiny(ctx, orc):
    from paper_1805_07384_amd import fpsz
    for shape in [(1,), (7,), (3, 3), (2, 2, 2)]:
        x = np.full(shape, 3.25, dtype=np.float32)
        print("case const", shape, flush=True)
        ob, _ = orc.compress(x, 80.0)
        st, blob, info, ws, xt = _gpu_compress(ctx, x, 80.0, 0)
        assert st == 0 and info["is_const"] == 1
        assert blob.cpu().numpy().tobytes() == ob
        y = ctx.decompress(blob)
        assert np.array_equal(y.cpu().numpy(), x)
    _parity(ctx, orc, np.array([1.0, 2.0], dtype=np.float32), 60.0, 0)
    _parity(ctx, orc, np.array([[0.0], [-1.0]], dtype=np.float64), 60.0, 0)


def test_error_statuses(ctx):
    from paper_1805_07384_amd import fpsz
    print("case errors", flush=True)
    x = np.linspace(0, 1, 5000, dtype=np.float32)
    x[1234] = np.nan
    st, *_ = _gpu_compress(ctx, x, 80.0, 0)
    assert st == fpsz.E_NONFINITE
    x[1234] = np.inf
    st, *_ = _gpu_compress(ctx, x, 80.0, 0)
    assert st == fpsz.E_NONFINITE
    st, *_ = _gpu_compress(ctx, np.linspace(0, 1, 5000, dtype=np.float32), 200.0, 0)
    assert st == fpsz.E_RANGE
    # capacity: the exact size is reported
    xs = synth.field_2d_grf(100, 100, seed=8)
    xt = torch.from_numpy(xs).cuda()
    ws = torch.empty(fpsz.compress_workspace_bytes(xs.shape), dtype=torch.uint8, device="cuda")
    big = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st, need, _ = ctx.compress_into(xt, 80.0, ws, big, 0)
    assert st == 0
    small = torch.empty(need - 8, dtype=torch.uint8, device="cuda")
    st, need2, _ = ctx.compress_into(xt, 80.0, ws, small, 0)
    assert st == fpsz.E_CAPACITY and need2 == need


def test_corrupt_blob_detected(ctx, orc):
    from paper_1805_07384_amd import fpsz
    print("case corrupt", flush=True)
    x = synth.field_2d_grf(200, 300, seed=4)
    blob, info = ctx.compress(torch.from_numpy(x).cuda(), 60.0)
    good = blob.cpu().numpy()
    rng = np.random.default_rng(7)
    for _ in range(16):
        bad = good.copy()
        i = int(rng.integers(256, len(bad)))
        bad[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        with pytest.raises(fpsz.FpszError) as e:
            ctx.decompress(torch.from_numpy(bad).cuda())
        assert e.value.status == fpsz.E_CORRUPT
    with pytest.raises(fpsz.FpszError):
        ctx.decompress(torch.from_numpy(good[:-8].copy()).cuda())


def test_deterministic_repeat(ctx):
    print("case determinism", flush=True)
    x = torch.from_numpy(synth.field_3d_lognormal(shape=(64, 64, 64), seed=3)).cuda()
    a, _ = ctx.compress(x, 100.0)
    for _ in range(3):
        b, _ = ctx.compress(x, 100.0)
        assert torch.equal(a, b)


FUSED_CASES = [((20000,), np.float32, 0), ((8193,), np.float64, 1), ((150, 300), np.float32, 0),
               ((65, 129), np.float64, 0), ((40, 37, 70), np.float32, 0),
               ((33, 17, 65), np.float64, 1), ((64, 64, 64), np.float32, 1),
               ((16, 16, 32), np.float32, 0)]


@pytest.mark.parametrize("shape,dt,domain", FUSED_CASES)
def test_decompress_verify_fused(ctx, orc, shape, dt, domain):
    # one pass that decompresses and takes the Eq. 4 statistics: the field is
    # the oracle's bit for bit, the statistics the oracle's (max |e| and the
    # count over eb exactly, the float64 SSE to rounding), repeated calls
    # identical, and the separate verify agrees
    from paper_1805_07384_amd import fpsz
    x = (synth.grf_numpy(shape, -3.0, 11) * 3.0 + 0.5).astype(dt)
    print("case fused shape=%s dtype=%s domain=%d" % (shape, x.dtype, domain), flush=True)
    ob, ot = orc.compress(x, 90.0, domain=domain, trace=True)
    oy = orc.decompress(ob)
    os_ = orc.stats(x, oy, ot["vr"], ot["eb"])
    blob = torch.from_numpy(np.frombuffer(ob, dtype=np.uint8).copy()).cuda()
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y, st1 = ctx.decompress_verify(blob, xt)
    _, st2 = ctx.decompress_verify(blob, xt)
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(oy))
    assert st1 == st2
    assert st1["n_over_eb"] == os_["n_over_eb"] == 0
    assert st1["max_abs_err"] == os_["max_abs_err"]
    assert abs(st1["sse"] - os_["sse"]) <= 1e-9 * os_["sse"]
    assert abs(st1["psnr"] - os_["psnr"]) <= 1e-9 * abs(os_["psnr"])
    sv = ctx.verify(xt, y, ot["vr"], ot["eb"])
    assert sv["max_abs_err"] == st1["max_abs_err"] and sv["n_over_eb"] == st1["n_over_eb"]
    assert abs(sv["sse"] - st1["sse"]) <= 1e-12 * sv["sse"]


def test_decompress_verify_constant_and_small_workspace(ctx, orc):
    from paper_1805_07384_amd import fpsz
    print("case fused constant", flush=True)
    x = np.full((7, 9), 2.5, dtype=np.float32)
    ob, _ = orc.compress(x, 80.0)
    blob = torch.from_numpy(np.frombuffer(ob, dtype=np.uint8).copy()).cuda()
    xt = torch.from_numpy(x).cuda()
    y, st = ctx.decompress_verify(blob, xt)
    assert np.array_equal(y.cpu().numpy(), x)
    assert st["sse"] == 0.0 and st["max_abs_err"] == 0.0 and st["n_over_eb"] == 0
    # a workspace too small for the check is refused, nothing is written
    x2 = synth.grf_numpy((50, 60), -3.0, 3).astype(np.float32)
    ob2, _ = orc.compress(x2, 80.0)
    blob2 = torch.from_numpy(np.frombuffer(ob2, dtype=np.uint8).copy()).cuda()
    out = torch.empty((50, 60), dtype=torch.float32, device="cuda")
    need = fpsz.decompress_workspace_bytes((50, 60), torch.float32)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    stt, _ = ctx.decompress_verify_into(blob2, blob2.numel(), small, out,
                                        torch.from_numpy(x2).cuda())
    assert stt == fpsz.E_CAPACITY


CLOSED_CASES = [((48, 40, 70), np.float32, 40.0, 0), ((48, 40, 70), np.float32, 60.0, 1),
                ((300, 200), np.float64, 40.0, 0), ((20000,), np.float32, 30.0, 0),
                ((64, 64, 64), np.float32, 100.0, 0)]


@pytest.mark.parametrize("shape,dt,psnr,domain", CLOSED_CASES)
def test_parity_closed_loop(ctx, orc, shape, dt, psnr, domain):
    # closed-loop compression: the factor is a float64 reduction, held to the
    # oracle's within 1e-9 relative; given the device's factor, the blob is
    # the oracle's scaled compression byte for byte, and decompression the
    # oracle's bit for bit
    from paper_1805_07384_amd import fpsz
    x = (synth.field_3d_lognormal(shape=shape, seed=2) if len(shape) == 3
         else synth.grf_numpy(shape, -3.0, 8) * 4.0 + 1.0).astype(dt)
    print("case closed shape=%s dtype=%s psnr=%s domain=%d" % (shape, x.dtype, psnr, domain),
          flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ws = torch.full((fpsz.compress_workspace_bytes(x.shape, xt.dtype),), 0xA5, dtype=torch.uint8,
                    device="cuda")
    blob = torch.full((fpsz.compress_bound(x.shape, xt.dtype),), 0x5A, dtype=torch.uint8,
                      device="cuda")
    st, nb, info = ctx.compress_closed_loop_into(xt, psnr, ws, blob, domain)
    assert st == 0
    s_gpu = info.eb_scale
    _, _, s_or = orc.compress_closed_loop(x, psnr, domain)
    assert abs(s_gpu - s_or) <= 1e-9 * s_or
    ob, ot = orc.compress_scaled(x, psnr, s_gpu, domain, trace=True)
    gb = blob[:nb].cpu().numpy().tobytes()
    assert gb == ob, "closed-loop blob differs from the oracle's at the device factor"
    assert info.eb == ot["eb"] and info.eb_rel == orc.eb_rel(psnr) * s_gpu
    y = ctx.decompress(blob[:nb])
    oy = orc.decompress(ob)
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(oy))
    # closer to the target than plain compression
    st_c = orc.stats(x, oy, ot["vr"], ot["eb"])
    b0, t0 = orc.compress(x, psnr, domain, trace=True)
    st_p = orc.stats(x, orc.decompress(b0), t0["vr"], t0["eb"])
    assert st_c["n_over_eb"] == 0
    if abs(st_p["psnr"] - psnr) > 0.01:
        assert abs(st_c["psnr"] - psnr) < abs(st_p["psnr"] - psnr)


INLOOP_CASES = [((20000,), np.float32, 80.0), ((8193,), np.float64, 120.0),
                ((150, 300), np.float32, 30.0), ((65, 129), np.float64, 100.0),
                ((40, 37, 70), np.float32, 120.0), ((16, 16, 32), np.float32, 60.0),
                ((33, 17, 65), np.float64, 80.0), ((64, 64, 64), np.float32, 100.0)]


@pytest.mark.parametrize("shape,dt,psnr", INLOOP_CASES)
def test_parity_inloop(ctx, orc, shape, dt, psnr):
    # the SZ 1.4-style in-loop variant: blob and reconstruction bit-exact
    # with the oracle's sequential loop; the fused check agrees
    from paper_1805_07384_amd import fpsz
    x = (synth.grf_numpy(shape, -3.0, 13) * 3.0 + 1.0).astype(dt)
    print("case inloop shape=%s dtype=%s psnr=%s" % (shape, x.dtype, psnr), flush=True)
    ob, ot = orc.compress_inloop(x, psnr, trace=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ws = torch.full((fpsz.compress_workspace_bytes(x.shape, xt.dtype),), 0xA5, dtype=torch.uint8,
                    device="cuda")
    blob = torch.full((fpsz.compress_bound(x.shape, xt.dtype),), 0x5A, dtype=torch.uint8,
                      device="cuda")
    st, nb, info = ctx.compress_inloop_into(xt, psnr, ws, blob)
    assert st == 0
    gb = blob[:nb].cpu().numpy().tobytes()
    if gb != ob:
        o = fpsz.workspace_offset(x.shape, xt.dtype, 4)
        c16 = ws[o:o + 2 * x.size].cpu().numpy().view(np.int16)
        d = np.nonzero(c16 != ot["code16"])[0]
        pytest.fail("in-loop blob differs: %d of %d codes differ, first %s gpu %s oracle %s"
                    % (len(d), x.size, d[:5], c16[d[:5]], ot["code16"][d[:5]]))
    assert info.variant == 1 and info.n_patches == ot["n_patches"] and info.n_outliers == 0
    y = ctx.decompress(blob[:nb])
    oy = orc.decompress(ob)
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(oy))
    y2, stv = ctx.decompress_verify(blob[:nb], xt)
    assert np.array_equal(_bits(y2.cpu().numpy()), _bits(oy))
    os_ = orc.stats(x, oy, ot["vr"], ot["eb"])
    assert stv["n_over_eb"] == 0 == os_["n_over_eb"]
    assert stv["max_abs_err"] == os_["max_abs_err"]
    assert abs(stv["sse"] - os_["sse"]) <= 1e-9 * os_["sse"]


def test_parity_inloop_stored_points(ctx, orc):
    # the float64 bin-edge field: many points whose reconstruction misses
    # the bound in floating point are stored exactly (two records each)
    import patchfield as pf
    from paper_1805_07384_amd import fpsz
    x = pf.f64_patch_field()
    print("case inloop stored points", flush=True)
    ob, ot = orc.compress_inloop(x, pf.PSNR, trace=True)
    assert ot["n_patches"] > 0
    xt = torch.from_numpy(x).cuda()
    ws = torch.empty(fpsz.compress_workspace_bytes(x.shape, xt.dtype), dtype=torch.uint8,
                     device="cuda")
    blob = torch.empty(fpsz.compress_bound(x.shape, xt.dtype), dtype=torch.uint8, device="cuda")
    st, nb, info = ctx.compress_inloop_into(xt, pf.PSNR, ws, blob)
    assert st == 0 and blob[:nb].cpu().numpy().tobytes() == ob
    y = ctx.decompress(blob[:nb])
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(orc.decompress(ob)))


XFORM_CASES = [((4096,), np.float32, 80.0), ((8196,), np.float64, 120.0),
               ((68, 132), np.float32, 40.0), ((68, 132), np.float64, 100.0),
               ((20, 36, 68), np.float32, 120.0), ((20, 36, 68), np.float64, 60.0),
               ((64, 64, 64), np.float32, 80.0)]


def _xform_run(ctx, x, psnr):
    from paper_1805_07384_amd import fpsz
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ws = torch.full((fpsz.compress_workspace_bytes(x.shape, xt.dtype),), 0xA5, dtype=torch.uint8,
                    device="cuda")
    blob = torch.full((fpsz.compress_bound(x.shape, xt.dtype),), 0x5A, dtype=torch.uint8,
                      device="cuda")
    st, nb, info = ctx.compress_xform_into(xt, psnr, ws, blob)
    return xt, ws, blob, st, nb, info


@pytest.mark.parametrize("shape,dt,psnr", XFORM_CASES)
def test_parity_xform(ctx, orc, shape, dt, psnr):
    # the orthogonal-transform variant: blob and reconstruction bit-exact
    # with the oracle; the fused check agrees with the oracle's statistics
    from paper_1805_07384_amd import fpsz
    x = (synth.grf_numpy(shape, -3.0, 21) * 4.0 - 2.0).astype(dt)
    print("case xform shape=%s dtype=%s psnr=%s" % (shape, x.dtype, psnr), flush=True)
    ob, ot = orc.compress_xform(x, psnr, trace=True)
    xt, ws, blob, st, nb, info = _xform_run(ctx, x, psnr)
    assert st == 0
    gb = blob[:nb].cpu().numpy().tobytes()
    if gb != ob:
        o = fpsz.workspace_offset(x.shape, xt.dtype, 4)
        c16 = ws[o:o + 2 * x.size].cpu().numpy().view(np.int16)
        d = np.nonzero(c16 != ot["code16"])[0]
        pytest.fail("transform blob differs: %d of %d codes differ, first %s gpu %s oracle %s"
                    % (len(d), x.size, d[:5], c16[d[:5]], ot["code16"][d[:5]]))
    assert info.variant == 2 and info.n_patches == 0
    assert info.n_outliers == ot["n_outliers"]
    y = ctx.decompress(blob[:nb])
    oy = orc.decompress(ob)
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(oy))
    y2, stv = ctx.decompress_verify(blob[:nb], xt)
    assert np.array_equal(_bits(y2.cpu().numpy()), _bits(oy))
    os_ = orc.stats(x, oy, ot["vr"], ot["eb"])
    assert stv["n_over_eb"] == os_["n_over_eb"]
    assert stv["max_abs_err"] == os_["max_abs_err"]
    assert abs(stv["sse"] - os_["sse"]) <= 1e-9 * os_["sse"]


def test_parity_xform_outliers_and_constant(ctx, orc):
    # white noise at 120 dB: coefficient bins beyond 2^15 are stored as
    # outlier records; a constant field gives the constant blob
    rng = np.random.default_rng(5)
    x = rng.uniform(-1.0, 1.0, size=(36, 40, 44)).astype(np.float64)
    print("case xform outliers", flush=True)
    ob, ot = orc.compress_xform(x, 120.0, trace=True)
    assert ot["n_outliers"] > 0
    xt, ws, blob, st, nb, info = _xform_run(ctx, x, 120.0)
    assert st == 0 and info.n_outliers == ot["n_outliers"]
    assert blob[:nb].cpu().numpy().tobytes() == ob
    y = ctx.decompress(blob[:nb])
    assert np.array_equal(_bits(y.cpu().numpy()), _bits(orc.decompress(ob)))
    c = np.full((8, 12), 3.25, dtype=np.float32)
    print("case xform constant", flush=True)
    ob, _ = orc.compress_xform(c, 80.0, trace=True)
    xt, ws, blob, st, nb, info = _xform_run(ctx, c, 80.0)
    assert st == 0 and blob[:nb].cpu().numpy().tobytes() == ob
    assert np.array_equal(ctx.decompress(blob[:nb]).cpu().numpy(), c)
    xt, ws, blob, st, nb, info = _xform_run(ctx, np.zeros((10, 12), np.float32), 80.0)
    assert st != 0
