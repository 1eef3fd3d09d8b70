"""fpsz_compress_async and fpsz_decompress_async (the entry points that write
their outcome to device memory and never synchronize) against the
synchronous calls: identical blobs, reconstructions and reports when called
directly and when captured in a graph and replayed (each replay checked,
with eager work and synchronizations between replays), and device-side
statuses (non-finite input, capacity, a header that does not match the
blob)."""
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


def _plain(ctx, xt, psnr, domain):
    from paper_1805_07384_amd import fpsz
    ws = torch.empty(fpsz.compress_workspace_bytes(xt.shape, xt.dtype), dtype=torch.uint8,
                     device="cuda")
    blob = torch.empty(fpsz.compress_bound(xt.shape, xt.dtype), dtype=torch.uint8, device="cuda")
    st, nb, info = ctx.compress_into(xt, psnr, ws, blob, domain)
    assert st == 0
    return blob[:nb].clone(), info


def _check(res, blob, pblob, pinfo):
    assert res.status == 0
    assert res.blob_bytes == pinfo.blob_bytes == pblob.numel()
    assert res.n_outliers == pinfo.n_outliers and res.n_patches == pinfo.n_patches
    assert res.vr == pinfo.vr and res.eb == pinfo.eb
    assert torch.equal(blob[:res.blob_bytes], pblob)


@pytest.mark.parametrize("shape,dt,psnr,domain", [((40, 37, 70), np.float32, 80.0, 1),
                                                  ((300, 200), np.float64, 120.0, 0),
                                                  ((20000,), np.float32, 40.0, 0)])
def test_async_matches_plain(ctx, shape, dt, psnr, domain):
    from paper_1805_07384_amd import fpsz
    x = (synth.grf_numpy(shape, -3.0, 8) * 5.0 + 1.0).astype(dt)
    print("case async shape=%s dtype=%s psnr=%s domain=%d" % (shape, x.dtype, psnr, domain),
          flush=True)
    xt = torch.from_numpy(x).cuda()
    pblob, pinfo = _plain(ctx, xt, psnr, domain)
    ws = torch.full((fpsz.compress_workspace_bytes(x.shape, xt.dtype),), 0xA5, dtype=torch.uint8,
                    device="cuda")
    blob = torch.full((fpsz.compress_bound(x.shape, xt.dtype),), 0x5A, dtype=torch.uint8,
                      device="cuda")
    res_t = torch.zeros(fpsz.ASYNC_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    assert ctx.compress_async_into(xt, psnr, ws, blob, res_t, domain) == 0
    _check(fpsz.async_result(res_t), blob, pblob, pinfo)


def test_async_in_a_graph(ctx):
    # captured once, replayed on three fields copied into the captured input
    from paper_1805_07384_amd import fpsz
    shape, psnr = (48, 64, 96), 80.0
    xs = [synth.field_3d_lognormal(shape=shape, seed=s) for s in (11, 12, 13)]
    xin = torch.from_numpy(xs[0]).cuda()
    ws = torch.empty(fpsz.compress_workspace_bytes(shape, torch.float32), dtype=torch.uint8,
                     device="cuda")
    blob = torch.empty(fpsz.compress_bound(shape, torch.float32), dtype=torch.uint8,
                       device="cuda")
    res_t = torch.zeros(fpsz.ASYNC_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # a warm-up call outside the capture
        assert ctx.compress_async_into(xin, psnr, ws, blob, res_t, fpsz.TILE, side) == 0
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("case async graph capture", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st = ctx.compress_async_into(xin, psnr, ws, blob, res_t, fpsz.TILE,
                                     torch.cuda.current_stream())
    assert st == 0
    for k, x in enumerate(xs):
        print("case async graph replay %d" % k, flush=True)
        xin.copy_(torch.from_numpy(x))
        res_t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        res = fpsz.async_result(res_t)
        pblob, pinfo = _plain(ctx, torch.from_numpy(x).cuda(), psnr, fpsz.TILE)
        _check(res, blob, pblob, pinfo)


def test_async_device_statuses(ctx):
    from paper_1805_07384_amd import fpsz
    x = synth.grf_numpy((64, 64), -3.0, 2).astype(np.float32)
    x[5, 7] = np.nan
    xt = torch.from_numpy(x).cuda()
    ws = torch.empty(fpsz.compress_workspace_bytes(x.shape, xt.dtype), dtype=torch.uint8,
                     device="cuda")
    blob = torch.empty(fpsz.compress_bound(x.shape, xt.dtype), dtype=torch.uint8, device="cuda")
    res_t = torch.zeros(fpsz.ASYNC_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    print("case async nonfinite", flush=True)
    assert ctx.compress_async_into(xt, 80.0, ws, blob, res_t) == 0
    assert fpsz.async_result(res_t).status == fpsz.E_NONFINITE
    # a blob buffer too small for the blob: CAPACITY with the size needed
    y = synth.grf_numpy((64, 64), -3.0, 2).astype(np.float32)
    yt = torch.from_numpy(y).cuda()
    pblob, pinfo = _plain(ctx, yt, 120.0, fpsz.GLOBAL)
    small = torch.empty(pblob.numel() // 2 // 8 * 8, dtype=torch.uint8, device="cuda")
    print("case async capacity", flush=True)
    assert ctx.compress_async_into(yt, 120.0, ws, small, res_t) == 0
    r = fpsz.async_result(res_t)
    assert r.status == fpsz.E_CAPACITY and r.blob_bytes == pblob.numel()


def _blob(ctx, x, psnr, domain):
    from paper_1805_07384_amd import fpsz
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    pblob, pinfo = _plain(ctx, xt, psnr, domain)
    return xt, pblob


def _dasync(ctx, blob, header, shape, dtype, orig=None, stream=None):
    from paper_1805_07384_amd import fpsz
    wd = torch.full((fpsz.decompress_workspace_bytes(shape, dtype),), 0xA5, dtype=torch.uint8,
                    device="cuda")
    out = torch.full(shape, 7.0, dtype=dtype, device="cuda")
    res = torch.zeros(fpsz.DECOMPRESS_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    st = ctx.decompress_async_into(blob, blob.numel(), header, wd, out, res, orig, stream)
    return st, out, res, wd


@pytest.mark.parametrize("shape,dt,psnr,domain", [((40, 37, 70), np.float32, 80.0, 1),
                                                  ((300, 200), np.float64, 120.0, 0),
                                                  ((20000,), np.float32, 40.0, 0)])
def test_decompress_async_matches_sync(ctx, shape, dt, psnr, domain):
    from paper_1805_07384_amd import fpsz
    x = (synth.grf_numpy(shape, -3.0, 9) * 5.0 + 1.0).astype(dt)
    print("case decompress async shape=%s dtype=%s psnr=%s" % (shape, x.dtype, psnr), flush=True)
    xt, blob = _blob(ctx, x, psnr, domain)
    header = blob[:256].cpu().numpy().tobytes()
    y_sync, st_sync = ctx.decompress_verify(blob, xt)
    st, out, res_t, _ = _dasync(ctx, blob, header, xt.shape, xt.dtype, xt)
    assert st == 0
    r = fpsz.decompress_result(res_t)
    assert r.status == 0 and r.checked == 1
    assert torch.equal(out.cpu(), y_sync.cpu())
    assert r.sse == st_sync["sse"] and r.max_abs_err == st_sync["max_abs_err"]
    assert r.n_over_eb == st_sync["n_over_eb"]
    assert abs(r.psnr - st_sync["psnr"]) <= 1e-12 * abs(st_sync["psnr"])
    # without an original: the reconstruction only
    st, out2, res_t, _ = _dasync(ctx, blob, header, xt.shape, xt.dtype, None)
    r = fpsz.decompress_result(res_t)
    assert st == 0 and r.status == 0 and r.checked == 0 and torch.equal(out2, out)


def test_decompress_async_header_mismatch_and_constant(ctx):
    from paper_1805_07384_amd import fpsz
    shape = (64, 96)
    xa = synth.grf_numpy(shape, -3.0, 3).astype(np.float32)
    xb = (synth.grf_numpy(shape, -3.0, 4) * 2.0).astype(np.float32)
    _, ba = _blob(ctx, xa, 80.0, 0)
    _, bb = _blob(ctx, xb, 80.0, 0)
    print("case decompress async header mismatch", flush=True)
    # blob b (zero-padded to blob a's size) with the header of blob a: the
    # host plan is valid, the device finds the blob's own header differs and
    # reports CORRUPT, never a fault
    m = max(ba.numel(), bb.numel())
    bbuf = torch.zeros(m, dtype=torch.uint8, device="cuda")
    bbuf[:bb.numel()] = bb
    st, _, res_t, _ = _dasync(ctx, bbuf[:ba.numel()], ba[:256].cpu().numpy().tobytes(), shape,
                              torch.float32)
    assert st == 0
    assert fpsz.decompress_result(res_t).status == fpsz.E_CORRUPT
    print("case decompress async constant", flush=True)
    c = np.full(shape, -1.5, dtype=np.float32)
    ct, cb = _blob(ctx, c, 80.0, 1)
    st, out, res_t, _ = _dasync(ctx, cb, cb[:256].cpu().numpy().tobytes(), shape, torch.float32,
                                ct)
    r = fpsz.decompress_result(res_t)
    assert st == 0 and r.status == 0 and r.checked == 1 and r.sse == 0.0
    assert torch.equal(out, ct)


def test_decompress_async_in_a_graph(ctx):
    # captured once, replayed three times (the output cleared by eager work
    # in between): every replay equals the synchronous call
    from paper_1805_07384_amd import fpsz
    x = synth.field_3d_lognormal(shape=(48, 64, 96), seed=21)
    xt, blob = _blob(ctx, x, 80.0, 1)
    header = blob[:256].cpu().numpy().tobytes()
    y_sync, st_sync = ctx.decompress_verify(blob, xt)
    wd = torch.empty(fpsz.decompress_workspace_bytes(xt.shape, xt.dtype), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty_like(xt)
    res_t = torch.zeros(fpsz.DECOMPRESS_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert ctx.decompress_async_into(blob, blob.numel(), header, wd, out, res_t, xt, side) == 0
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("case decompress async graph capture", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st = ctx.decompress_async_into(blob, blob.numel(), header, wd, out, res_t, xt,
                                       torch.cuda.current_stream())
    assert st == 0
    for k in range(3):
        print("case decompress async graph replay %d" % k, flush=True)
        out.fill_(0.0)
        res_t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        r = fpsz.decompress_result(res_t)
        assert r.status == 0 and r.checked == 1
        assert torch.equal(out, y_sync)
        assert r.sse == st_sync["sse"] and r.n_over_eb == st_sync["n_over_eb"]
