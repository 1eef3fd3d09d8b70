"""fpsz_compress_async (the compress entry point that writes its outcome to
device memory and never synchronizes) against fpsz_compress: identical blobs
and reports when called directly, when captured in a graph and replayed on
new data (each replay checked against the direct call, with eager work and
synchronizations between replays), and device-side statuses."""
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
