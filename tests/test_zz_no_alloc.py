"""fpsz_compress_static (the compress entry point that allocates nothing:
its workspace is the library's static device array) against fpsz_compress on
the same inputs: byte-identical blobs and identical reports, on two calls in
a row (the second smaller, so it runs on what the first left in the array),
and the size limit refused before any launch."""
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


def _both(ctx, x: np.ndarray, psnr: float, domain: int):
    from paper_1805_07384_amd import fpsz
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    cap = fpsz.compress_bound(x.shape, xt.dtype)
    ws = torch.full((fpsz.compress_workspace_bytes(x.shape, xt.dtype),), 0xA5,
                    dtype=torch.uint8, device="cuda")
    b1 = torch.full((cap,), 0x5A, dtype=torch.uint8, device="cuda")
    b2 = torch.full((cap,), 0x3C, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    st1, n1, i1 = ctx.compress_into(xt, psnr, ws, b1, domain)
    st2, n2, i2 = ctx.compress_static(xt, psnr, b2, domain)
    torch.cuda.synchronize()
    assert st1 == 0 and st2 == 0, (st1, st2)
    assert n1 == n2
    assert torch.equal(b1[:n1], b2[:n2])
    assert i1.as_dict() == i2.as_dict()
    return i2.as_dict()


def test_static_matches_plain_two_calls():
    from paper_1805_07384_amd import fpsz
    c = fpsz.Context(0) if torch.cuda.is_available() else pytest.skip("no GPU")
    # first call: 3D float32 GRF with patches at 120 dB (several MB of workspace)
    x1 = synth.field_3d_lognormal(shape=(80, 96, 160), seed=4)
    print("case static 1: shape=%s float32 psnr=120" % (x1.shape,), flush=True)
    info = _both(c, x1, 120.0, fpsz.GLOBAL)
    assert info["n_patches"] > 0
    # second call, smaller: float64 with outliers and two-record patches,
    # TILE domain
    import patchfield as pf
    x2 = pf.f64_patch_field()
    print("case static 2: shape=%s float64 psnr=%s" % (x2.shape, pf.PSNR), flush=True)
    info = _both(c, x2, pf.PSNR, fpsz.TILE)
    assert info["n_outliers"] > 0 and info["n_patches"] > 0
    # the same small field again, GLOBAL domain, f32
    x3 = synth.field_2d_grf(200, 130, seed=2)
    print("case static 3: shape=%s float32 psnr=60" % (x3.shape,), flush=True)
    _both(c, x3, 60.0, fpsz.GLOBAL)


def test_static_refuses_oversized_field():
    from paper_1805_07384_amd import fpsz
    c = fpsz.Context(0) if torch.cuda.is_available() else pytest.skip("no GPU")
    shape = (256, 256, 640)  # 2 bytes per point of residual codes alone exceed 64 MiB
    assert fpsz.compress_workspace_bytes(shape, torch.float32) > fpsz.STATIC_WORKSPACE_BYTES
    print("case static oversized: shape=%s" % (shape,), flush=True)
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    blob = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st, nb, _ = c.compress_static(x, 80.0, blob)
    assert st == fpsz.E_CAPACITY and nb == 0
    assert b"static workspace" in c.lib.fpsz_last_error(c.handle)
