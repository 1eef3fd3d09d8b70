"""The request loop (fpsz_server_*) on the GPU, through the C ABI.

Every request served in a mix -- admitted by HBM budget, batched with other
requests of its round, overlapped with other rounds on other streams -- must
give exactly what the plain call gives alone.  The budget must hold at all
times, and bad requests must fail alone.
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


def _small_trace(n, seed, rate):
    # the serving trace recipe at small sizes (64 KiB .. 8 MiB, median 1 MiB)
    return synth.serve_trace(n_req=n, rate=rate, seed=seed, median_bytes=1 << 20, sigma_ln=1.0,
                             min_bytes=64 << 10, max_bytes=8 << 20)


@pytest.mark.parametrize("rate,budget_mib,streams", [(1e6, 64, 1), (1e6, 64, 4), (400.0, 1024, 2)])
def test_served_equals_plain(ctx, rate, budget_mib, streams):
    from paper_1805_07384_amd import serving
    print("case serve rate=%g budget=%d MiB streams=%d" % (rate, budget_mib, streams), flush=True)
    trace = _small_trace(80, seed=11, rate=rate)
    work = serving.build_workload(trace, pool_size=12, ctx=ctx)
    plain, ps = serving.replay_plain(ctx, work)
    served, ss = serving.replay_served(ctx, work, hbm_budget=budget_mib << 20,
                                       arena_bytes=budget_mib << 20, max_inflight=32,
                                       n_streams=streams)
    st = ss["server"]
    print("plain", ps["latency"], "served", ss["latency"], st, flush=True)
    assert all(o[0] == 0 for o in plain)
    assert serving.same_results(plain, served) == 0
    assert st["completed"] == st["submitted"] == len(work) and st["failed"] == 0
    assert st["peak_held_bytes"] <= budget_mib << 20
    if rate > 1e5 and streams == 1:
        # a burst on one stream: arrivals wait while the stream is busy and
        # are admitted together (whether two of one round share a field
        # class, and so share a launch, depends on arrival timing; the
        # loaded served leg of the benchmark reports those launches)
        assert st["peak_inflight"] > 1 and st["rounds"] < st["submitted"]
    # a sample of the served results against the CPU oracle itself
    import oracle
    comp = [i for i, w in enumerate(work) if w["kind"] == "compress"][:3]
    deco = [i for i, w in enumerate(work) if w["kind"] == "decompress"][:2]
    for i in comp:
        w = work[i]
        _, buf, nb = served[i]
        ob, _ = oracle.compress(w["x"].cpu().numpy(), w["psnr"])
        assert buf[:nb].cpu().numpy().tobytes() == ob, "served blob %d differs from the oracle" % i
    for i in deco:
        w = work[i]
        _, buf, _ = served[i]
        oy = oracle.decompress(w["blob"][:w["nbytes"]].cpu().numpy().tobytes())
        assert np.array_equal(buf.cpu().numpy().view(np.uint32), oy.view(np.uint32))


def test_server_rejects_bad_requests(ctx):
    from paper_1805_07384_amd import fpsz
    print("case serve errors", flush=True)
    srv = fpsz.Server(ctx, hbm_budget=8 << 20, arena_bytes=8 << 20, max_inflight=4, n_streams=1)
    x = torch.from_numpy(synth.field_2d_grf(64, 80, seed=2)).cuda()
    blob = torch.empty(fpsz.compress_bound((64, 80)), dtype=torch.uint8, device="cuda")
    big = torch.zeros((1024, 4096), dtype=torch.float32, device="cuda")  # 16 MiB > budget
    big_blob = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    a = srv.submit_compress(x, 80.0, blob)
    b = srv.submit_compress(big, 80.0, big_blob)
    ra, rb = srv.wait(a), srv.wait(b)
    assert ra["status"] == fpsz.OK and rb["status"] == fpsz.E_CAPACITY
    nb = ra["out_bytes"]
    # decompress with a shape that differs from the blob's
    wrong = torch.empty((80, 64), dtype=torch.float32, device="cuda")
    c = srv.submit_decompress(blob, nb, wrong)
    assert srv.wait(c)["status"] == fpsz.E_INVALID_ARG
    # corrupted blob
    bad = blob[:nb].clone()
    bad[nb // 2] ^= 0x10
    out = torch.empty((64, 80), dtype=torch.float32, device="cuda")
    d = srv.submit_decompress(bad, nb, out)
    assert srv.wait(d)["status"] == fpsz.E_CORRUPT
    # and a good one still works afterwards
    e = srv.submit_decompress(blob, nb, out)
    assert srv.wait(e)["status"] == fpsz.OK
    ref = ctx.decompress(blob[:nb])
    assert torch.equal(out, ref)
    srv.close()
