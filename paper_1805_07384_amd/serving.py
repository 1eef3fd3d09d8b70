"""Replay of a seeded request trace through the library's server
(continuous batching, HBM-budget admission) and through one-at-a-time plain
calls, on the same device-resident inputs.

Arrivals follow the trace's Poisson times in real time.  Latency is arrival to
completion; the served replay reads completion times from the server's
clock, mapped onto the replay clock at the start.  Both replays write to
their own output buffers so their results can be compared bit for bit.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import fpsz, synth


def build_workload(trace, device="cuda", pool_size=64, ctx=None, alpha=-3.0, log=None):
    """Device-resident inputs for every request of ``trace``.

    Compress requests get a float32 field of their shape cut from a periodic
    GRF (spectrum k^alpha) of the same dimensionality at a seeded offset.
    Decompress requests pick one blob from a pool of ``pool_size`` blobs made
    beforehand (by plain calls) from fields of the trace's own size mix; the
    request's output shape is that blob's field shape."""
    ctx = ctx or fpsz.default_context(torch.device(device).index or 0)
    bases = synth.periodic_bases(alpha, device=device)
    comp = [r for r in trace if r["kind"] == "compress"]
    pool_src = comp[:pool_size] if len(comp) >= pool_size else comp
    pool = []
    if log:
        log("blob pool of %d" % len(pool_src))
    for r in pool_src:
        x = synth.periodic_crop(bases, r["shape"], r["seed"] + 7)
        b, info = ctx.compress(x, r["psnr"])
        pool.append({"blob": b, "nbytes": int(b.numel()), "shape": tuple(x.shape)})
        del x
    work = []
    for i, r in enumerate(trace):
        if log and i % 50 == 0:
            torch.cuda.synchronize()
            log("request inputs %d / %d" % (i, len(trace)))
        w = dict(r)
        if r["kind"] == "compress":
            x = synth.periodic_crop(bases, r["shape"], r["seed"])
            w["x"] = x
            w["bytes"] = x.numel() * 4
            # the raw size and 1 MiB: blobs up to 120 dB stay below 32 bits a point
            w["cap"] = x.numel() * 4 + (1 << 20)
        else:
            p = pool[min(int(r["pick"] * len(pool)), len(pool) - 1)]
            w["blob"], w["nbytes"], w["shape"] = p["blob"], p["nbytes"], p["shape"]
            w["bytes"] = int(np.prod(p["shape"])) * 4
        work.append(w)
    torch.cuda.synchronize()
    return work


def _lat_stats(lat):
    lat = np.asarray(lat, dtype=np.float64)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}


def replay_plain(ctx, work, device="cuda"):
    """One request at a time, in arrival order, each a synchronous plain call."""
    max_c = max([w["x"].numel() for w in work if w["kind"] == "compress"] or [1])
    max_d = max([int(np.prod(w["shape"])) for w in work if w["kind"] == "decompress"] or [1])
    shp_c = [w["x"].shape for w in work if w["kind"] == "compress"]
    shp_d = [w["shape"] for w in work if w["kind"] == "decompress"]
    ws_c = torch.empty(max([fpsz.compress_workspace_bytes(tuple(s)) for s in shp_c] or [256]),
                       dtype=torch.uint8, device=device)
    ws_d = torch.empty(max([fpsz.decompress_workspace_bytes(tuple(s)) for s in shp_d] or [256]),
                       dtype=torch.uint8, device=device)
    outs = []
    lat = []
    total = 0
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for w in work:
        while time.perf_counter() - t0 < w["t"]:
            pass
        if w["kind"] == "compress":
            blob = torch.empty(w["cap"], dtype=torch.uint8, device=device)
            st, nb, _ = ctx.compress_into(w["x"], w["psnr"], ws_c, blob, fpsz.GLOBAL, stream)
            outs.append((st, blob, nb))
        else:
            out = torch.empty(w["shape"], dtype=torch.float32, device=device)
            st = ctx.decompress_into(w["blob"], w["nbytes"], ws_d, out, stream)
            outs.append((st, out, w["bytes"]))
        done = time.perf_counter() - t0
        lat.append(done - w["t"])
        total += w["bytes"]
    span = time.perf_counter() - t0 - work[0]["t"]
    del max_c, max_d
    return outs, {"latency": _lat_stats(lat), "gbps": total / span / 1e9, "span_s": span,
                  "requests": len(work)}


def replay_served(ctx, work, hbm_budget, arena_bytes, max_inflight=64, n_streams=4,
                  device="cuda"):
    """The same trace through the server: each request is submitted at its
    arrival time; completions are collected as they come."""
    srv = fpsz.Server(ctx, hbm_budget, arena_bytes, max_inflight, n_streams)
    outs = [None] * len(work)
    ids = {}
    # allocate every output before the clock starts (the server allocates nothing)
    bufs = []
    for w in work:
        if w["kind"] == "compress":
            bufs.append(torch.empty(w["cap"], dtype=torch.uint8, device=device))
        else:
            bufs.append(torch.empty(w["shape"], dtype=torch.float32, device=device))
    torch.cuda.synchronize()
    res = {}
    t0 = time.perf_counter()
    off = srv.stats()["now"] - (time.perf_counter() - t0)  # server clock at replay t = 0
    pending = []
    for i, w in enumerate(work):
        while time.perf_counter() - t0 < w["t"]:
            if pending:
                r = srv.poll(pending[0])
                if r is not None:
                    res[pending.pop(0)] = r
        if w["kind"] == "compress":
            rid = srv.submit_compress(w["x"], w["psnr"], bufs[i])
        else:
            rid = srv.submit_decompress(w["blob"], w["nbytes"], bufs[i])
        ids[i] = rid
        pending.append(rid)
    for rid in pending:
        res[rid] = srv.wait(rid)
    stats = srv.stats()
    srv.close()
    lat = []
    total = 0
    last = 0.0
    for i, w in enumerate(work):
        r = res[ids[i]]
        done = r["t_done"] - off
        lat.append(done - w["t"])
        last = max(last, done)
        total += w["bytes"]
        outs[i] = (r["status"], bufs[i], r["out_bytes"])
    span = last - work[0]["t"]
    return outs, {"latency": _lat_stats(lat), "gbps": total / span / 1e9, "span_s": span,
                  "requests": len(work), "server": stats}


def same_results(a, b) -> int:
    """Number of requests whose status and output differ between two replays."""
    bad = 0
    for (sa, ta, na), (sb, tb, nb) in zip(a, b):
        if sa != sb or na != nb:
            bad += 1
        elif sa == fpsz.OK and ta.dtype == torch.uint8:
            bad += int(not torch.equal(ta[:na], tb[:nb]))
        elif sa == fpsz.OK:
            bad += int(not torch.equal(ta.view(torch.int32), tb.view(torch.int32)))
    return bad
