#!/usr/bin/env python3
"""Benchmark of fixed-PSNR SZ-style compression on one MI355X.

Workload (one step): the 3D float32 512^3 field exp(g), g a unit-variance
Gaussian random field with power spectrum k^(-11/3) (a lognormal(0,1)
density contrast), compressed, decompressed and checked (Eq. 4 PSNR) at
each target PSNR of the sweep 40/60/80/100/120 dB.  Inputs are generated on
the GPU from a fixed seed and are resident in HBM before timing starts.

value = uncompressed bytes pushed through compress + decompress + verify per
second, summed over the sweep (GB/s, 1e9 B/s).  Per-target compress and
decompress rates, |PSNR - target| and operation-level roofline fractions
(algorithmic bytes: compress 2s + b/8, decompress b/8 + s, decompress with
the check b/8 + 2s per point, over 8 TB/s) are reported beside it, with the
device-copy bandwidth measured in the same run.  Side legs: the 2D float32
512x512 field (latency per call), the 3D float64 1024^3 field with spikes at
100 dB, 120 batched 1800x3600 fields, and a served request trace at two
arrival rates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--edge", type=int, default=512, help="cube edge of the 3D field")
    ap.add_argument("--psnrs", default="40,60,80,100,120")
    # TILE restarts the Lorenzo stencil at each tile: the same reconstruction
    # as GLOBAL (Theorem 1), no face projections in decompression, and on the
    # benchmark field slightly smaller blobs; GLOBAL is measured as a leg
    ap.add_argument("--domain", choices=["global", "tile"], default="tile")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=128,
                    help="planes of the field the CPU oracle is timed on")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-kernel HIP-event timing")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 120-field batched-vs-plain leg")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served-vs-plain request-trace leg")
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--served-rates", default="200,3000,20000",
                    help="arrival rates (requests/s) the trace is replayed at")
    ap.add_argument("--no-other-domain", action="store_true",
                    help="skip the sweep leg in the other Lorenzo domain")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the closed-loop, in-loop and transform legs")
    ap.add_argument("--no-c1", action="store_true", help="skip the 512x512 latency leg")
    ap.add_argument("--no-c5", action="store_true", help="skip the 1024^3 float64 leg")
    ap.add_argument("--separate-verify", action="store_true",
                    help="check each reconstruction with its own fpsz_verify call instead of "
                         "in the decompression pass (fpsz_decompress_verify)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy the field once with a plain device copy "
                         "(the reference kernel for scaling HBM byte counters)")
    return ap.parse_args()


# Source files whose kernels the HBM traffic figures under profiles/ were
# measured on; a figure whose recorded hash differs is stale and not reported.
SRC_FILES = ["paper_1805_07384_amd/csrc/compress.hip", "paper_1805_07384_amd/csrc/decompress.hip",
             "paper_1805_07384_amd/csrc/api.hip", "paper_1805_07384_amd/csrc/batch.hip",
             "paper_1805_07384_amd/csrc/serve.hip", "paper_1805_07384_amd/csrc/fpsz_internal.h",
             "paper_1805_07384_amd/csrc/host_common.h", "paper_1805_07384_amd/build.py",
             "include/fpsz.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_lognormal512_sweep.txt")


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read() + b"\0")
    return h.hexdigest()


def measured_traffic(domain: str):
    """Per-launch HBM bytes of each stage (FETCH_SIZE + WRITE_SIZE, scaled by
    the copy-kernel calibration) from the committed counter summary, or {}
    when the summary is missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    rec, tr = None, {}
    with open(TRAFFIC_FILE) as fh:
        for ln in fh:
            f = ln.split()
            if len(f) == 2 and f[0] == "source_sha256":
                rec = f[1]
            elif len(f) == 4 and f[0] == "traffic" and f[1] == domain:
                tr[f[2]] = float(f[3])
    return tr if rec == source_hash() else {}


# Algorithmic bytes per element of each kernel (s = element size, b = bits
# per value of the blob).  Compression must read the field twice (the bound
# needs the global value range before any point is quantized) and write the
# blob; decompression reads the blob and writes the field; the check reads
# both fields.  The residual-code intermediate (2 B per point, written by
# quant and read by encode; written by decode and read by rec), halos and
# face arrays are implementation traffic, not algorithmic.
# With the check in the decompression pass, the reconstruction kernel also
# reads the original (s more bytes); the reconstruction is not read back.
def algorithmic_bytes(stage: str, n: int, s: int, b: float, fused_check: bool = False) -> float:
    per = {
        "range": s,
        "quant": s,
        "encode": b / 8.0,
        "decode": b / 8.0,
        "rec": 2.0 * s if fused_check else s,
        "decode_rec": b / 8.0 + (2.0 * s if fused_check else s),
        "verify": 2.0 * s,
    }.get(stage)
    return None if per is None else per * n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_cpu, psnrs, planes, domain):
    """The CPU oracle, untuned, single-threaded, on a contiguous slab of the
    same field; per-stage wall times from the oracle's own timers."""
    import numpy as np

    import oracle

    sample = np.ascontiguousarray(x_cpu[:planes])
    stages = {}
    t0 = time.perf_counter()
    for p in psnrs:
        blob, t = oracle.compress(sample, p, domain, trace=False)
        y = oracle.decompress(blob)
        h = oracle.header(blob)
        oracle.stats(sample, y, h["vr"], h["eb"])
        for k, v in oracle.stage_times().items():
            stages[k] = stages.get(k, 0.0) + v
    dt = time.perf_counter() - t0
    gbps = sample.nbytes * len(psnrs) / dt / 1e9
    ne = sample.size * len(psnrs)
    return {"value": round(gbps, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "float32 slab %s of the benchmark field, %s domain, compress+decompress+Eq.4 "
                      "stats at %s dB (%.1f s)" % (list(sample.shape), "TILE" if domain else "GLOBAL",
                                                  "/".join("%g" % p for p in psnrs), dt),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "stage_ns_per_point": {k: round(v / ne * 1e9, 2) for k, v in stages.items()}}


def op_fracs(n, s, bits, t_c, t_d, t_dc=None):
    """Operation-level fractions of the 8 TB/s HBM peak on algorithmic bytes:
    compress 2s + b/8 (the range read, the quantization read, the blob write),
    decompress b/8 + s (blob read, field write), decompress with the check
    b/8 + 2s (the original read too)."""
    b8 = bits / 8.0
    out = {"compress": round((2 * s + b8) * n / t_c / 1e9 / HBM_PEAK_GBPS, 4)}
    if t_d:
        out["decompress"] = round((b8 + s) * n / t_d / 1e9 / HBM_PEAK_GBPS, 4)
    if t_dc:
        out["decompress_check"] = round((b8 + 2 * s) * n / t_dc / 1e9 / HBM_PEAK_GBPS, 4)
    return out


def device_copy_gbps(x, reps=10):
    """Bandwidth of a plain device copy of the field (read + write bytes)."""
    import numpy as np
    import torch

    y = torch.empty_like(x)
    ts = []
    for _ in range(reps + 2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    del y
    return 2.0 * x.numel() * x.element_size() / float(np.median(ts[2:])) / 1e9


def timed_calls(fn, reps, warm=3):
    import numpy as np
    import torch

    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), float(np.percentile(ts, 90))


def c1_leg(ctx, dev, domain):
    """2D float32 512x512 GRF (k^-3) on [-50, 50] at 80 dB: a latency-bound
    call; median and p90 of 30 calls each after 3 warm-ups, in the sweep's
    Lorenzo domain, and the same calls in the other domain."""
    import torch

    from paper_1805_07384_amd import fpsz, synth

    x = synth.field_2d_grf(512, 512, seed=1, backend="torch", device=dev).contiguous()
    ws_c = torch.empty(fpsz.compress_workspace_bytes(tuple(x.shape)), dtype=torch.uint8, device=dev)
    ws_d = torch.empty(fpsz.decompress_workspace_bytes(tuple(x.shape)), dtype=torch.uint8,
                       device=dev)
    blob = torch.empty(fpsz.compress_bound(tuple(x.shape)), dtype=torch.uint8, device=dev)
    out = torch.empty_like(x)
    n, s = x.numel(), 4

    def one(dom):
        st, nb, info = ctx.compress_into(x, 80.0, ws_c, blob, dom)
        assert st == fpsz.OK
        c = timed_calls(lambda: ctx.compress_into(x, 80.0, ws_c, blob, dom), 30)
        d = timed_calls(lambda: ctx.decompress_into(blob, nb, ws_d, out), 30)
        dv = timed_calls(lambda: ctx.decompress_verify_into(blob, nb, ws_d, out, x), 30)
        st2, stats = ctx.decompress_verify_into(blob, nb, ws_d, out, x)
        return {"domain": "tile" if dom == fpsz.TILE else "global",
                "compress_us": round(c[0] * 1e6, 1), "compress_us_p90": round(c[1] * 1e6, 1),
                "decompress_us": round(d[0] * 1e6, 1), "decompress_us_p90": round(d[1] * 1e6, 1),
                "decompress_check_us": round(dv[0] * 1e6, 1),
                "bits_per_value": round(info.bits_per_value, 4),
                "achieved_psnr": round(stats.psnr, 4), "dpsnr": round(stats.psnr - 80.0, 4),
                "n_over_eb": stats.n_over_eb,
                "op_frac": op_fracs(n, s, info.bits_per_value, c[0], d[0], dv[0])}

    r = {"workload": "2D float32 512x512 GRF k^-3 on [-50, 50], seed 1, 80 dB"}
    r.update(one(domain))
    r["other_domain"] = one(fpsz.GLOBAL if domain == fpsz.TILE else fpsz.TILE)
    return r


def c5_leg(ctx, dev, domain):
    """3D float64 1024^3 GRF (k^-3) with 1 % spikes of 1000 sigma at 100 dB:
    device-resident compress and decompress with the fused Eq. 4 check,
    median of 3 calls each after one warm-up, in the sweep's Lorenzo domain
    and in the other."""
    import torch

    from paper_1805_07384_amd import fpsz, synth

    shape = (1024, 1024, 1024)
    x = synth.field_3d_spiky_f64(shape=shape, seed=5, backend="torch", device=dev).contiguous()
    torch.cuda.synchronize()
    n, s = x.numel(), 8
    ws_c = torch.empty(fpsz.compress_workspace_bytes(shape, x.dtype), dtype=torch.uint8, device=dev)
    ws_d = torch.empty(fpsz.decompress_workspace_bytes(shape, x.dtype), dtype=torch.uint8,
                       device=dev)
    blob = torch.empty(n * 4 + (1 << 20), dtype=torch.uint8, device=dev)
    out = torch.empty_like(x)

    def one(dom):
        st, nb, info = ctx.compress_into(x, 100.0, ws_c, blob, dom)
        if st != fpsz.OK:
            raise fpsz.FpszError(st, "C5 compress")
        c = timed_calls(lambda: ctx.compress_into(x, 100.0, ws_c, blob, dom), 3, warm=1)
        d = timed_calls(lambda: ctx.decompress_into(blob, nb, ws_d, out), 3, warm=1)
        dv = timed_calls(lambda: ctx.decompress_verify_into(blob, nb, ws_d, out, x), 3, warm=1)
        st2, stats = ctx.decompress_verify_into(blob, nb, ws_d, out, x)
        return {"domain": "tile" if dom == fpsz.TILE else "global",
                "compress_ms": round(c[0] * 1e3, 3), "decompress_ms": round(d[0] * 1e3, 3),
                "decompress_check_ms": round(dv[0] * 1e3, 3),
                "compress_gbps": round(n * s / c[0] / 1e9, 1),
                "decompress_gbps": round(n * s / d[0] / 1e9, 1),
                "bits_per_value": round(info.bits_per_value, 4), "n_outliers": info.n_outliers,
                "n_patches": info.n_patches, "achieved_psnr": round(stats.psnr, 4),
                "dpsnr": round(stats.psnr - 100.0, 4), "n_over_eb": stats.n_over_eb,
                "op_frac": op_fracs(n, s, info.bits_per_value, c[0], d[0], dv[0])}

    res = {"workload": "3D float64 1024^3 GRF k^-3 plus 1%% spikes of 1000 sigma, seed 5, 100 dB",
           "bytes": n * s}
    res.update(one(domain))
    res["other_domain"] = one(fpsz.GLOBAL if domain == fpsz.TILE else fpsz.TILE)
    del x, blob, ws_c, ws_d, out
    torch.cuda.empty_cache()
    return res


def progress(msg):
    print("[bench %.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def batched_leg(ctx, dev):
    """120 2D f32 1800x3600 fields (slope U[-4,-2], range 10^U(-3,4), target
    U[40,120] dB): 120 plain calls vs one batch (captured graph, autotuned
    launch shapes).  Compress only, inputs resident; median of 3 runs each."""
    import numpy as np
    import torch

    from paper_1805_07384_amd import fpsz, synth

    spec = synth.batch_fields_spec(120, seed=3)
    progress("batched leg: generating 120 fields")
    xs = [synth.batch_field(sp, backend="torch", device=dev).contiguous() for sp in spec]
    torch.cuda.synchronize()
    progress("batched leg: plain calls")
    psnrs = [sp["psnr"] for sp in spec]
    caps = [fpsz.compress_bound(tuple(x.shape)) // 2 for x in xs]
    blobs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    total = sum(x.numel() * 4 for x in xs)
    ws = torch.empty(fpsz.compress_workspace_bytes((1800, 3600)), dtype=torch.uint8, device=dev)
    pblob = torch.empty(max(caps), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def plain_once():
        sizes = []
        for x, p in zip(xs, psnrs):
            st, nb, _ = ctx.compress_into(x, p, ws, pblob, fpsz.GLOBAL, stream)
            if st != fpsz.OK:
                raise fpsz.FpszError(st, "plain compress")
            sizes.append(nb)
        return sizes

    plain_once()
    tp = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        psz = plain_once()
        tp.append(time.perf_counter() - t0)
    progress("batched leg: batch + autotune")
    b = fpsz.Batch(ctx, xs, psnrs, blobs, graph=True)
    b.run()
    tuned_ms = b.autotune(reps=2)
    progress("batched leg: timed batch runs")
    tb = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, nb, info, sts = b.run()
        tb.append(time.perf_counter() - t0)
    shape = b.launch_shape(0)
    b.close()
    progress("batched leg: accuracy check")
    # accuracy per field (untimed): decompress + Eq. 4
    dws = torch.empty(fpsz.decompress_workspace_bytes((1800, 3600)), dtype=torch.uint8, device=dev)
    out = torch.empty((1800, 3600), dtype=torch.float32, device=dev)
    dps, over = [], 0
    for i, x in enumerate(xs):
        if ctx.decompress_into(blobs[i], nb[i], dws, out, stream) != fpsz.OK:
            raise fpsz.FpszError(fpsz.E_CORRUPT, "batched blob %d" % i)
        stt = ctx.verify(x, out, info[i]["vr"], info[i]["eb"])
        dps.append(stt["psnr"] - psnrs[i])
        over += stt["n_over_eb"]
    # the same fields through the closed-loop correction (one call each)
    progress("batched leg: closed-loop accuracy")
    dps_c = []
    for i, x in enumerate(xs):
        st, nbc, ic = ctx.compress_closed_loop_into(x, psnrs[i], ws, pblob, fpsz.GLOBAL, stream)
        if st != fpsz.OK or ctx.decompress_into(pblob, nbc, dws, out, stream) != fpsz.OK:
            raise fpsz.FpszError(st, "closed-loop field %d" % i)
        stt = ctx.verify(x, out, ic.vr, ic.eb)
        dps_c.append(stt["psnr"] - psnrs[i])
        over += stt["n_over_eb"]
    tp_m, tb_m = float(np.median(tp)), float(np.median(tb))
    res = {"workload": "120 2D float32 1800x3600 GRF fields, slope U[-4,-2], range 10^U(-3,4), "
                       "target U[40,120] dB, seed 3",
           "bytes": total, "plain_gbps": round(total / tp_m / 1e9, 2),
           "batched_gbps": round(total / tb_m / 1e9, 2), "speedup": round(tp_m / tb_m, 3),
           "plain_ms": round(tp_m * 1e3, 3), "batched_ms": round(tb_m * 1e3, 3),
           "autotuned_ms": round(tuned_ms, 3), "launch_shape": shape,
           "identical_sizes": psz == list(nb),
           "mean_abs_dpsnr": round(float(np.mean(np.abs(dps))), 4),
           "meet_rate": round(float(np.mean([d >= 0 for d in dps])), 4), "n_over_eb": int(over),
           "closed_loop": {"mean_abs_dpsnr": round(float(np.mean(np.abs(dps_c))), 5),
                           "max_abs_dpsnr": round(float(np.max(np.abs(dps_c))), 5),
                           "meet_rate": round(float(np.mean([d >= 0 for d in dps_c])), 4)},
           "plain_max_abs_dpsnr": round(float(np.max(np.abs(dps))), 5)}
    del xs, blobs, ws, pblob, dws, out
    torch.cuda.empty_cache()
    return res


def served_leg(ctx, dev, n_req, rates):
    """Seeded request trace (Poisson arrivals, 70 % compress / 30 % decompress,
    lognormal sizes median 16 MiB in [1 MiB, 2 GiB], 1D/2D/3D, targets
    U[40,120] dB) replayed in real time through the server and through
    one-at-a-time plain calls, at each arrival rate (the same requests, the
    arrival times scaled)."""
    import torch

    from paper_1805_07384_amd import serving, synth

    trace = synth.serve_trace(n_req=n_req, rate=rates[0], seed=4)
    progress("served leg: building %d requests" % n_req)
    work = serving.build_workload(trace, device=dev, pool_size=64, ctx=ctx, log=progress)
    out = {"workload": "%d requests, Poisson arrivals, 70/30 compress/decompress, lognormal size "
                       "median 16 MiB [1 MiB, 2 GiB], 1D/2D/3D GRF k^-3, target U[40,120] dB, "
                       "seed 4; budget 64 GiB, 4 streams, 64 slots" % n_req, "rates": {}}
    for rate in rates:
        w_r = [dict(w, t=w["t"] * rates[0] / rate) for w in work]
        progress("served leg: plain replay at %g/s" % rate)
        plain, ps = serving.replay_plain(ctx, w_r, device=dev)
        progress("served leg: served replay at %g/s" % rate)
        served, ss = serving.replay_served(ctx, w_r, hbm_budget=64 << 30, arena_bytes=24 << 30,
                                           max_inflight=64, n_streams=4, device=dev)
        progress("served leg: comparing results")
        diff = serving.same_results(plain, served)
        rnd = lambda d: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
        out["rates"]["%g" % rate] = {
            "plain": rnd({**ps["latency"], "gbps": ps["gbps"], "span_s": ps["span_s"]}),
            "served": rnd({**ss["latency"], "gbps": ss["gbps"], "span_s": ss["span_s"]}),
            "results_differing": diff,
            "plain_failed": sum(1 for o in plain if o[0] != 0),
            "server": {k: ss["server"][k] for k in ("rounds", "batched_launches", "peak_inflight",
                                                    "peak_held_bytes", "failed")}}
        del plain, served, w_r
        torch.cuda.empty_cache()
    del work
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); multi-GPU sharding "
              "is a design note, not an implementation." % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1805_07384_amd import fpsz, synth

    psnrs = [float(p) for p in args.psnrs.split(",")]
    domain = fpsz.GLOBAL if args.domain == "global" else fpsz.TILE
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shape = (args.edge, args.edge, args.edge)
    x = synth.field_3d_lognormal(shape=shape, seed=args.seed, backend="torch", device=dev)
    x = x.contiguous()
    n = x.numel()
    s = x.element_size()
    ctx = fpsz.Context(0)
    if not args.no_profile:
        ctx.set_profiling(True)
    ws_c = torch.empty(fpsz.compress_workspace_bytes(shape, x.dtype), dtype=torch.uint8, device=dev)
    ws_d = torch.empty(fpsz.decompress_workspace_bytes(shape, x.dtype), dtype=torch.uint8, device=dev)
    ws_v = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    cap = n * s + (64 << 20)
    blob = torch.empty(cap, dtype=torch.uint8, device=dev)
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def one_step(rec):
        for p in psnrs:
            t0 = time.perf_counter()
            st, nb, info = ctx.compress_into(x, p, ws_c, blob, domain, stream)
            t1 = time.perf_counter()
            if st != fpsz.OK:
                raise fpsz.FpszError(st, "compress at %g dB" % p)
            stages_c = ctx.stage_times()
            if args.separate_verify:
                st = ctx.decompress_into(blob, nb, ws_d, out, stream)
                t2 = time.perf_counter()
                if st != fpsz.OK:
                    raise fpsz.FpszError(st, "decompress at %g dB" % p)
                stages_d = ctx.stage_times()
                st, stats = ctx.verify_into(x, out, info.vr, info.eb, ws_v, stream)
                t3 = time.perf_counter()
                if st != fpsz.OK:
                    raise fpsz.FpszError(st, "verify at %g dB" % p)
                stages_v = ctx.stage_times()
            else:
                # one pass: decompress and take the Eq. 4 statistics of each tile
                # against the original as it is written
                st, stats = ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream)
                t2 = t3 = time.perf_counter()
                if st != fpsz.OK:
                    raise fpsz.FpszError(st, "decompress + verify at %g dB" % p)
                stages_d = ctx.stage_times()
                stages_v = []
            if rec is not None:
                r = rec.setdefault(p, {"c": [], "d": [], "v": [], "stages": {}, "info": None,
                                       "stats": None})
                r["c"].append(t1 - t0)
                r["d"].append(t2 - t1)
                r["v"].append(t3 - t2)
                r["info"] = info.as_dict()
                r["stats"] = stats.as_dict()
                for nm, ms in stages_c + stages_d + stages_v:
                    r["stages"].setdefault(nm, []).append(ms)

    progress("sweep: warm-up")
    for _ in range(args.warmup):
        one_step(None)
    progress("sweep: timed steps")
    rec = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.copy_calibration:
        out.copy_(x)
        torch.cuda.synchronize()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    # decompression alone (no check), per target, outside the timed steps
    dec_only = {}
    if not args.separate_verify:
        progress("decompress-only timing")
        for p in psnrs:
            st, nb, _ = ctx.compress_into(x, p, ws_c, blob, domain, stream)
            dec_only[p] = timed_calls(lambda: ctx.decompress_into(blob, nb, ws_d, out, stream),
                                      5, warm=1)[0]
    copy_gbps = device_copy_gbps(x)
    # the same sweep in the other Lorenzo domain (blob size and speed)
    other = "global" if args.domain == "tile" else "tile"
    other_leg = []
    for p in ([] if args.no_other_domain else psnrs):
        if p == psnrs[0]:
            progress("%s-domain legs" % other)
        od = fpsz.GLOBAL if other == "global" else fpsz.TILE
        st, nb, io = ctx.compress_into(x, p, ws_c, blob, od, stream)
        if st != fpsz.OK:
            raise fpsz.FpszError(st, "%s domain at %g dB" % (other, p))
        tco = timed_calls(lambda: ctx.compress_into(x, p, ws_c, blob, od, stream), 3, warm=1)[0]
        tdo = timed_calls(lambda: ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream), 3,
                          warm=1)[0]
        st, sto = ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream)
        other_leg.append({"psnr": p, "dpsnr": round(sto.psnr - p, 5),
                          "bits_per_value": round(io.bits_per_value, 4),
                          "compress_gbps": round(n * s / tco / 1e9, 2),
                          "decompress_check_gbps": round(n * s / tdo / 1e9, 2),
                          "n_over_eb": sto.n_over_eb,
                          "op_frac": op_fracs(n, s, io.bits_per_value, tco, None, tdo)})
    # the closed-loop correction on the benchmark field at each target
    closed, inloop, xform = [], [], []
    for p in ([] if args.no_variants else psnrs):
        if p == psnrs[0]:
            progress("closed-loop legs")
        st, nb, ic = ctx.compress_closed_loop_into(x, p, ws_c, blob, domain, stream)
        if st != fpsz.OK:
            raise fpsz.FpszError(st, "closed loop at %g dB" % p)
        tcl = timed_calls(lambda: ctx.compress_closed_loop_into(x, p, ws_c, blob, domain, stream),
                          3, warm=1)[0]
        st, stc = ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream)
        closed.append({"psnr": p, "dpsnr": round(stc.psnr - p, 5), "eb_scale": ic.eb_scale,
                       "bits_per_value": round(ic.bits_per_value, 4),
                       "compress_gbps": round(n * s / tcl / 1e9, 2), "n_over_eb": stc.n_over_eb})
    # the SZ 1.4-style in-loop variant (tile domain) on the same field
    for p in ([] if args.no_variants else psnrs):
        if p == psnrs[0]:
            progress("in-loop legs")
        st, nb, ii = ctx.compress_inloop_into(x, p, ws_c, blob, stream)
        if st != fpsz.OK:
            raise fpsz.FpszError(st, "in-loop at %g dB" % p)
        til = timed_calls(lambda: ctx.compress_inloop_into(x, p, ws_c, blob, stream), 3, warm=1)[0]
        tdl = timed_calls(lambda: ctx.decompress_into(blob, nb, ws_d, out, stream), 3, warm=1)[0]
        st, sti = ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream)
        inloop.append({"psnr": p, "dpsnr": round(sti.psnr - p, 5),
                       "bits_per_value": round(ii.bits_per_value, 4), "n_stored": ii.n_patches,
                       "compress_gbps": round(n * s / til / 1e9, 2),
                       "decompress_gbps": round(n * s / tdl / 1e9, 2), "n_over_eb": sti.n_over_eb,
                       "op_frac": op_fracs(n, s, ii.bits_per_value, til, tdl)})
    # the orthogonal-transform variant (Theorem 3) on the same field
    for p in ([] if args.no_variants else psnrs):
        if p == psnrs[0]:
            progress("transform legs")
        st, nb, ix = ctx.compress_xform_into(x, p, ws_c, blob, stream)
        if st != fpsz.OK:
            raise fpsz.FpszError(st, "transform at %g dB" % p)
        txf = timed_calls(lambda: ctx.compress_xform_into(x, p, ws_c, blob, stream), 3, warm=1)[0]
        tdx = timed_calls(lambda: ctx.decompress_into(blob, nb, ws_d, out, stream), 3, warm=1)[0]
        st, stx = ctx.decompress_verify_into(blob, nb, ws_d, out, x, stream)
        xform.append({"psnr": p, "dpsnr": round(stx.psnr - p, 5),
                      "bits_per_value": round(ix.bits_per_value, 4), "n_outliers": ix.n_outliers,
                      "compress_gbps": round(n * s / txf / 1e9, 2),
                      "decompress_gbps": round(n * s / tdx / 1e9, 2),
                      "op_frac": op_fracs(n, s, ix.bits_per_value, txf, tdx)})
    total_bytes = n * s * len(psnrs)
    value = total_bytes / ((t1 - t0) / args.steps) / 1e9

    per_target = []
    kernel_ms = {}
    for p in psnrs:
        r = rec[p]
        c = float(np.median(r["c"]))
        d = float(np.median(r["d"]))
        v = float(np.median(r["v"]))
        info, stats = r["info"], r["stats"]
        stage_avg = {nm: round(float(np.mean(v)), 4) for nm, v in r["stages"].items()}
        if args.separate_verify:
            fr = op_fracs(n, s, info["bits_per_value"], c, d)
        else:
            fr = op_fracs(n, s, info["bits_per_value"], c, dec_only[p], d)
        per_target.append({
            "psnr": p, "achieved_psnr": round(stats["psnr"], 4),
            "dpsnr": round(stats["psnr"] - p, 4), "bits_per_value": round(info["bits_per_value"], 4),
            "compress_gbps": round(n * s / c / 1e9, 2), "decompress_gbps": round(n * s / d / 1e9, 2),
            "verify_gbps": round(n * s / v / 1e9, 2) if v > 0 else None,
            "n_outliers": info["n_outliers"], "n_patches": info["n_patches"],
            "max_abs_err_over_eb": stats["max_abs_err"] / info["eb"], "n_over_eb": stats["n_over_eb"],
            "op_frac": fr,
            "decompress_only_gbps": round(n * s / dec_only[p] / 1e9, 2) if p in dec_only else None,
            "kernel_ms": stage_avg,
        })
        for nm, ms_list in r["stages"].items():
            kernel_ms.setdefault(nm, []).append((float(np.mean(ms_list)), p, info["bits_per_value"]))

    roofline = None
    kernels = {}
    fused = not args.separate_verify
    if kernel_ms:
        # per-kernel average over the sweep: achieved algorithmic GB/s
        for nm, lst in kernel_ms.items():
            ms = float(np.mean([a for a, _, _ in lst]))
            alg = [algorithmic_bytes(nm, n, s, b, fused) for _, _, b in lst]
            entry = {"ms": round(ms, 5)}
            if alg[0] is not None:
                gbps = float(np.mean([a / (m * 1e-3) / 1e9 for a, (m, _, _) in zip(alg, lst)]))
                entry["alg_gbps"] = round(gbps, 1)
                entry["frac"] = round(gbps / HBM_PEAK_GBPS, 4)
            kernels[nm] = entry
        timed = {k: v for k, v in kernels.items() if "alg_gbps" in v}
        dom = max(timed, key=lambda k: timed[k]["ms"])
        tr = measured_traffic(args.domain) if shape == (512, 512, 512) else {}
        roofline = {"bound": "hbm", "kernel": dom, "achieved": timed[dom]["alg_gbps"],
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": timed[dom]["frac"],
                    "traffic": tr.get(dom),
                    "algorithmic_bytes_per_launch": round(float(np.mean(
                        [algorithmic_bytes(dom, n, s, b, fused) for _, _, b in kernel_ms[dom]])))}
        for k, v in tr.items():
            if k in kernels:
                kernels[k]["traffic"] = v
    # whole operations against the HBM peak and against the measured copy
    op_level = {}
    for key in ("compress", "decompress", "decompress_check"):
        vals = [t["op_frac"][key] for t in per_target if key in t["op_frac"]]
        if vals:
            op_level[key] = {"mean_frac": round(float(np.mean(vals)), 4),
                             "per_target": vals,
                             "mean_frac_of_copy": round(float(np.mean(vals)) * HBM_PEAK_GBPS / copy_gbps, 4)}
    alg_step = 0.0
    for t in per_target:
        b8 = t["bits_per_value"] / 8.0
        alg_step += (2 * s + b8) * n + ((b8 + s) * n if args.separate_verify else (b8 + 2 * s) * n)
        if args.separate_verify:
            alg_step += 2 * s * n
    step_frac = alg_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS

    line = {
        "metric": "compress+decompress+verify GB/s at target PSNR (sweep), |dPSNR| dB",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D float32 %dx%dx%d lognormal(0,1) field exp(GRF k^-11/3), seed %d, "
                               "targets %s dB, %s Lorenzo domain"
                               % (args.edge, args.edge, args.edge, args.seed,
                                  "/".join("%g" % p for p in psnrs), args.domain),
                   "shape": list(shape), "psnrs": psnrs, "domain": args.domain,
                   "verify": "separate" if args.separate_verify else "in the decompression pass"},
        "mean_abs_dpsnr": round(float(np.mean([abs(t["dpsnr"]) for t in per_target])), 4),
        "per_target": per_target,
        "closed_loop": closed,
        "other_domain": {"domain": other, "per_target": other_leg},
        "inloop": inloop,
        "xform": xform,
        "op_roofline": {"peak_gbps": HBM_PEAK_GBPS, "device_copy_gbps": round(copy_gbps, 1),
                        "step_frac": round(step_frac, 4),
                        "step_frac_of_copy": round(step_frac * HBM_PEAK_GBPS / copy_gbps, 4),
                        **op_level},
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        planes = min(args.cpu_planes, args.edge)
        line["cpu_baseline"] = cpu_baseline(x.cpu().numpy(), psnrs, planes, int(domain))
    del ws_c, ws_d, blob, out
    if not args.no_c1:
        progress("512x512 latency leg")
        line["c1_512x512"] = c1_leg(ctx, dev, domain)
    if not args.no_c5:
        progress("1024^3 float64 leg")
        del x
        torch.cuda.empty_cache()
        line["c5_1024cube_f64"] = c5_leg(ctx, dev, domain)
    if not args.no_batched:
        line["batched"] = batched_leg(ctx, dev)
    if not args.no_served:
        rates = [float(r) for r in args.served_rates.split(",")]
        line["served"] = served_leg(ctx, dev, args.served_requests, rates)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
