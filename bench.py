#!/usr/bin/env python3
"""Benchmark: homomorphic analytics on a compressed 512^3 binary32 field on one
MI355X, against full decompression + the same operations on the same GPU.

Workload (the large-field configuration): a 512^3 binary32 field (64
Gaussian bumps, sigma 8..64 cells, times a log-normal(0, 0.1) texture,
seed 0), compressed on the GPU with a value-range relative bound (default
1e-4) and blocks of S = 32.  A timed STEP is one pass of the analytics over
one compressed copy of the field, straight from the compressed bytes:
  mean      fused decode + block sums through the decorrelated stage (D_p)
  variance  fused decode + exact sum q, sum q^2 through D_q
  gradient  magnitude of the central-difference gradient, through D_q
The reported value is GB/s of ORIGINAL data (n * 4 bytes per step / step
time).  Inputs are resident in HBM before timing; the step rotates over
several distinct copies of the compressed stream (together well above the
256 MB last-level cache) so repeated steps cannot be served from cache.

Also measured on the same GPU and reported beside it: the full-decompress
baseline (decode to floats, then the same three operations on the floats),
every stage of partial decompression, every operation on every
materialised stage, compression, the same step at the large field's other
configurations (rel eb 1e-4 and 1e-2, S = 32 and 64; each with its
roofline), the plan both enqueued directly and replayed as a HIP graph, the
secondary workloads (vector field, block-mean streams, HSZp-nd, out-of-core
slabs, batches, serving), each over three copies of its inputs in turn, and
the CPU checker (oracle) timed on a bounded slab of the same field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--shape", type=str, default="512,512,512")
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--cpu-planes", type=int, default=256, help="slab of the field the CPU checker is timed on")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the per-stage table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain streaming kernel of known traffic (512 MiB in, 512 MiB out) "
                         "to scale memory counters under rocprofv3")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workloads")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-vector", action="store_true", help="skip the vector-field (divergence, curl) workload")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^3 latency workload")
    ap.add_argument("--no-hszx", action="store_true", help="skip the block-mean (HSZx) workload")
    ap.add_argument("--no-lorenzo", action="store_true", help="skip the HSZp-nd (Lorenzo) workload")
    ap.add_argument("--no-ooc", action="store_true", help="skip the out-of-core (host-resident slabs) workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other eb / block-size configurations of the large field")
    ap.add_argument("--no-tune", action="store_true", help="time the step with the default launch shape")
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--queries", type=int, default=20000)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--traffic", type=float, default=None,
                    help="HBM bytes per launch of the dominant kernel from counters (reported as roofline.traffic)")
    a = ap.parse_args()
    a.tune = None
    return a


def log(msg):
    print(msg, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "k_batch_gradmag_q8_512cube_counters.txt")
KTRACE = os.path.join(ROOT, "profiles", "k_batch_gradmag_q8_512cube_kernel_trace.txt")
KERNEL_SOURCES = ("grad4.hip", "hsz_device.hpp", "hsz_launch.hpp", "batch.cpp")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_25206_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _record(path, tag):
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith(tag + ":"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("source_sha") == kernel_source_sha():
                return rec
    return None


def counter_record():
    """The committed counter summary of the step's gradient kernel, or None
    when there is none or the kernel sources changed since it was taken."""
    return _record(COUNTERS, "TRAFFIC_JSON")


def ktrace_record():
    """The committed kernel-trace summary of the step (the gradient kernel's
    own average duration under rocprofv3), or None when there is none or the
    kernel sources changed since it was taken."""
    return _record(KTRACE, "KTRACE_JSON")


def counter_traffic():
    """HBM bytes per launch of the step's gradient kernel (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the same counter reads for a streaming
    kernel of known size), or None."""
    rec = counter_record()
    return int(rec["bytes_per_launch"]) if rec else None


VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.3 T 32-bit lane operations per second


def counter_valu(launch_ms):
    """VALU work of the step's gradient kernel from the committed SQ_INSTS_VALU
    count (wave instructions per launch, 64 lanes each), as a rate over the
    measured launch time against the chip's 32-bit VALU peak, or None."""
    rec = counter_record()
    if not rec or "valu_insts" not in rec:
        return None
    ops = float(rec["valu_insts"]) * 64
    tops = ops / (launch_ms * 1e-3) / 1e12
    return {"lane_ops_per_launch": int(ops), "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 1),
            "unit": "T lane-ops/s", "frac": round(tops / VALU_PEAK_TOPS, 4)}


def grad_kernel_label(h, block, tune):
    """Name of the batched gradient kernel a plan of the step runs for this
    stream and launch shape (informational)."""
    tile_x = int((tune or {}).get("grad_tile_x", 0))
    acc = 1 if h.max_abs_q < 65536 else 2
    if block == 32 and h.max_abs_q < 8192 and tile_x >= 0:
        # the 512-column tile with the statistics inside finishes the plan's pass itself
        return "k_batch_gradmag_q8_tail" if tile_x != 256 else "k_batch_gradmag_q4<32,256,1>"
    return f"k_batch_grad<{block},3,4,float,{acc}>"


def measure_config(a, xg, eb, block, full, tune=None):
    """One configuration of the large field: the step (one batched pass of
    mean via D_p + variance via D_q + gradient magnitude via D_q), the three
    operations launched separately, full decompression + the same operations,
    and (full) the table of every stage and every operation on every stage.
    Compressed inputs rotate over a.copies copies and materialised stages
    over three buffers (3 x 512 MiB per stage), so no row is timed on bytes
    left in the last-level caches by the previous launch."""
    import torch

    from paper_2603_25206_amd import hsz

    dev = xg.device
    n = xg.numel()
    orig_bytes = n * xg.element_size()
    c0 = hsz.compress(xg, eb, rel=True, block=block)
    h = c0.header
    copies = [c0] + [hsz.Compressed(c0.data.clone(), h) for _ in range(a.copies - 1)]
    torch.cuda.synchronize()
    log(f"[bench] eb {eb:g} S {block}: {c0.nbytes / 2**20:.1f} MiB, ratio {c0.ratio:.2f}, max|q| {h.max_abs_q}")
    nc, R = len(copies), 3
    stream = torch.cuda.current_stream()
    S48 = [torch.empty(64, dtype=torch.uint8, device=dev) for _ in range(3)]
    gbuf = torch.empty(n * 4, dtype=torch.uint8, device=dev)
    qbufs = [torch.empty(n * 4, dtype=torch.uint8, device=dev) for _ in range(R)]
    fbufs = [torch.empty(n * 4 + 64, dtype=torch.uint8, device=dev) for _ in range(R)]
    dbufs = [torch.empty(4 * (n + h.nb) + 64, dtype=torch.uint8, device=dev) for _ in range(R)] if full else []
    ws_bytes = max(hsz.op_workspace_bytes(h, op) for op in (hsz.MEAN, hsz.VAR, hsz.GRADMAG, hsz.LAPLACIAN))
    ws = [hsz.workspace(ws_bytes, dev, key=f"bench{k}") for k in range(3)]

    def C(k):
        return copies[k % nc]

    def timed(fns, steps, warmup):
        """Run the list of (label, fn(k)) for steps k; per-label HIP event times."""
        for k in range(warmup):
            for _, fn in fns:
                fn(k)
        torch.cuda.synchronize()
        evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in fns]
               for _ in range(steps)]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for k in range(steps):
            for j, (_, fn) in enumerate(fns):
                evs[k][j][0].record(stream)
                fn(k)
                evs[k][j][1].record(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        per = {lab: float(np.mean([evs[k][j][0].elapsed_time(evs[k][j][1]) for k in range(steps)]))
               for j, (lab, _) in enumerate(fns)}
        return start.elapsed_time(stop) / steps, per

    # ---- the three operations launched one by one -------------------------------------
    def f_mean(k):
        hsz.op_fused(C(k), hsz.DELTA, hsz.MEAN, out=S48[0], ws=ws[0], check=False, raw=True)

    def f_var(k):
        hsz.op_fused(C(k), hsz.QUANT, hsz.VAR, out=S48[1], ws=ws[1], check=False, raw=True)

    def f_grad(k):
        hsz.op_fused(C(k), hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws[2], check=False, raw=True)

    sep_fns = [("mean_fused_delta", f_mean), ("var_fused_quant", f_var), ("gradmag_quant", f_grad)]
    ms_sep, per_sep = timed(sep_fns, a.steps, a.warmup)
    st_v, st_m = hsz.stats_of(S48[1]), hsz.stats_of(S48[0])

    # ---- the step: one batched pass, the three analytics sharing one decode -------------
    # Per copy, a plan of three jobs over the whole field; mean and variance
    # are summed inside the gradient tiles.  Block indexes are built once per
    # stream, as a resident stream keeps them.
    for c in copies:
        c.build_index()

    def jobs_of(c):
        return [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
    if tune is None and not a.no_tune:
        # the autotuner times each candidate over all the copies in turn and
        # rejects any that changes a result
        from paper_2603_25206_amd import tune as tuner
        tune, _ = tuner.tune(jobs_of(copies[0]), reps=3, cache_path=None,
                             alternates=[jobs_of(c) for c in copies[1:]])
        log(f"[bench] eb {eb:g} S {block}: launch shape (autotuned) {tune}")
    step_stream = torch.cuda.Stream()
    plans = [hsz.Plan(jobs_of(c), tune=tune, stream=step_stream) for c in copies]

    def step_times(pl, steps, warmup):
        for k in range(warmup):
            pl[k % len(pl)].launch()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(step_stream)
        for k in range(steps):
            evs[k][0].record(step_stream)
            pl[k % len(pl)].launch()
            evs[k][1].record(step_stream)
        stop.record(step_stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))

    ms_step, ms_replay = step_times(plans, a.steps, a.warmup)
    res = plans[0].results()
    if (res[1]["s1"], res[1]["s2"], res[1]["var"]) != (st_v["s1"], st_v["s2"], st_v["var"]) or \
            res[0]["mean"] != st_m["mean"] or not torch.equal(res[2].reshape(-1), gbuf.view(torch.float32)):
        raise RuntimeError("batched step disagrees with the separate operations")
    for pl in plans:
        pl.close()
    # the same plans replaying the HIP graph captured at creation
    gtune = dict(tune or {}, graph_replay=1)
    gplans = [hsz.Plan(jobs_of(c), tune=gtune, stream=step_stream) for c in copies]
    ms_graph, _ = step_times(gplans, max(5, a.steps // 2), 2)
    gres = gplans[0].results()
    if not torch.equal(gres[2], res[2]) or gres[1]["s2"] != res[1]["s2"]:
        raise RuntimeError("graph replay disagrees with direct launch")
    for pl in gplans:
        pl.close()

    # ---- baseline: full decompression + the same ops on floats ------------------------
    fviews = [hsz.stage_view(b, h, hsz.FLOAT) for b in fbufs]

    def b_dec(k):
        hsz.decompress_to_stage(C(k), hsz.FLOAT, out=fbufs[k % R])

    def b_op(op, out, w):
        return lambda k: hsz.op_on_stage(fviews[k % R], h, hsz.FLOAT, op, out=out, ws=w, check=False, raw=True)

    base_fns = [("decompress_float", b_dec), ("mean_float", b_op(hsz.MEAN, S48[0], ws[0])),
                ("var_float", b_op(hsz.VAR, S48[1], ws[1])), ("gradmag_float", b_op(hsz.GRADMAG, gbuf, ws[2]))]
    ms_base, per_base = timed(base_fns, max(5, a.steps // 2), 2)
    st_bv = hsz.stats_of(S48[1])

    # ---- per-stage table ------------------------------------------------------------
    extra = {}
    if full:
        def dec(stage, bufs):
            return lambda k: hsz.decompress_to_stage(C(k), stage, out=bufs[k % R])
        _, per = timed([("decompress_delta", dec(hsz.DELTA, dbufs)), ("decompress_quant", dec(hsz.QUANT, qbufs)),
                        ("decompress_float", dec(hsz.FLOAT, fbufs))], 6, 2)
        extra.update(per)
        views = {"delta": (hsz.DELTA, [hsz.stage_view(b, h, hsz.DELTA) for b in dbufs]),
                 "quant": (hsz.QUANT, [hsz.stage_view(b, h, hsz.QUANT) for b in qbufs]),
                 "float": (hsz.FLOAT, fviews)}

        def on(stn, op, out):
            st, vs = views[stn]
            return lambda k: hsz.op_on_stage(vs[k % R], h, st, op, out=out, ws=ws[2], check=False, raw=True)

        def fu(st, op, out):
            return lambda k: hsz.op_fused(C(k), st, op, out=out, ws=ws[2], check=False, raw=True)
        rows = []
        for stn, st in (("delta", hsz.DELTA), ("quant", hsz.QUANT), ("float", hsz.FLOAT)):
            for opn, op in (("mean", hsz.MEAN), ("var", hsz.VAR)):
                rows += [(f"{opn}_on_{stn}", on(stn, op, S48[2])), (f"{opn}_fused_{stn}", fu(st, op, S48[2]))]
        for stn, st in (("quant", hsz.QUANT), ("float", hsz.FLOAT)):
            rows += [(f"gradmag_on_{stn}", on(stn, hsz.GRADMAG, gbuf)),
                     (f"laplacian_on_{stn}", on(stn, hsz.LAPLACIAN, gbuf)),
                     (f"laplacian_fused_{stn}", fu(st, hsz.LAPLACIAN, gbuf))]
        _, per = timed(rows, 6, 2)
        extra.update(per)
        cbuf = torch.empty_like(c0.data)

        def comp(k):
            hsz.compress(xg, eb, rel=True, block=block, out=cbuf, check=False)
        _, per = timed([("compress", comp)], 4, 1)
        extra.update(per)

    # ---- roofline of the step's dominant kernel ---------------------------------------
    # Its algorithmic bytes: the compressed stream read once plus the f32
    # magnitude written (the sums add none, the avoided floats are never
    # counted).  Its duration here is the HIP-event time of one plan launch,
    # which also holds the reset and finalize kernels and the gaps between
    # them: 'frac' is a lower bound on the kernel's own fraction.
    cbytes = c0.nbytes
    alg_step = cbytes + 4 * n
    achieved = alg_step / (ms_replay * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": grad_kernel_label(h, block, tune) + " (mean+var+gradmag, one decode)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(alg_step),
                "launch_ms": round(ms_replay, 4)}
    ach_sep = alg_step / (per_sep["gradmag_quant"] * 1e-3) / 1e9
    roofline_sep = {"bound": "hbm", "kernel": "gradient magnitude alone (op_fused)",
                    "achieved": round(ach_sep, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach_sep / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(alg_step),
                    "launch_ms": round(per_sep["gradmag_quant"], 4)}
    row = {
        "eb": eb, "block": block, "ratio": round(c0.ratio, 3), "compressed_bytes": cbytes,
        "max_abs_q": int(h.max_abs_q), "copies": nc,
        "ms_per_step": round(ms_step, 4), "gbs_orig": round(orig_bytes / (ms_step * 1e-3) / 1e9, 1),
        "plan_ms_direct": round(ms_replay, 4), "plan_ms_graph_replay": round(ms_graph, 4),
        "launch_shape": tune, "roofline": roofline,
        "separate_ops": {"gbs_orig": round(orig_bytes / (ms_sep * 1e-3) / 1e9, 1), "ms_per_step": round(ms_sep, 4),
                         "per_op_ms": {k: round(v, 4) for k, v in per_sep.items()}, "roofline": roofline_sep},
        "full_decompress_baseline": {"gbs_orig": round(orig_bytes / (ms_base * 1e-3) / 1e9, 1),
                                     "ms_per_step": round(ms_base, 4),
                                     "per_op_ms": {k: round(v, 4) for k, v in per_base.items()},
                                     "speedup_homomorphic": round(ms_base / ms_step, 3),
                                     "speedup_separate_ops": round(ms_base / ms_sep, 3)},
        "check": {"var_int_route": st_v["var"], "var_float_route": st_bv["var"], "mean": st_m["mean"]},
    }
    if full:
        row["stage_table_ms"] = {k: round(v, 4) for k, v in extra.items()}
    log(f"[bench] eb {eb:g} S {block}: step {ms_step:.4f} ms (plan {ms_replay:.4f} direct, {ms_graph:.4f} graph), "
        f"separate {ms_sep:.4f}, full-decompress {ms_base:.4f}, frac {roofline['frac']}")
    del copies, plans, gplans, gbuf, qbufs, fbufs, dbufs, ws, S48
    torch.cuda.empty_cache()
    return row, h


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2603_25206_amd import hsz, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shape = tuple(int(v) for v in a.shape.split(","))
    spec = synth.large_field_spec(seed=0, shape=shape)
    t0 = time.time()
    x = synth.make_field(spec)
    log(f"[bench] field {shape} generated in {time.time() - t0:.1f}s")
    n = x.size
    orig_bytes = x.nbytes
    xg = torch.from_numpy(x).to(dev)

    main_row, h = measure_config(a, xg, a.eb, a.block, full=not a.no_extra, tune=a.tune)
    if a.calibrate_copy:
        # a plain streaming kernel of known traffic for scaling memory counters:
        # bitwise NOT of 2^27 int32 reads 512 MiB and writes 512 MiB
        src = torch.zeros(2**27, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    roofline = dict(main_row["roofline"])
    roofline["traffic"] = a.traffic if a.traffic is not None else counter_traffic()
    roofline["valu"] = counter_valu(main_row["plan_ms_direct"])
    kt = ktrace_record()
    if kt is not None and kt.get("kernel", "") in roofline["kernel"]:
        own = roofline["alg_bytes_per_launch"] / (kt["avg_us"] * 1e-6) / 1e9
        roofline["frac_kernel"] = round(own / HBM_PEAK_GBS, 4)
        roofline["kernel_avg_us_profiled"] = kt["avg_us"]
    else:
        roofline["frac_kernel"] = None

    ms_step = main_row["ms_per_step"]
    value = orig_bytes / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "GB/s (orig. data) homomorphic op vs full-decompress+op at eb; p50/p99 query ms",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, shape))} f32 gaussian-mixture x lognormal texture, "
                               f"rel eb {a.eb:g}, S={a.block}; step = mean + var + gradmag(D_q) from the "
                               f"compressed bytes, one batched pass (one plan launch): the mean (asked via D_p) "
                               f"and the variance (via D_q) are the exact integer sums of q taken in the "
                               f"gradient's decode (sum of the D_p weighted deltas = sum q)",
                   "global_batch": 1, "field_bytes": orig_bytes, "compressed_bytes": main_row["compressed_bytes"],
                   "ratio": main_row["ratio"], "parallelism": "single-gpu"},
        "separate_ops": main_row["separate_ops"],
        "full_decompress_baseline": main_row["full_decompress_baseline"],
        "stage_table_ms": main_row.get("stage_table_ms", {}),
        "step_launch_shape": main_row["launch_shape"],
        "plan_ms_direct": main_row["plan_ms_direct"],
        "plan_ms_graph_replay": main_row["plan_ms_graph_replay"],
        "roofline": roofline,
        "check": main_row["check"],
    }
    if not a.no_configs:
        rows = []
        for eb, block in ((1e-4, 32), (1e-4, 64), (1e-2, 32), (1e-2, 64)):
            if (eb, block) == (a.eb, a.block):
                continue
            r, _ = measure_config(a, xg, eb, block, full=False)
            rows.append(r)
        out["large_field_configs"] = rows
    del xg
    torch.cuda.empty_cache()
    if not a.no_small:
        out["small_field"] = bench_small(a, log)
    if not a.no_vector:
        out["vector_field"] = bench_vector(a, log)
        torch.cuda.empty_cache()
    if not a.no_hszx:
        out["block_mean"] = bench_hszx(a, log)
        torch.cuda.empty_cache()
    if not a.no_lorenzo:
        out["lorenzo_nd"] = bench_lorenzo(a, log)
        torch.cuda.empty_cache()
    if not a.no_ooc:
        out["out_of_core"] = bench_ooc(a, log)
        torch.cuda.empty_cache()
    if not a.no_batch:
        out["batching"] = bench_batches(a, log)
        torch.cuda.empty_cache()
    if not a.no_serve:
        out["serving"] = bench_serving(a, log)
        torch.cuda.empty_cache()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, x, a)
    print(json.dumps(out), flush=True)


def _events_ms(fn, reps, stream):
    """Median HIP-event time of one call; fn is a callable or a list of
    callables (the same work over distinct copies of its inputs), called in
    turn so that no timed call reads bytes the previous one left in cache."""
    import torch
    fns = fn if isinstance(fn, (list, tuple)) else [fn]
    for f in fns:
        f()
    torch.cuda.synchronize()
    ts = []
    for r in range(max(reps, len(fns))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fns[r % len(fns)]()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


ROT = 3  # copies of every secondary row's inputs (each >= 512 MiB for the 512^3 fields)


def _clones(c, k=ROT):
    from paper_2603_25206_amd import hsz
    return [c] + [hsz.Compressed(c.data.clone(), c.header) for _ in range(k - 1)]


def bench_vector(a, log):
    """A three-component 512^3 binary32 vector field (NYX-velocity sized; each
    component the large-field recipe with its own seed, rel eb 1e-4, S=32):
    divergence and curl straight from the three streams through D_q, on the
    materialised quantized stage, and after full decompression of every
    component (decode to floats + the operation on the floats).  Three
    copies of the streams and of the stage buffers are used in turn."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = (512, 512, 512)
    comps, orig = [], 0
    for k in range(3):
        f = synth.make_field_torch(synth.large_field_spec(seed=400 + k, shape=shape), "cuda")
        comps.append(hsz.compress(f, a.eb, rel=True, block=32))
        orig += f.numel() * f.element_size()
        del f
    torch.cuda.synchronize()
    sets = list(zip(*[_clones(c) for c in comps]))  # ROT sets of three components
    dev = comps[0].data.device
    cur = torch.cuda.current_stream()
    headers = [c.header for c in comps]
    n = comps[0].header.n
    outs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(3)]
    ws = hsz.workspace(hsz.vector_workspace_bytes(headers), dev, key="bench-vec")
    res = {"components": 3, "shape": list(shape), "orig_bytes": orig,
           "compressed_bytes": sum(c.nbytes for c in comps), "copies": ROT}
    qbufs = [[torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(3)] for _ in range(ROT)]
    fbufs = [[torch.empty(4 * n + 64, dtype=torch.uint8, device=dev) for _ in range(3)] for _ in range(ROT)]
    for op in ("divergence", "curl"):
        nout = 3 if op == "curl" else 1

        def fused(k):
            return lambda: hsz.vector_op_fused(list(sets[k]), op, outs=outs[:nout], ws=ws, check=False)

        def on_q(k):
            def f():
                for c, b in zip(sets[k], qbufs[k]):
                    hsz.decompress_to_stage(c, hsz.QUANT, out=b)
                hsz.vector_op_on_stage([b[: 4 * n] for b in qbufs[k]], headers, hsz.QUANT, op, outs=outs[:nout],
                                       ws=ws, check=False)
            return f

        def full(k):
            def f():
                for c, b in zip(sets[k], fbufs[k]):
                    hsz.decompress_to_stage(c, hsz.FLOAT, out=b)
                hsz.vector_op_on_stage(fbufs[k], headers, hsz.FLOAT, op, outs=outs[:nout], ws=ws, check=False)
            return f
        ms_f = _events_ms([fused(k) for k in range(ROT)], 6, cur)
        ms_q = _events_ms([on_q(k) for k in range(ROT)], 6, cur)
        ms_b = _events_ms([full(k) for k in range(ROT)], 6, cur)
        res[op] = {"fused_quant_ms": round(ms_f, 4), "gbs_orig": round(orig / ms_f / 1e6, 1),
                   "decompress_quant_then_op_ms": round(ms_q, 4), "full_decompress_then_op_ms": round(ms_b, 4),
                   "speedup_vs_full_decompress": round(ms_b / ms_f, 3)}
    log(f"[bench] vector field: {res}")
    del comps, sets, outs, qbufs, fbufs
    return res


def bench_small(a, log):
    """The 64^3 binary32 field (8 bumps, sigma 4-16 cells, N(0, 1e-3) noise;
    rel eb 1e-3, S=32), where every launch is latency: compression, the step
    (one plan launch: mean via D_p, variance via D_q, gradient magnitude via
    D_q), the three operations launched one by one and full decompression +
    the operations, each the median of many HIP-event-timed calls; the
    step's results are checked equal to the operations run one by one (the
    oracle comparison of this field is a parity test)."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    spec = synth.small_field_spec(seed=0)
    x = synth.make_field(spec)
    xt = torch.from_numpy(x).cuda()
    eb = 1e-3
    c = hsz.compress(xt, eb, rel=True, block=32)
    c.build_index()
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    jobs = [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
    res = {"shape": list(spec.shape), "rel_eb": eb, "block": 32, "ratio": round(c.ratio, 3)}
    res["compress_us"] = round(1e3 * _events_ms(lambda: hsz.compress(xt, eb, rel=True, block=32), 50, cur), 1)
    ps = torch.cuda.Stream()  # a plan is captured, so it runs on a stream of its own
    for graph in (False, True):
        plan = hsz.Plan(jobs, tune={"graph_replay": graph}, stream=ps)
        res["step_graph_us" if graph else "step_us"] = round(1e3 * _events_ms(plan.launch, 100, ps), 1)
        plan.launch()
        mean, var, mag = plan.results()
        plan.close()
    s48 = torch.empty(64, dtype=torch.uint8, device="cuda")
    gout = torch.empty(4 * x.size, dtype=torch.uint8, device="cuda")
    ws = hsz.workspace(hsz.op_workspace_bytes(c.header, hsz.GRADMAG), "cuda", key="bench-small")
    def ops():
        hsz.op_fused(c, hsz.DELTA, hsz.MEAN, out=s48, ws=ws, check=False, raw=True)
        hsz.op_fused(c, hsz.QUANT, hsz.VAR, out=s48, ws=ws, check=False, raw=True)
        hsz.op_fused(c, hsz.QUANT, hsz.GRADMAG, out=gout, ws=ws, check=False, raw=True)
    res["separate_ops_us"] = round(1e3 * _events_ms(ops, 100, cur), 1)
    fbuf = torch.empty(4 * x.size + 64, dtype=torch.uint8, device="cuda")
    def full():
        f = hsz.decompress_to_stage(c, hsz.FLOAT, out=fbuf)
        hsz.op_on_stage(f, c.header, hsz.FLOAT, hsz.MEAN)
        hsz.op_on_stage(f, c.header, hsz.FLOAT, hsz.VAR)
        hsz.op_on_stage(f, c.header, hsz.FLOAT, hsz.GRADMAG)
    res["full_decompress_then_ops_us"] = round(1e3 * _events_ms(full, 50, cur), 1)
    m1 = hsz.op_fused(c, hsz.DELTA, hsz.MEAN)
    v1 = hsz.op_fused(c, hsz.QUANT, hsz.VAR)
    g1 = hsz.op_fused(c, hsz.QUANT, hsz.GRADMAG)
    ok = ((mean["n"], mean["s1"]) == (m1["n"], m1["s1"]) and (var["s1"], var["s2"]) == (v1["s1"], v1["s2"])
          and torch.equal(mag, g1))
    if not ok:
        raise RuntimeError("64^3 step differs from the operations run one by one")
    log(f"[bench] 64^3 field: {res}")
    return res


def bench_hszx(a, log):
    """The step's 512^3 binary32 field compressed in both decorrelation modes
    (rel eb 1e-4, S=32): compression time and ratio, the mean from the block
    means alone (Eq. (mean_m)), the exact mean via D_p, the variance via D_q,
    the spread about the integer metadata mean via D_p (Sec. V-A),
    the gradient magnitude (fused from the delta stream; decode to D_q then
    the stencil for block-mean streams), and full decompression + the mean
    on floats.  Three copies of each stream and stage buffer are used in
    turn."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = tuple(int(v) for v in a.shape.split(","))
    x = synth.make_field_torch(synth.large_field_spec(seed=0, shape=shape), "cuda")
    dev, cur = x.device, torch.cuda.current_stream()
    orig = x.numel() * x.element_size()
    n = x.numel()
    res = {"shape": list(shape), "orig_bytes": orig, "copies": ROT}
    s48 = torch.empty(64, dtype=torch.uint8, device=dev)
    gbuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    qbufs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(ROT)]
    fbufs = [torch.empty(4 * n + 64, dtype=torch.uint8, device=dev) for _ in range(ROT)]
    for mode, mean_dec in (("delta", False), ("block_mean", True)):
        c = hsz.compress(x, a.eb, rel=True, block=a.block, mean_dec=mean_dec)
        torch.cuda.synchronize()
        cs = _clones(c)
        h = c.header
        ws = hsz.workspace(max(hsz.op_workspace_bytes(h, op) for op in (hsz.MEAN, hsz.VAR, hsz.GRADMAG)), dev,
                           key="bench-hszx")

        def comp():
            hsz.compress(x, a.eb, rel=True, block=a.block, mean_dec=mean_dec)

        def stat(via, op):
            return [lambda ck=ck: hsz.op_fused(ck, via, op, out=s48, ws=ws, check=False, raw=True) for ck in cs]

        def grad(k):
            def f():
                if mean_dec:
                    hsz.decompress_to_stage(cs[k], hsz.QUANT, out=qbufs[k])
                    hsz.op_on_stage(hsz.stage_view(qbufs[k], h, hsz.QUANT), h, hsz.QUANT, hsz.GRADMAG, out=gbuf,
                                    ws=ws, check=False, raw=True)
                else:
                    hsz.op_fused(cs[k], hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws, check=False, raw=True)
            return f

        def full_mean(k):
            def f():
                hsz.decompress_to_stage(cs[k], hsz.FLOAT, out=fbufs[k])
                hsz.op_on_stage(hsz.stage_view(fbufs[k], h, hsz.FLOAT), h, hsz.FLOAT, hsz.MEAN, out=s48, ws=ws,
                                check=False, raw=True)
            return f

        r = {"ratio": round(c.ratio, 3), "compress_ms": round(_events_ms(comp, 5, cur), 4)}
        if mean_dec:
            r["mean_meta_ms"] = round(_events_ms(stat(hsz.META, hsz.MEAN), 10, cur), 4)
            m_meta = hsz.stats_of(s48)["mean"]
        r["mean_delta_ms"] = round(_events_ms(stat(hsz.DELTA, hsz.MEAN), 10, cur), 4)
        m_exact = hsz.stats_of(s48)["mean"]
        r["var_quant_ms"] = round(_events_ms(stat(hsz.QUANT, hsz.VAR), 10, cur), 4)
        if mean_dec:
            r["var_mt_delta_ms"] = round(_events_ms(stat(hsz.DELTA, hsz.VAR_MT), 10, cur), 4)
        r["gradmag_ms"] = round(_events_ms([grad(k) for k in range(ROT)], 6, cur), 4)
        r["full_decompress_mean_ms"] = round(_events_ms([full_mean(k) for k in range(ROT)], 6, cur), 4)
        if mean_dec:
            r["mean_meta_gbs_orig"] = round(orig / r["mean_meta_ms"] / 1e6, 1)
            r["speedup_mean_meta_vs_full"] = round(r["full_decompress_mean_ms"] / r["mean_meta_ms"], 2)
            r["mean_meta_minus_exact"] = m_meta - m_exact
            if abs(m_meta - m_exact) > h.eb_abs:
                raise RuntimeError("mean from the block means is farther than eps from the exact mean")
        r["eb_abs"] = h.eb_abs
        res[mode] = r
        del c, cs, ws
    log(f"[bench] block-mean: {res}")
    del x, gbuf, qbufs, fbufs
    return res


def bench_lorenzo(a, log):
    """The step's 512^3 binary32 field as an HSZp-nd stream (rel eb 1e-4,
    S=32, 2x4x4 blocks): compression time and ratio, decoding to each stage,
    the mean with nd weights and Alg. 4 on D_p, the derivative along each
    axis on D_p (Eq. (derivative_Dp)) against the same derivative from D_q
    (decode to D_q + stencil) and after full decompression; and the same
    field as an HSZp stream (deltas across block borders of the flat field):
    ratio, compression, D_p and D_q decoding, mean and variance on D_p.
    Three copies of each stream and stage buffer are used in turn."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = tuple(int(v) for v in a.shape.split(","))
    x = synth.make_field_torch(synth.large_field_spec(seed=0, shape=shape), "cuda")
    dev, cur = x.device, torch.cuda.current_stream()
    orig = x.numel() * x.element_size()
    n = x.numel()
    c = hsz.compress(x, a.eb, rel=True, block=a.block, lorenzo=True)
    torch.cuda.synchronize()
    cs = _clones(c)
    h = c.header
    ws = hsz.workspace(hsz.op_workspace_bytes(h, hsz.DERIV), dev, key="bench-lz")
    s48 = torch.empty(64, dtype=torch.uint8, device=dev)
    obuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    sbufs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(ROT)]

    def each(f):
        return [(lambda k=k: f(k)) for k in range(ROT)]
    res = {"shape": list(shape), "orig_bytes": orig, "ratio": round(c.ratio, 3), "copies": ROT,
           "compress_ms": round(_events_ms(lambda: hsz.compress(x, a.eb, rel=True, block=a.block, lorenzo=True), 5,
                                           cur), 4)}
    for st, name in ((hsz.DELTA, "decode_p_ms"), (hsz.QUANT, "decode_q_ms"), (hsz.FLOAT, "decode_f_ms")):
        res[name] = round(_events_ms(each(lambda k: hsz.decompress_to_stage(cs[k], st, out=sbufs[k])), 6, cur), 4)
    res["mean_p_ms"] = round(_events_ms(each(lambda k: hsz.op_fused(cs[k], hsz.DELTA, hsz.MEAN, out=s48, ws=ws,
                                                                    check=False, raw=True)), 10, cur), 4)
    res["var_p_ms"] = round(_events_ms(each(lambda k: hsz.op_fused(cs[k], hsz.DELTA, hsz.VAR, out=s48, ws=ws,
                                                                   check=False, raw=True)), 10, cur), 4)
    for ax in range(len(shape)):
        r = {}
        r["via_p_ms"] = round(_events_ms(each(lambda k: hsz.op_fused(cs[k], hsz.DELTA, hsz.DERIV, axis=ax, out=obuf,
                                                                     ws=ws, check=False, raw=True)), 6, cur), 4)

        def via_q(k):
            hsz.decompress_to_stage(cs[k], hsz.QUANT, out=sbufs[k])
            hsz.op_on_stage(hsz.stage_view(sbufs[k], h, hsz.QUANT), h, hsz.QUANT, hsz.DERIV, axis=ax, out=obuf,
                            ws=ws, check=False, raw=True)

        def full(k):
            hsz.decompress_to_stage(cs[k], hsz.FLOAT, out=sbufs[k])
            hsz.op_on_stage(hsz.stage_view(sbufs[k], h, hsz.FLOAT), h, hsz.FLOAT, hsz.DERIV, axis=ax, out=obuf,
                            ws=ws, check=False, raw=True)
        r["decode_q_then_deriv_ms"] = round(_events_ms(each(via_q), 6, cur), 4)
        r["full_decompress_then_deriv_ms"] = round(_events_ms(each(full), 6, cur), 4)
        res[f"deriv_axis{ax}"] = r
    # the Laplacian: Eq. (laplacian_Dp) on D_p, the stencil on D_q, and full decompression + the float stencil
    wsl = hsz.workspace(hsz.op_workspace_bytes(h, hsz.LAPLACIAN), dev, key="bench-lz-lap")

    def lap_q(k):
        hsz.decompress_to_stage(cs[k], hsz.QUANT, out=sbufs[k])
        hsz.op_on_stage(hsz.stage_view(sbufs[k], h, hsz.QUANT), h, hsz.QUANT, hsz.LAPLACIAN, out=obuf, ws=wsl,
                        check=False, raw=True)

    def lap_f(k):
        hsz.decompress_to_stage(cs[k], hsz.FLOAT, out=sbufs[k])
        hsz.op_on_stage(hsz.stage_view(sbufs[k], h, hsz.FLOAT), h, hsz.FLOAT, hsz.LAPLACIAN, out=obuf, ws=wsl,
                        check=False, raw=True)
    res["laplacian"] = {
        "via_p_ms": round(_events_ms(each(lambda k: hsz.op_fused(cs[k], hsz.DELTA, hsz.LAPLACIAN, out=obuf, ws=wsl,
                                                                 check=False, raw=True)), 6, cur), 4),
        "decode_q_then_laplacian_ms": round(_events_ms(each(lap_q), 6, cur), 4),
        "full_decompress_then_laplacian_ms": round(_events_ms(each(lap_f), 6, cur), 4)}
    del wsl
    # HSZp: deltas across the blocks of the flat field (device-wide prefix sum for D_q)
    cf = hsz.compress(x, a.eb, rel=True, block=a.block, inter_block=True)
    torch.cuda.synchronize()
    cfs = _clones(cf)
    wsf = hsz.workspace(hsz.op_workspace_bytes(cf.header, hsz.VAR), dev, key="bench-flat")
    flat = {"ratio": round(cf.ratio, 3),
            "compress_ms": round(_events_ms(lambda: hsz.compress(x, a.eb, rel=True, block=a.block,
                                                                 inter_block=True), 5, cur), 4)}
    for st, name in ((hsz.DELTA, "decode_p_ms"), (hsz.QUANT, "decode_q_ms")):
        flat[name] = round(_events_ms(each(lambda k: hsz.decompress_to_stage(cfs[k], st, out=sbufs[k])), 6, cur), 4)
    flat["mean_p_ms"] = round(_events_ms(each(lambda k: hsz.op_fused(cfs[k], hsz.DELTA, hsz.MEAN, out=s48, ws=wsf,
                                                                     check=False, raw=True)), 10, cur), 4)
    flat["var_p_ms"] = round(_events_ms(each(lambda k: hsz.op_fused(cfs[k], hsz.DELTA, hsz.VAR, out=s48, ws=wsf,
                                                                    check=False, raw=True)), 10, cur), 4)
    res["inter_block_1d"] = flat
    log(f"[bench] lorenzo-nd / inter-block: {res}")
    del x, c, cs, cf, cfs, ws, wsf, obuf, sbufs
    torch.cuda.empty_cache()
    res["vector_field"] = bench_lorenzo_vector(a, log)
    return res


def bench_lorenzo_vector(a, log):
    """A three-component 512^3 binary32 vector field (each component the
    large-field recipe with its own seed) as HSZp-nd streams (rel eb 1e-4,
    S=32): divergence and curl on D_p (every term's numerator from its
    component's p, fused from the streams), through D_q (decode every
    component, then the stencil) and after full decompression.  Three copies
    of the streams and stage buffers are used in turn."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = (512, 512, 512)
    comps, orig = [], 0
    for k in range(3):
        f = synth.make_field_torch(synth.large_field_spec(seed=400 + k, shape=shape), "cuda")
        comps.append(hsz.compress(f, a.eb, rel=True, block=32, lorenzo=True))
        orig += f.numel() * f.element_size()
        del f
    torch.cuda.synchronize()
    sets = list(zip(*[_clones(c) for c in comps]))
    dev = comps[0].data.device
    cur = torch.cuda.current_stream()
    headers = [c.header for c in comps]
    n = comps[0].header.n
    outs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(3)]
    ws = hsz.workspace(hsz.vector_workspace_bytes(headers), dev, key="bench-lz-vec")
    bufs = [[torch.empty(4 * n + 64, dtype=torch.uint8, device=dev) for _ in range(3)] for _ in range(ROT)]
    res = {"components": 3, "shape": list(shape), "orig_bytes": orig, "compressed_bytes": sum(c.nbytes for c in comps),
           "copies": ROT}
    for op in ("divergence", "curl"):
        nout = 3 if op == "curl" else 1

        def via_p(k):
            return lambda: hsz.vector_op_fused(list(sets[k]), op, via=hsz.DELTA, outs=outs[:nout], ws=ws, check=False)

        def staged(k, st):
            def f():
                for c, b in zip(sets[k], bufs[k]):
                    hsz.decompress_to_stage(c, st, out=b)
                hsz.vector_op_on_stage([b[: 4 * n] for b in bufs[k]], headers, st, op, outs=outs[:nout], ws=ws,
                                       check=False)
            return f
        ms_p = _events_ms([via_p(k) for k in range(ROT)], 6, cur)
        ms_q = _events_ms([staged(k, hsz.QUANT) for k in range(ROT)], 6, cur)
        ms_f = _events_ms([staged(k, hsz.FLOAT) for k in range(ROT)], 6, cur)
        res[op] = {"via_p_ms": round(ms_p, 4), "decode_q_then_op_ms": round(ms_q, 4),
                   "full_decompress_then_op_ms": round(ms_f, 4), "gbs_orig_via_p": round(orig / ms_p / 1e6, 1),
                   "speedup_p_vs_full": round(ms_f / ms_p, 3), "speedup_q_vs_full": round(ms_f / ms_q, 3)}
    log(f"[bench] lorenzo-nd vector field: {res}")
    del comps, sets, outs, bufs, ws
    return res


def bench_ooc(a, log):
    """The step's 512^3 binary32 field in pinned host memory, compressed as 8
    slabs of 64 planes with the whole field's quantizer and kept on the host;
    mean, variance and gradient magnitude streamed through the device slab by
    slab (Alg. 3's window; the results equal the whole field's).  Host-device
    copies are inside every time, so these rates are bound by the link, not
    by HBM; the in-HBM step is the headline."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = tuple(int(v) for v in a.shape.split(","))
    xg = synth.make_field_torch(synth.large_field_spec(seed=0, shape=shape), "cuda")
    x = torch.empty(xg.shape, dtype=xg.dtype, pin_memory=True)
    x.copy_(xg)
    del xg
    torch.cuda.synchronize()
    orig = x.numel() * x.element_size()
    planes = max(1, shape[0] // 8)
    t0 = time.time()
    slabs = hsz.compress_slabs(x, a.eb, planes, rel=True, block=a.block)
    torch.cuda.synchronize()
    res = {"slabs": len(slabs), "planes_per_slab": planes, "orig_bytes": orig,
           "compressed_bytes": sum(int(h.total_bytes) for _, h in slabs),
           "compress_slabs_s": round(time.time() - t0, 3)}
    for op in ("mean", "var", "gradmag"):
        hsz.ooc_op(slabs, op)  # warm-up (workspace, streams)
        ts = []
        for _ in range(3):
            t1 = time.time()
            hsz.ooc_op(slabs, op)
            ts.append(time.time() - t1)
        ms = float(np.median(ts)) * 1e3
        res[op] = {"ms": round(ms, 3), "gbs_orig": round(orig / ms / 1e6, 1)}
    log(f"[bench] out-of-core: {res}")
    del x, slabs
    return res


def bench_batches(a, log):
    """Many fields of uneven shapes analysed in one pass: each field gets mean
    (via D_p), variance (via D_q) and gradient magnitude (via D_q).  Timed as
    a plan launch with the autotuned launch shape (workgroups per CU, planes
    per tile, workgroup shape of the gradient tiles), enqueued directly and
    replayed as the HIP graph captured at creation, against the same jobs as
    separate single-field launches and against full decompression + the
    operations on floats.  Three copies of every batch are launched in turn
    (the tuner's candidates too)."""
    import torch

    from paper_2603_25206_amd import hsz, synth, tune

    res = {}
    workloads = {
        "12 uneven f32 fields (4x 100x500x500, 4x 256x384x384, 4x 1800x3600), rel eb 1e-2/1e-3/1e-4, S=32":
            synth.batch_specs(),
        "8 f64 256^3 fields with tanh fronts, rel eb 1e-6, S=32":
            [(synth.front_field_spec(i), 1e-6) for i in range(8)],
    }
    for name, specs in workloads.items():
        comps, orig = [], 0
        for sp, rel in specs:
            f = synth.make_field_torch(sp, "cuda")
            comps.append(hsz.compress(f, rel, rel=True, block=32))
            orig += f.numel() * f.element_size()
            del f
        sets = list(zip(*[_clones(c) for c in comps]))
        for cs in sets:
            for c in cs:
                c.build_index()

        def jobs_of(cs):
            js = []
            for c in cs:
                js += [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
            return js
        jobsets = [jobs_of(cs) for cs in sets]
        best, timings = tune.tune(jobsets[0], reps=3, cache_path=None, alternates=jobsets[1:])
        st = torch.cuda.Stream()
        row = {"fields": len(comps), "jobs": len(jobsets[0]), "orig_bytes": orig,
               "compressed_bytes": sum(c.nbytes for c in comps), "copies": ROT,
               "autotuned": best, "candidates_tried": len(timings)}
        ref = None
        for label, t in (("plan_ms", best), ("plan_ms_graph_replay", dict(best, graph_replay=1)),
                         ("plan_separate_stats_ms", dict(best, separate_stats=1))):
            plans = [hsz.Plan(js, tune=t, stream=st) for js in jobsets]
            row[label] = round(_events_ms([p.launch for p in plans], 6, st), 4)
            got = plans[0].results()
            for p in plans:
                p.close()
            if ref is None:
                ref = got
            elif not all(tune._same(x, y) for x, y in zip(ref, got)):
                raise RuntimeError(f"batch results differ between launch modes ({label})")
        cur = torch.cuda.current_stream()
        dev = comps[0].data.device
        outs = [hsz._result_for(j, dev)[0] for j in jobsets[0]]
        wsz = max(hsz.op_workspace_bytes(c.header, hsz.GRADMAG) for c in comps)
        ws = hsz.workspace(wsz, dev, key="bench-single")

        def singles(k):
            def f():
                for j, o in zip(jobsets[k], outs):
                    hsz.op_fused(j.c, j.via, j.op, out=o, ws=ws, check=False, raw=True)
            return f
        ms_single = _events_ms([singles(k) for k in range(ROT)], 3, cur)
        fsize = max(c.header.n * (4 if c.header.dtype == 1 else 8) for c in comps) + 64
        fbufs = [torch.empty(fsize, dtype=torch.uint8, device=dev) for _ in range(ROT)]

        def baseline(k):
            def f():
                for j0, c in enumerate(sets[k]):
                    hsz.decompress_to_stage(c, hsz.FLOAT, out=fbufs[k])
                    fv = hsz.stage_view(fbufs[k], c.header, hsz.FLOAT)
                    for op, o in ((hsz.MEAN, outs[3 * j0]), (hsz.VAR, outs[3 * j0 + 1]),
                                  (hsz.GRADMAG, outs[3 * j0 + 2])):
                        hsz.op_on_stage(fv, c.header, hsz.FLOAT, op, out=o, ws=ws, check=False, raw=True)
            return f
        ms_base = _events_ms([baseline(k) for k in range(ROT)], 3, cur)
        ms_plan = row["plan_ms"]
        row.update({"gbs_orig": round(orig / ms_plan / 1e6, 1),
                    "single_launches_ms": round(ms_single, 4), "full_decompress_ms": round(ms_base, 4),
                    "speedup_vs_single": round(ms_single / ms_plan, 3),
                    "speedup_vs_full_decompress": round(ms_base / ms_plan, 3)})
        res[name] = row
        log(f"[bench] batch {name}: {row}")
        del comps, sets, jobsets, outs, fbufs
        torch.cuda.empty_cache()
    return res


def bench_serving(a, log):
    """Compressed snapshots resident in HBM (even: 512^3, odd: 100x500x500,
    f32, rel eb 1e-3, S=32), a Poisson stream of queries (mean, variance or
    gradient magnitude over a random box with sides 32..256), continuous
    batching over 4 stream slots within a 4 GiB budget: the slots'
    workspaces and statistics regions and the result arena are allocated
    when the executor is built, and each result is released by its consumer
    as soon as it completes.  The headline rate, then a sweep of arrival
    rates up to saturation (mean batch size, latency, the throughput
    ceiling)."""
    import torch

    from paper_2603_25206_amd import hsz, synth
    from paper_2603_25206_amd.serve import GpuExecutor, Server, make_queries, summary

    snaps, shapes = [], []
    t0 = time.time()
    for k in range(a.snapshots):
        sp = synth.snapshot_spec(k)
        f = synth.make_field_torch(sp, "cuda")
        snaps.append(hsz.compress(f, 1e-3, rel=True, block=32))
        shapes.append(tuple(sp.shape))
        del f
    torch.cuda.synchronize()
    log(f"[bench] serving: {a.snapshots} snapshots in {time.time() - t0:.1f}s, "
        f"{sum(c.nbytes for c in snaps) / 2**30:.2f} GiB compressed")
    ex = GpuExecutor(snaps, n_slots=4, mem_budget=4 << 30, max_batch=64)

    def serve(qs, freeze_gc=True):
        srv = Server(ex, mem_budget=ex.result_budget, max_batch=64, hold_results=True)
        srv.on_done = srv.release  # the consumer takes each result as it completes
        t1 = time.perf_counter()
        done = srv.run(qs, freeze_gc=freeze_gc)
        wall = time.perf_counter() - t1
        r = summary(done, wall, bytes_per_elem=4)
        r.update({"batches": srv.stats.launched_batches,
                  "mean_batch": round(float(np.mean(srv.stats.batch_sizes)), 2),
                  "max_batch": int(max(srv.stats.batch_sizes)), "max_in_flight": srv.stats.max_in_flight,
                  "max_result_mem_mib": round(srv.stats.max_mem / 2**20, 1),
                  "sched_max_round_gap_ms": srv.stats.max_round_gap * 1e3,
                  "sched_max_launch_ms": srv.stats.max_launch * 1e3,
                  "sched_max_collect_ms": srv.stats.max_collect * 1e3,
                  "gc_pauses": srv.stats.gc_pauses, "gc_max_pause_ms": srv.stats.gc_max_pause * 1e3})
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}

    serve(make_queries(shapes, 200, rate_hz=a.rate, seed=1))  # warm-up
    s = serve(make_queries(shapes, a.queries, rate_hz=a.rate, seed=7))
    # the same trace with the collector scanning every object (no freeze)
    s["no_gc_freeze"] = {k: v for k, v in serve(make_queries(shapes, a.queries, rate_hz=a.rate, seed=7),
                                                 freeze_gc=False).items()
                         if k in ("p50_ms", "p99_ms", "p999_ms", "max_ms", "max_wait_ms", "sched_max_round_gap_ms",
                                  "gc_pauses", "gc_max_pause_ms")}
    s.update({"snapshots": a.snapshots, "rate_hz": a.rate, "slots": ex.n_slots,
              "budget_bytes": 4 << 30, "workspace_and_stats_bytes": ex.budget_fixed,
              "result_arena_bytes": ex.result_budget})
    sweep = []
    for rate in (500.0, 2000.0, 8000.0, 32000.0, 128000.0):
        r = serve(make_queries(shapes, 4000, rate_hz=rate, seed=11))
        r["rate_hz"] = rate
        sweep.append(r)
        log(f"[bench] serving sweep {rate:g} q/s: qps {r['qps']:.0f}, mean batch {r['mean_batch']}, "
            f"p50 {r['p50_ms']:.3f} p99 {r['p99_ms']:.3f} max {r['max_ms']:.3f} ms")
    s["rate_sweep"] = sweep
    s["throughput_ceiling_qps"] = round(max(r["qps"] for r in sweep), 1)
    ex.close()
    log(f"[bench] serving: {s}")
    return s


def cpu_baseline(spec, x, a):
    """The oracle as it stands (single thread, plain C) on a slab of the same
    field: decompress to floats, then mean, variance and gradient magnitude
    on the floats -- the same analytics as one step.  GB/s of original data."""
    import oracle
    planes = min(a.cpu_planes, x.shape[0])
    slab = np.ascontiguousarray(x[:planes])
    buf = oracle.compress(slab, a.eb, rel=True, block=a.block)
    reps, dt = 0, 0.0
    while reps < 4 and (reps == 0 or dt < 10.0):  # about 10 s of CPU work
        t0 = time.perf_counter()
        xf = oracle.decompress(buf, oracle.FLOAT)
        oracle.mean(xf)
        oracle.var(xf)
        oracle.gradmag(xf)
        dt += time.perf_counter() - t0
        reps += 1
        del xf
    out = {"value": round(reps * slab.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"{planes}x{x.shape[1]}x{x.shape[2]} slab of the same field ({slab.nbytes / 2**20:.0f} MiB) "
                     f"x {reps} passes: decompress to floats + mean + var + gradmag, {dt:.1f} s"}
    out["all_cores"] = cpu_all_cores(x, a)
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_all_cores(x, a):
    """The same single-thread oracle on every core of the host's share at
    once: the field cut into one slab of consecutive planes per thread, each
    slab compressed as a field of its own (untimed), then every thread
    decompresses its slab to floats and computes mean, variance and gradient
    magnitude on it (the C calls release the interpreter lock, so the
    threads run in parallel).  Slab 0's results are checked equal to a run
    of the same calls alone.  GB/s of original data over the wall time."""
    import concurrent.futures as cf

    import oracle
    ncpu = os.cpu_count() or 1
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    threads = max(1, min(16, ncpu, int(os.environ.get("OMP_NUM_THREADS") or ncpu)))
    planes = max(2, x.shape[0] // threads)
    slabs = [np.ascontiguousarray(x[k * planes:(k + 1) * planes]) for k in range(threads)]
    with cf.ThreadPoolExecutor(threads) as ex:
        bufs = list(ex.map(lambda s: oracle.compress(s, a.eb, rel=True, block=a.block), slabs))

    def work(k):
        xf = oracle.decompress(bufs[k], oracle.FLOAT)
        return oracle.mean(xf), oracle.var(xf), oracle.gradmag(xf)
    reps, dt, first = 0, 0.0, None
    with cf.ThreadPoolExecutor(threads) as ex:
        while reps < 8 and (reps == 0 or dt < 6.0):
            t0 = time.perf_counter()
            res = list(ex.map(work, range(threads)))
            dt += time.perf_counter() - t0
            reps += 1
            if first is None:
                first = res[0]
            del res
    m, v, g = work(0)
    if not (m == first[0] and v == first[1] and np.array_equal(g, first[2])):
        raise RuntimeError("oracle run concurrently disagrees with the same run alone")
    nbytes = sum(s.nbytes for s in slabs)
    return {"value": round(reps * nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "nproc": ncpu, "cpu_model": _cpu_model(),
            "sample": f"{threads} slabs of {planes}x{x.shape[1]}x{x.shape[2]} (the field's first "
                      f"{threads * planes} planes, {nbytes / 2**20:.0f} MiB), each its own stream, one thread each, "
                      f"x {reps} passes: decompress to floats + mean + var + gradmag, {dt:.1f} s wall; "
                      f"slab 0 equal to the same calls run alone"}


if __name__ == "__main__":
    main()
