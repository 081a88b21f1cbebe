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
materialised stage, compression, and the CPU checker (oracle) timed on a
bounded slab of the same field.
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
    ap.add_argument("--no-hszx", action="store_true", help="skip the block-mean (HSZx) workload")
    ap.add_argument("--no-lorenzo", action="store_true", help="skip the HSZp-nd (Lorenzo) workload")
    ap.add_argument("--no-ooc", action="store_true", help="skip the out-of-core (host-resident slabs) workload")
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


COUNTERS = os.path.join(ROOT, "profiles", "k_batch_grad_gradmag_512cube_counters.txt")
KERNEL_SOURCES = ("grad.hip", "hsz_device.hpp", "hsz_launch.hpp")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_25206_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_record():
    """The committed counter summary of the step's gradient kernel, or None
    when there is none or the kernel sources changed since it was taken."""
    try:
        with open(COUNTERS) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith("TRAFFIC_JSON:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("source_sha") == kernel_source_sha():
                return rec
    return None


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
    c0 = hsz.compress(xg, a.eb, rel=True, block=a.block)
    h = c0.header
    log(f"[bench] compressed: {c0.nbytes / 2**20:.1f} MiB, ratio {c0.ratio:.2f}, max|q| {h.max_abs_q}")
    copies = [c0] + [hsz.Compressed(c0.data.clone(), h) for _ in range(a.copies - 1)]
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    S48 = [torch.empty(64, dtype=torch.uint8, device=dev) for _ in range(3)]
    gbuf = torch.empty(n * 4, dtype=torch.uint8, device=dev)
    qbuf = torch.empty(n * 4, dtype=torch.uint8, device=dev)
    fbuf = torch.empty(n * 4 + 64, dtype=torch.uint8, device=dev)
    dbuf = torch.empty(4 * (n + h.nb) + 64, dtype=torch.uint8, device=dev)
    ws_bytes = max(hsz.op_workspace_bytes(h, op) for op in (hsz.MEAN, hsz.VAR, hsz.GRADMAG))
    ws = [hsz.workspace(ws_bytes, dev, key=f"bench{k}") for k in range(3)]

    def timed(name, fns, steps, warmup):
        """Run the list of (label, fn(copy)) per step; per-label HIP event times."""
        for i in range(warmup):
            for _, fn in fns:
                fn(copies[i % len(copies)])
        torch.cuda.synchronize()
        evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in fns]
               for _ in range(steps)]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for i in range(steps):
            c = copies[i % len(copies)]
            for j, (_, fn) in enumerate(fns):
                evs[i][j][0].record(stream)
                fn(c)
                evs[i][j][1].record(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        per = {lab: float(np.mean([evs[i][j][0].elapsed_time(evs[i][j][1]) for i in range(steps)]))
               for j, (lab, _) in enumerate(fns)}
        return total_ms / steps, per

    # ---- the step: homomorphic analytics from compressed bytes ----------------------
    def f_mean(c):
        hsz.op_fused(c, hsz.DELTA, hsz.MEAN, out=S48[0], ws=ws[0], check=False, raw=True)

    def f_var(c):
        hsz.op_fused(c, hsz.QUANT, hsz.VAR, out=S48[1], ws=ws[1], check=False, raw=True)

    def f_grad(c):
        try:
            hsz.op_fused(c, hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws[2], check=False, raw=True)
        except hsz.HszError as e:
            if e.code != hsz.ERR_UNSUPPORTED:
                raise
            hsz.decompress_to_stage(c, hsz.QUANT, out=qbuf)
            hsz.op_on_stage(hsz.stage_view(qbuf, h, hsz.QUANT), h, hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws[2],
                            check=False, raw=True)

    sep_fns = [("mean_fused_delta", f_mean), ("var_fused_quant", f_var), ("gradmag_quant", f_grad)]
    ms_sep, per_sep = timed("separate", sep_fns, a.steps, a.warmup)
    st_v = hsz.stats_of(S48[1])
    st_m = hsz.stats_of(S48[0])

    # ---- the step: one batched pass, the three analytics sharing one decode -------------
    # Per copy, a plan of three jobs (mean via D_p, variance via D_q,
    # gradient magnitude via D_q) over the whole field; mean and variance are
    # summed inside the gradient tiles.  Block indexes are built once per
    # stream, as a resident stream keeps them.
    for c in copies:
        c.build_index()
    if a.tune is None and not a.no_tune:
        # the launch shape of the step's plan: the autotuner times each
        # candidate on the actual jobs and rejects any that changes a result
        from paper_2603_25206_amd import tune as tuner
        jobs0 = [hsz.Job(copies[0], "mean", hsz.DELTA), hsz.Job(copies[0], "var", hsz.QUANT),
                 hsz.Job(copies[0], "gradmag", hsz.QUANT)]
        a.tune, _ = tuner.tune(jobs0, reps=5, cache_path=None)
        log(f"[bench] step launch shape (autotuned): {a.tune}")
    step_stream = torch.cuda.Stream()
    plans = []
    for c in copies:
        jobs = [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
        plans.append(hsz.Plan(jobs, tune=a.tune, stream=step_stream))
    for i in range(a.warmup):
        plans[i % len(plans)].launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(step_stream)
    for i in range(a.steps):
        evs[i][0].record(step_stream)
        plans[i % len(plans)].launch()
        evs[i][1].record(step_stream)
    stop.record(step_stream)
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / a.steps
    ms_replay = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    res = plans[0].results()
    if (res[1]["s1"], res[1]["s2"], res[1]["var"]) != (st_v["s1"], st_v["s2"], st_v["var"]) or \
            res[0]["mean"] != st_m["mean"] or not torch.equal(res[2].reshape(-1), gbuf.view(torch.float32)):
        raise RuntimeError("batched step disagrees with the separate operations")
    for pl in plans:
        pl.close()

    # ---- baseline: full decompression + the same ops on floats ------------------------
    def b_dec(c):
        hsz.decompress_to_stage(c, hsz.FLOAT, out=fbuf)

    fview = hsz.stage_view(fbuf, h, hsz.FLOAT)

    def b_mean(c):
        hsz.op_on_stage(fview, h, hsz.FLOAT, hsz.MEAN, out=S48[0], ws=ws[0], check=False, raw=True)

    def b_var(c):
        hsz.op_on_stage(fview, h, hsz.FLOAT, hsz.VAR, out=S48[1], ws=ws[1], check=False, raw=True)

    def b_grad(c):
        hsz.op_on_stage(fview, h, hsz.FLOAT, hsz.GRADMAG, out=gbuf, ws=ws[2], check=False, raw=True)

    base_fns = [("decompress_float", b_dec), ("mean_float", b_mean), ("var_float", b_var), ("gradmag_float", b_grad)]
    ms_base, per_base = timed("baseline", base_fns, max(5, a.steps // 2), 2)
    st_bv = hsz.stats_of(S48[1])

    # ---- per-stage table ------------------------------------------------------------
    extra = {}
    if not a.no_extra:
        def dec(stage, out):
            return lambda c: hsz.decompress_to_stage(c, stage, out=out)
        rows = [("decompress_delta", dec(hsz.DELTA, dbuf)), ("decompress_quant", dec(hsz.QUANT, qbuf)),
                ("decompress_float", dec(hsz.FLOAT, fbuf))]
        _, per = timed("decode", rows, 6, 2)
        extra.update(per)
        dview = hsz.stage_view(dbuf, h, hsz.DELTA)
        qview = hsz.stage_view(qbuf, h, hsz.QUANT)
        rows = []
        for stn, st, view in (("delta", hsz.DELTA, dview), ("quant", hsz.QUANT, qview), ("float", hsz.FLOAT, fview)):
            for opn, op in (("mean", hsz.MEAN), ("var", hsz.VAR)):
                rows.append((f"{opn}_on_{stn}", (lambda v, s_, o: lambda c: hsz.op_on_stage(
                    v, h, s_, o, out=S48[2], ws=ws[2], check=False, raw=True))(view, st, op)))
                rows.append((f"{opn}_fused_{stn}", (lambda s_, o: lambda c: hsz.op_fused(
                    c, s_, o, out=S48[2], ws=ws[2], check=False, raw=True))(st, op)))
        for stn, st, view in (("quant", hsz.QUANT, qview), ("float", hsz.FLOAT, fview)):
            rows.append((f"gradmag_on_{stn}", (lambda v, s_: lambda c: hsz.op_on_stage(
                v, h, s_, hsz.GRADMAG, out=gbuf, ws=ws[2], check=False, raw=True))(view, st)))
            rows.append((f"laplacian_on_{stn}", (lambda v, s_: lambda c: hsz.op_on_stage(
                v, h, s_, hsz.LAPLACIAN, out=gbuf, ws=ws[2], check=False, raw=True))(view, st)))
            rows.append((f"laplacian_fused_{stn}", (lambda s_: lambda c: hsz.op_fused(
                c, s_, hsz.LAPLACIAN, out=gbuf, ws=ws[2], check=False, raw=True))(st)))
        _, per = timed("ops", rows, 6, 2)
        extra.update(per)
        # compression (input resident in HBM)
        cbuf = torch.empty_like(c0.data)

        def comp(c):
            hsz.compress(xg, a.eb, rel=True, block=a.block, out=cbuf, check=False)
        _, per = timed("compress", [("compress", comp)], 4, 1)
        extra.update(per)
    if a.calibrate_copy:
        # a plain streaming kernel of known traffic for scaling memory counters:
        # bitwise NOT of 2^27 int32 reads 512 MiB and writes 512 MiB
        src = torch.zeros(2**27, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()

    # ---- roofline of the dominant kernel of the step -------------------------------------
    cbytes = c0.nbytes
    alg = {  # algorithmic bytes per launch (compressed input + outputs; never the avoided floats)
        "mean_fused_delta": cbytes,
        "var_fused_quant": cbytes,
        "gradmag_quant": cbytes + 4 * n,  # fused: read the compressed stream once, write the f32 magnitude
        "decompress_quant": cbytes + 4 * n,
        "decompress_float": cbytes + 4 * n,
        "decompress_delta": cbytes + 4 * n + 4 * h.nb,
        "gradmag_on_quant": 8 * n,
        "gradmag_float": 8 * n,
    }
    # dominant kernel of the step: the batched gradient kernel with shared
    # statistics; its algorithmic bytes are the compressed stream read once
    # plus the f32 magnitude written (the sums add none).  Its duration is
    # the HIP-event time of one plan launch, which also holds the reset and
    # finalize kernels and the gaps between them, so 'achieved' is a lower
    # bound on the kernel's own rate.
    alg_step = cbytes + 4 * n
    achieved = alg_step / (ms_replay * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_batch_grad<32,3,4,float,1> (mean+var+gradmag, one decode)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": a.traffic if a.traffic is not None else counter_traffic(),
                "valu": counter_valu(ms_replay),
                "alg_bytes_per_launch": int(alg_step), "launch_ms": round(ms_replay, 4)}
    dom = "gradmag_quant"
    ach_sep = alg[dom] / (per_sep[dom] * 1e-3) / 1e9
    roofline_sep = {"bound": "hbm", "kernel": "k_grad_fused<32,3,4,float> (gradmag alone)",
                    "achieved": round(ach_sep, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach_sep / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(alg[dom]),
                    "launch_ms": round(per_sep[dom], 4)}

    value = orig_bytes / (ms_step * 1e-3) / 1e9
    base_value = orig_bytes / (ms_base * 1e-3) / 1e9
    out = {
        "metric": "GB/s (orig. data) homomorphic op vs full-decompress+op at eb; p50/p99 query ms",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, shape))} f32 gaussian-mixture x lognormal texture, "
                               f"rel eb {a.eb:g}, S={a.block}; step = mean(D_p) + var(D_q) + gradmag(D_q) "
                               f"from the compressed bytes, one batched pass (one plan launch)",
                   "global_batch": 1, "field_bytes": orig_bytes, "compressed_bytes": cbytes,
                   "ratio": round(c0.ratio, 3), "parallelism": "single-gpu"},
        "separate_ops": {"value": round(orig_bytes / (ms_sep * 1e-3) / 1e9, 1), "unit": "GB/s",
                         "ms_per_step": round(ms_sep, 4), "per_op_ms": {k: round(v, 4) for k, v in per_sep.items()},
                         "roofline": roofline_sep},
        "full_decompress_baseline": {"value": round(base_value, 1), "unit": "GB/s", "ms_per_step": round(ms_base, 4),
                                     "per_op_ms": {k: round(v, 4) for k, v in per_base.items()},
                                     "speedup_homomorphic": round(ms_base / ms_step, 3),
                                     "speedup_separate_ops": round(ms_base / ms_sep, 3)},
        "stage_table_ms": {k: round(v, 4) for k, v in extra.items()},
        "step_launch_shape": a.tune,
        "roofline": roofline,
        "check": {"var_int_route": st_v["var"], "var_float_route": st_bv["var"], "mean": st_m["mean"]},
    }

    del copies, plans, gbuf, qbuf, fbuf, dbuf
    torch.cuda.empty_cache()
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
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def bench_vector(a, log):
    """A three-component 512^3 binary32 vector field (NYX-velocity sized; each
    component the large-field recipe with its own seed, rel eb 1e-4, S=32):
    divergence and curl straight from the three streams through D_q, on the
    materialised quantized stage, and after full decompression of every
    component (decode to floats + the operation on the floats)."""
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
    dev = comps[0].data.device
    cur = torch.cuda.current_stream()
    headers = [c.header for c in comps]
    n = comps[0].header.n
    outs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(3)]
    ws = hsz.workspace(hsz.vector_workspace_bytes(headers), dev, key="bench-vec")
    res = {"components": 3, "shape": list(shape), "orig_bytes": orig,
           "compressed_bytes": sum(c.nbytes for c in comps)}
    qbufs = [torch.empty(4 * n, dtype=torch.uint8, device=dev) for _ in range(3)]
    fbufs = [torch.empty(4 * n + 64, dtype=torch.uint8, device=dev) for _ in range(3)]
    for op in ("divergence", "curl"):
        nout = 3 if op == "curl" else 1

        def fused():
            hsz.vector_op_fused(comps, op, outs=outs[:nout], ws=ws, check=False)

        def on_q():
            for c, b in zip(comps, qbufs):
                hsz.decompress_to_stage(c, hsz.QUANT, out=b)
            hsz.vector_op_on_stage([b[: 4 * n] for b in qbufs], headers, hsz.QUANT, op, outs=outs[:nout], ws=ws,
                                   check=False)

        def full():
            for c, b in zip(comps, fbufs):
                hsz.decompress_to_stage(c, hsz.FLOAT, out=b)
            hsz.vector_op_on_stage(fbufs, headers, hsz.FLOAT, op, outs=outs[:nout], ws=ws, check=False)
        ms_f = _events_ms(fused, 5, cur)
        ms_q = _events_ms(on_q, 5, cur)
        ms_b = _events_ms(full, 5, cur)
        res[op] = {"fused_quant_ms": round(ms_f, 4), "gbs_orig": round(orig / ms_f / 1e6, 1),
                   "decompress_quant_then_op_ms": round(ms_q, 4), "full_decompress_then_op_ms": round(ms_b, 4),
                   "speedup_vs_full_decompress": round(ms_b / ms_f, 3)}
    log(f"[bench] vector field: {res}")
    del comps, outs, qbufs, fbufs
    return res


def bench_hszx(a, log):
    """The step's 512^3 binary32 field compressed in both decorrelation modes
    (rel eb 1e-4, S=32): compression time and ratio, the mean from the block
    means alone (Eq. (mean_m)), the exact mean via D_p, the variance via D_q,
    the spread about the integer metadata mean via D_p (Sec. V-A),
    the gradient magnitude (fused from the delta stream; decode to D_q then
    the stencil for block-mean streams), and full decompression + the mean
    on floats."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = tuple(int(v) for v in a.shape.split(","))
    x = synth.make_field_torch(synth.large_field_spec(seed=0, shape=shape), "cuda")
    dev, cur = x.device, torch.cuda.current_stream()
    orig = x.numel() * x.element_size()
    n = x.numel()
    res = {"shape": list(shape), "orig_bytes": orig}
    s48 = torch.empty(64, dtype=torch.uint8, device=dev)
    gbuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    qbuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    fbuf = torch.empty(4 * n + 64, dtype=torch.uint8, device=dev)
    for mode, mean_dec in (("delta", False), ("block_mean", True)):
        c = hsz.compress(x, a.eb, rel=True, block=a.block, mean_dec=mean_dec)
        torch.cuda.synchronize()
        h = c.header
        ws = hsz.workspace(max(hsz.op_workspace_bytes(h, op) for op in (hsz.MEAN, hsz.VAR, hsz.GRADMAG)), dev,
                           key="bench-hszx")

        def comp():
            hsz.compress(x, a.eb, rel=True, block=a.block, mean_dec=mean_dec)

        def stat(via, op):
            return lambda: hsz.op_fused(c, via, op, out=s48, ws=ws, check=False, raw=True)

        def grad():
            if mean_dec:
                hsz.decompress_to_stage(c, hsz.QUANT, out=qbuf)
                hsz.op_on_stage(hsz.stage_view(qbuf, h, hsz.QUANT), h, hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws,
                                check=False, raw=True)
            else:
                hsz.op_fused(c, hsz.QUANT, hsz.GRADMAG, out=gbuf, ws=ws, check=False, raw=True)

        fview = hsz.stage_view(fbuf, h, hsz.FLOAT)

        def full_mean():
            hsz.decompress_to_stage(c, hsz.FLOAT, out=fbuf)
            hsz.op_on_stage(fview, h, hsz.FLOAT, hsz.MEAN, out=s48, ws=ws, check=False, raw=True)

        r = {"ratio": round(c.ratio, 3), "compress_ms": round(_events_ms(comp, 5, cur), 4)}
        if mean_dec:
            r["mean_meta_ms"] = round(_events_ms(stat(hsz.META, hsz.MEAN), 10, cur), 4)
            m_meta = hsz.stats_of(s48)["mean"]
        r["mean_delta_ms"] = round(_events_ms(stat(hsz.DELTA, hsz.MEAN), 10, cur), 4)
        m_exact = hsz.stats_of(s48)["mean"]
        r["var_quant_ms"] = round(_events_ms(stat(hsz.QUANT, hsz.VAR), 10, cur), 4)
        if mean_dec:
            r["var_mt_delta_ms"] = round(_events_ms(stat(hsz.DELTA, hsz.VAR_MT), 10, cur), 4)
        r["gradmag_ms"] = round(_events_ms(grad, 5, cur), 4)
        r["full_decompress_mean_ms"] = round(_events_ms(full_mean, 5, cur), 4)
        if mean_dec:
            r["mean_meta_gbs_orig"] = round(orig / r["mean_meta_ms"] / 1e6, 1)
            r["speedup_mean_meta_vs_full"] = round(r["full_decompress_mean_ms"] / r["mean_meta_ms"], 2)
            r["mean_meta_minus_exact"] = m_meta - m_exact
            if abs(m_meta - m_exact) > h.eb_abs:
                raise RuntimeError("mean from the block means is farther than eps from the exact mean")
        r["eb_abs"] = h.eb_abs
        res[mode] = r
        del c, ws
    log(f"[bench] block-mean: {res}")
    del x, gbuf, qbuf, fbuf
    return res


def bench_lorenzo(a, log):
    """The step's 512^3 binary32 field as an HSZp-nd stream (rel eb 1e-4,
    S=32, 2x4x4 blocks): compression time and ratio, decoding to each stage,
    the mean with nd weights and Alg. 4 on D_p, the derivative along each
    axis on D_p (Eq. (derivative_Dp)) against the same derivative from D_q
    (decode to D_q + stencil) and after full decompression; and the same
    field as an HSZp stream (deltas across block borders of the flat field):
    ratio, compression, D_p and D_q decoding, mean and variance on D_p."""
    import torch

    from paper_2603_25206_amd import hsz, synth

    shape = tuple(int(v) for v in a.shape.split(","))
    x = synth.make_field_torch(synth.large_field_spec(seed=0, shape=shape), "cuda")
    dev, cur = x.device, torch.cuda.current_stream()
    orig = x.numel() * x.element_size()
    n = x.numel()
    c = hsz.compress(x, a.eb, rel=True, block=a.block, lorenzo=True)
    torch.cuda.synchronize()
    h = c.header
    ws = hsz.workspace(hsz.op_workspace_bytes(h, hsz.DERIV), dev, key="bench-lz")
    s48 = torch.empty(64, dtype=torch.uint8, device=dev)
    obuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    sbuf = torch.empty(4 * n, dtype=torch.uint8, device=dev)
    res = {"shape": list(shape), "orig_bytes": orig, "ratio": round(c.ratio, 3),
           "compress_ms": round(_events_ms(lambda: hsz.compress(x, a.eb, rel=True, block=a.block, lorenzo=True), 5,
                                           cur), 4)}
    for st, name in ((hsz.DELTA, "decode_p_ms"), (hsz.QUANT, "decode_q_ms"), (hsz.FLOAT, "decode_f_ms")):
        res[name] = round(_events_ms(lambda: hsz.decompress_to_stage(c, st, out=sbuf), 5, cur), 4)
    res["mean_p_ms"] = round(_events_ms(lambda: hsz.op_fused(c, hsz.DELTA, hsz.MEAN, out=s48, ws=ws, check=False,
                                                             raw=True), 10, cur), 4)
    res["var_p_ms"] = round(_events_ms(lambda: hsz.op_fused(c, hsz.DELTA, hsz.VAR, out=s48, ws=ws, check=False,
                                                            raw=True), 10, cur), 4)
    fview = hsz.stage_view(sbuf, h, hsz.FLOAT)
    qview = hsz.stage_view(sbuf, h, hsz.QUANT)
    for ax in range(len(shape)):
        r = {}
        r["via_p_ms"] = round(_events_ms(lambda: hsz.op_fused(c, hsz.DELTA, hsz.DERIV, axis=ax, out=obuf, ws=ws,
                                                              check=False, raw=True), 5, cur), 4)

        def via_q():
            hsz.decompress_to_stage(c, hsz.QUANT, out=sbuf)
            hsz.op_on_stage(qview, h, hsz.QUANT, hsz.DERIV, axis=ax, out=obuf, ws=ws, check=False, raw=True)

        def full():
            hsz.decompress_to_stage(c, hsz.FLOAT, out=sbuf)
            hsz.op_on_stage(fview, h, hsz.FLOAT, hsz.DERIV, axis=ax, out=obuf, ws=ws, check=False, raw=True)
        r["decode_q_then_deriv_ms"] = round(_events_ms(via_q, 5, cur), 4)
        r["full_decompress_then_deriv_ms"] = round(_events_ms(full, 5, cur), 4)
        res[f"deriv_axis{ax}"] = r
    # HSZp: deltas across the blocks of the flat field (device-wide prefix sum for D_q)
    cf = hsz.compress(x, a.eb, rel=True, block=a.block, inter_block=True)
    torch.cuda.synchronize()
    wsf = hsz.workspace(hsz.op_workspace_bytes(cf.header, hsz.VAR), dev, key="bench-flat")
    flat = {"ratio": round(cf.ratio, 3),
            "compress_ms": round(_events_ms(lambda: hsz.compress(x, a.eb, rel=True, block=a.block,
                                                                 inter_block=True), 5, cur), 4)}
    for st, name in ((hsz.DELTA, "decode_p_ms"), (hsz.QUANT, "decode_q_ms")):
        flat[name] = round(_events_ms(lambda: hsz.decompress_to_stage(cf, st, out=sbuf), 5, cur), 4)
    flat["mean_p_ms"] = round(_events_ms(lambda: hsz.op_fused(cf, hsz.DELTA, hsz.MEAN, out=s48, ws=wsf, check=False,
                                                              raw=True), 10, cur), 4)
    flat["var_p_ms"] = round(_events_ms(lambda: hsz.op_fused(cf, hsz.DELTA, hsz.VAR, out=s48, ws=wsf, check=False,
                                                             raw=True), 10, cur), 4)
    res["inter_block_1d"] = flat
    log(f"[bench] lorenzo-nd / inter-block: {res}")
    del x, c, cf, ws, wsf, obuf, sbuf
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
    a plan launch with the autotuned launch shape, against the same
    jobs as separate single-field launches and against full decompression +
    the operations on floats."""
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
        jobs = []
        for c in comps:
            jobs += [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
        best, timings = tune.tune(jobs, reps=3, cache_path=None)
        plan = hsz.Plan(jobs, tune=best)
        ms_plan = _events_ms(plan.launch, 5, plan.stream)
        plan.close()
        plan = hsz.Plan(jobs, tune=dict(best, separate_stats=1))
        ms_plan_sep = _events_ms(plan.launch, 5, plan.stream)
        plan.close()
        cur = torch.cuda.current_stream()
        outs = [hsz._result_for(j, comps[0].data.device)[0] for j in jobs]
        wsz = max(hsz.op_workspace_bytes(c.header, hsz.GRADMAG) for c in comps)
        ws = hsz.workspace(wsz, comps[0].data.device, key="bench-single")

        def singles():
            for j, o in zip(jobs, outs):
                hsz.op_fused(j.c, j.via, j.op, out=o, ws=ws, check=False, raw=True)
        ms_single = _events_ms(singles, 3, cur)
        fbufs = [torch.empty(c.header.n * (4 if c.header.dtype == 1 else 8) + 64, dtype=torch.uint8,
                             device=c.data.device) for c in comps[:1]]

        def baseline():
            for c, j0 in zip(comps, range(len(comps))):
                fb = fbufs[0]
                if fb.numel() < c.header.n * (4 if c.header.dtype == 1 else 8):
                    fb = fbufs[0] = torch.empty(c.header.n * 8 + 64, dtype=torch.uint8, device=c.data.device)
                hsz.decompress_to_stage(c, hsz.FLOAT, out=fb)
                fv = hsz.stage_view(fb, c.header, hsz.FLOAT)
                for op, o in ((hsz.MEAN, outs[3 * j0]), (hsz.VAR, outs[3 * j0 + 1]), (hsz.GRADMAG, outs[3 * j0 + 2])):
                    hsz.op_on_stage(fv, c.header, hsz.FLOAT, op, out=o, ws=ws, check=False, raw=True)
        ms_base = _events_ms(baseline, 3, cur)
        res[name] = {"fields": len(comps), "jobs": len(jobs), "orig_bytes": orig,
                     "compressed_bytes": sum(c.nbytes for c in comps),
                     "plan_ms": round(ms_plan, 4), "gbs_orig": round(orig / ms_plan / 1e6, 1),
                     "plan_separate_stats_ms": round(ms_plan_sep, 4),
                     "single_launches_ms": round(ms_single, 4), "full_decompress_ms": round(ms_base, 4),
                     "speedup_vs_single": round(ms_single / ms_plan, 3),
                     "speedup_vs_full_decompress": round(ms_base / ms_plan, 3),
                     "autotuned": best, "candidates_tried": len(timings)}
        log(f"[bench] batch {name}: {res[name]}")
        del comps, jobs, outs, fbufs
        torch.cuda.empty_cache()
    return res


def bench_serving(a, log):
    """Compressed snapshots resident in HBM (even: 512^3, odd: 100x500x500,
    f32, rel eb 1e-3, S=32), a Poisson stream of queries (mean, variance or
    gradient magnitude over a random box with sides 32..256), continuous
    batching over 4 stream slots with a 4 GiB result budget."""
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
    ex = GpuExecutor(snaps, n_slots=4)
    srv = Server(ex, mem_budget=4 << 30, max_batch=64)
    warm = make_queries(shapes, 200, rate_hz=a.rate, seed=1)
    srv.run(warm)
    srv.done.clear()
    srv.stats = type(srv.stats)()
    qs = make_queries(shapes, a.queries, rate_hz=a.rate, seed=7)
    t0 = time.perf_counter()
    done = srv.run(qs)
    wall = time.perf_counter() - t0
    s = summary(done, wall, bytes_per_elem=4)
    s.update({"snapshots": a.snapshots, "rate_hz": a.rate, "slots": ex.n_slots,
              "batches": srv.stats.launched_batches,
              "mean_batch": round(float(np.mean(srv.stats.batch_sizes)), 2),
              "max_in_flight": srv.stats.max_in_flight})
    s = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}
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
    return {"value": round(reps * slab.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{planes}x{x.shape[1]}x{x.shape[2]} slab of the same field ({slab.nbytes / 2**20:.0f} MiB) "
                      f"x {reps} passes: decompress to floats + mean + var + gradmag, {dt:.1f} s"}


if __name__ == "__main__":
    main()
