#!/usr/bin/env python
"""Throughput of kernelised linear global attention on one MI355X.

Workload (the long-context single-GPU shard): T = 256 frames x 64 x 128
patches = 2,097,152 tokens, batch 1, 8 heads, d = 128, bf16 Q/K/V drawn
N(0, variance 0.5) and an upstream gradient N(0, 1), all synthetic and
generated in HBM before timing.  One step = forward (summary, FP64
combine, apply) + backward (query pass, dS reduction, FP64 combine, key
pass): every step of the hot path.  The same step in fp32, the forward
alone, per-kernel HIP-event timings and the FP64 CPU oracle on a bounded
sample are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Only one GPU is supported: --gpus above 1 exits.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
BF16_PEAK_TFLOPS = 2500.0      # dense MFMA bf16
FP32_PEAK_TFLOPS = 157.3       # fp32 (matrix and vector)

METRIC = "attn tokens/s fwd & fwd+bwd at 2M tok, BF16 vs FP32; serve p50/p99 ms"
WORKLOAD = dict(B=1, H=8, N=2097152, d=128, grid=(256, 64, 128), std_qkv=0.5 ** 0.5)

# Tensor passes over HBM per launch of each kernel (each pass = B*H*N*d
# elements): what the kernel has to read and write for its part of the
# method, not what it happens to fetch.
KERNEL_PASSES = {
    "summary_fwd": 2,   # read K, V
    "apply": 2,         # read Q, write O
    "bwd_query": 3,     # read Q, dO; write dQ
    "summary_bwd": 2,   # read Q, dO
    "bwd_query_ds": 3,  # fused: read Q, dO; write dQ (and the dS, dz partials)
    "bwd_key": 4,       # read K, V; write dK, dV
}

# the plain stream with each kernel's read/write mix (the fused query
# backward reads twice what it writes and matches none of them)
KERNEL_STREAM = {"summary_fwd": "read", "summary_bwd": "read", "apply": "copy", "bwd_key": "copy"}


def stream_ceilings(nbytes, reps=5):
    """GB/s of the library's plain read, write and copy streams over
    `nbytes` (a copy counts its reads and its writes), each the mean over
    `reps` launches timed by the library's kernel timer."""
    import torch
    import paper_2604_16590_amd as la
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    la.stream_probe("write", a, pattern=0x3C003C00)
    la.stream_probe("copy", b, a)
    torch.cuda.synchronize()
    la.profile_enable(True)
    for _ in range(reps):
        la.stream_probe("read", b, a)
        la.stream_probe("write", b, pattern=0)
        la.stream_probe("copy", b, a)
    stats = la.profile_read()
    la.profile_enable(False)
    out = {}
    for kind, moved in (("read", nbytes), ("write", nbytes), ("copy", 2 * nbytes)):
        launches, ms = stats["stream_" + kind]
        out[kind] = round(moved / (ms / launches * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def kernel_mma(dtype, d):
    """Matrix-core FLOPs per launch of each kernel, in units of 2*B*H*N*d^2.

    Only the method's products count (operand re-layout products do not).
    bf16 applies S (and, in the query backward, S again) as two operands
    hi + lo, so those products count twice; the fused query backward at
    d = 128 uses the hi part only.  fp32 applies S as one fp32 operand.
    """
    two = 2 if dtype == "bf16" else 1
    return {"summary_fwd": 1, "apply": two, "bwd_query": two, "summary_bwd": 1,
            "bwd_query_ds": (1 if d >= 128 else 2) + 1, "bwd_key": 2}


def mma_flops_per_step(kernels, dtype, elems, d):
    table = kernel_mma(dtype, d)
    return sum(table[k] * kernels[k]["launches_per_step"] * 2 * elems * d
               for k in table if k in kernels)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp32", action="store_true", help="skip the fp32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-others", action="store_true", help="skip the other workload shapes")
    ap.add_argument("--serve-window", type=int, default=200,
                    help="arrivals per serving point (the 2,000-arrival window takes minutes)")
    ap.add_argument("--cpu-tokens", type=int, default=262144,
                    help="tokens per head of the oracle sample (8 heads, d = 128)")
    ap.add_argument("--tiled-step", action="store_true",
                    help="only time the fused tiled step (T256 x 64 x 128, 16 heads of d = 64) "
                         "and print one JSON line (for profiling its kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write the profiles/ summaries from the rocprofv3 output under DIR "
                         "(trace/, fetch/, write/, copy_fetch/, copy_write/) and exit (no GPU)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(dtype, with_grad=True):
    import torch
    import paper_2604_16590_amd as la
    w = WORKLOAD
    shape = (w["B"], w["H"], w["N"], w["d"])
    xs = []
    for sid in range(4 if with_grad else 3):
        x = torch.empty(shape, dtype=dtype, device="cuda:0")
        la.gen_fill(x, seed=1002, stream_id=sid, std=w["std_qkv"] if sid < 3 else 1.0)
        xs.append(x)
    torch.cuda.synchronize()
    return xs


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_table(stats, steps, elems, esize):
    out = {}
    for name, (launches, ms) in stats.items():
        avg = ms / max(launches, 1)
        row = {"launches_per_step": launches / steps, "avg_ms": round(avg, 4)}
        if name in KERNEL_PASSES:
            nbytes = KERNEL_PASSES[name] * elems * esize
            row["alg_GB"] = round(nbytes / 1e9, 3)
            row["GB_s"] = round(nbytes / (avg * 1e-3) / 1e9, 1)
        out[name] = row
    return out


# the sources the long-context step's kernels and their launch choices are
# built from (the counter figures go stale when any of these changes)
STEP_SOURCES = ("la_api.cpp", "la_backward.hip", "la_device.h", "la_forward.hip",
                "la_kernels.h", "la_profile.cpp", "la_profile.h", "la_summary.h")


# the sources of the fused tiled step's kernels
TILED_SOURCES = ("la_device.h", "la_kernels.h", "la_profile.cpp", "la_profile.h", "la_summary.h",
                 "la_tiled.hip")


def source_digest(files=STEP_SOURCES):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2604_16590_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters_long_context_bf16.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


TILED_STEP = {"dims": (256, 64, 128), "core": (8, 16, 16), "halo": (2, 4, 4), "H": 16, "d": 64}


def tiled_step_fields():
    """Q, K, V fields [T, Y, X, H, d] of the tiled step's grid (seeded
    synthetic bf16) and its output field."""
    import torch
    import paper_2604_16590_amd as la
    t = TILED_STEP
    qkv = []
    for sid in range(3):
        x = torch.empty(t["dims"] + (t["H"], t["d"]), dtype=torch.bfloat16, device="cuda:0")
        la.gen_fill(x.view(1, 1, -1, t["H"] * t["d"]), seed=1004, stream_id=sid)
        qkv.append(x)
    return qkv, torch.empty_like(qkv[0])


def tiled_step_only(steps, warmup):
    """The fused tiled step alone (the kernels of the tiled profile)."""
    import torch
    import paper_2604_16590_amd as la
    t = TILED_STEP
    qkv, o = tiled_step_fields()
    fused = lambda: la.tiled_forward(*qkv, t["core"], t["halo"], out=o)
    for _ in range(warmup):
        fused()
    torch.cuda.synchronize()
    la.profile_enable(True)
    for _ in range(steps):
        fused()
    kst = la.profile_read()
    la.profile_enable(False)
    print(json.dumps({"workload": "fused tiled step, T256 x 64 x 128, cores 8 x 16 x 16, halos "
                                  "2 x 4 x 4, 16 heads of d = 64, bf16",
                      "steps": steps, "warmup": warmup,
                      "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in kst.items()},
                      "tiled_source_digest": source_digest(TILED_SOURCES)}), flush=True)


def other_workloads(steps):
    """tokens/s of the same path at the other bf16 workload shapes: the
    fwd+bwd shape at d = 64 (B2 H16, T64 x 64 x 64 = 262,144 tokens) and the
    grid forward (B4 H16, T8 x 32 x 64 = 16,384 tokens, d = 64)."""
    import torch
    import paper_2604_16590_amd as la
    out = {}
    for name, (B, H, N, d), bwd, grid in (
            ("fwd_bwd_B2_H16_N262144_d64", (2, 16, 262144, 64), True, None),
            ("fwd_B4_H16_N16384_d64", (4, 16, 16384, 64), False, (8, 32, 64))):
        xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(4)]
        for sid, x in enumerate(xs):
            la.gen_fill(x, seed=1001, stream_id=sid, grid=grid if sid < 3 else None)
        plan = la.Plan(*xs[:3], dout=xs[3])

        def step():
            plan.forward()
            if bwd:
                plan.backward()

        t = time_steps(step, max(steps, 20), 3)
        out[name] = {"tokens_per_s": round(B * N / t, 1), "ms_per_step": round(t * 1e3, 4)}
        if not bwd:
            # the small grid (537 MB moved) fits largely in the 256 MB
            # Infinity Cache across back-to-back steps: time it also with L2
            # and the Infinity Cache flushed before every step (a 1 GiB write
            # stream), each step bracketed by its own events, median of >= 20
            out[name].update(flushed_step(plan.forward, max(steps, 20), B * N,
                                          4 * B * H * N * d * 2))
        log("%s %.3f ms" % (name, t * 1e3))
        del plan, xs
        torch.cuda.empty_cache()

    # summary reuse: new queries against a cached (S, z) of the long-context
    # shape (the apply alone: read Q, write O)
    w = WORKLOAD
    B, H, N, d = w["B"], w["H"], w["N"], w["d"]
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(4)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1002, stream_id=sid, std=w["std_qkv"])
    _, S, z = la.forward(*xs[:3], return_summary=True)
    t = time_steps(lambda: la.apply(xs[3], S, z, out=xs[0]), max(steps, 20), 3)
    out["apply_cached_summary_B1_H8_N2097152_d128"] = {
        "tokens_per_s": round(B * N / t, 1), "ms_per_step": round(t * 1e3, 4),
        "GB_s": round(2 * B * H * N * d * 2 / t / 1e9, 1)}
    log("apply with a cached summary %.3f ms" % (t * 1e3))
    # the noise-gated layer output: spatial attention blended in place into
    # the temporal branch's output (apply against a cached summary, then the
    # gated apply: read Q and the other branch, write O)
    sigma = torch.full((B,), 0.7, dtype=torch.float64, device="cuda:0")
    t = time_steps(lambda: la.apply_gated(xs[3], S, z, xs[1], sigma, 0.5, out=xs[1]),
                   max(steps, 20), 3)
    out["apply_gated_in_place_B1_H8_N2097152_d128"] = {
        "tokens_per_s": round(B * N / t, 1), "ms_per_step": round(t * 1e3, 4),
        "GB_s": round(3 * B * H * N * d * 2 / t / 1e9, 1)}
    log("gated apply in place %.3f ms" % (t * 1e3))
    del xs, S, z
    torch.cuda.empty_cache()

    # the paper's tiles with halos: extract and Hann-weighted blend of a
    # [T256, 64, 128, C=1024] bf16 field, cores 8 x 16 x 16, halos 2 x 4 x 4
    dims, core, halo, C = (256, 64, 128), (8, 16, 16), (2, 4, 4), 1024
    field = torch.empty(dims + (C,), dtype=torch.bfloat16, device="cuda:0")
    la.gen_fill(field.view(1, 1, -1, C), seed=1003, stream_id=0)
    tiles = la.tile_extract(field, core, halo)
    t_ex = time_steps(lambda: la.tile_extract(field, core, halo), max(steps, 10), 2)
    t_bl = time_steps(lambda: la.tile_blend(tiles, dims, core, halo), max(steps, 10), 2)
    fb, tb = field.numel() * 2, tiles.numel() * 2
    out["tiles_T256_Y64_X128_C1024"] = {
        "core": core, "halo": halo, "tile_bytes": tb, "field_bytes": fb,
        "extract_ms": round(t_ex * 1e3, 4), "extract_GB_s": round((fb + tb) / t_ex / 1e9, 1),
        "blend_ms": round(t_bl * 1e3, 4), "blend_GB_s": round((fb + tb) / t_bl / 1e9, 1)}
    log("tiles: extract %.3f ms, blend %.3f ms" % (t_ex * 1e3, t_bl * 1e3))
    del field, tiles
    torch.cuda.empty_cache()

    # the whole tiled step on the same grid, 16 heads of d = 64: fused
    # (la_tiled_forward: tile summaries read K, V in place, one pass reads Q
    # and writes O) against the composition that materialises the tiles
    qkv, o = tiled_step_fields()
    fused = lambda: la.tiled_forward(*qkv, core, halo, out=o)
    t_f = time_steps(fused, max(steps, 10), 2)
    la.profile_enable(True)
    for _ in range(5):
        fused()
    kst = la.profile_read()
    la.profile_enable(False)
    t_u = time_steps(lambda: la.tiled_attention(*qkv, core, halo), 3, 1)
    nbytes = 4 * fb
    out["tiled_step_T256_Y64_X128_H16_d64"] = {
        "core": core, "halo": halo, "fused_ms": round(t_f * 1e3, 4),
        "fused_tokens_per_s": round(dims[0] * dims[1] * dims[2] / t_f, 1),
        "alg_GB": round(nbytes / 1e9, 3), "fused_GB_s": round(nbytes / t_f / 1e9, 1),
        "fused_frac_of_hbm_peak": round(nbytes / t_f / 1e9 / HBM_PEAK_GBS, 4),
        "fused_kernels_ms": {k: round(v[1] / v[0], 4) for k, v in kst.items()},
        "unfused_ms": round(t_u * 1e3, 4)}
    log("tiled step: fused %.3f ms, unfused %.3f ms" % (t_f * 1e3, t_u * 1e3))
    del qkv, o
    torch.cuda.empty_cache()
    return out


def flushed_step(fn, steps, tokens, nbytes):
    """Median time of fn() with the caches flushed before each call, and a
    per-kernel breakdown from a second pass under the kernel timer.  The
    flush reads 1 GiB (four times the Infinity Cache): a flush by writing
    would leave the caches full of dirty lines whose write-back then lands
    in the timed call."""
    import torch
    import paper_2604_16590_amd as la
    flush = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
    sink = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for i in range(3):
        la.stream_probe("read", sink, flush)
        fn()
    for i, (e0, e1) in enumerate(ev):
        la.stream_probe("read", sink, flush)
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    med = ms[len(ms) // 2]
    la.profile_enable(True)
    for i in range(steps):
        la.stream_probe("read", sink, flush)
        fn()
    stats = la.profile_read()
    la.profile_enable(False)
    del flush
    kern = {k: round(v[1] / v[0], 4) for k, v in stats.items() if not k.startswith("stream_")}
    return {"flushed_ms_median": round(med, 4), "flushed_tokens_per_s": round(tokens / (med * 1e-3), 1),
            "flushed_GB_s": round(nbytes / (med * 1e-3) / 1e9, 1),
            "flushed_frac_of_hbm_peak": round(nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "flushed_kernels_ms": kern}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_sample(shape, dtype, seed, std, backward=True, grid=None):
    """The FP64 oracle (as it stands) on one seeded sample: seconds of host
    time, and the GPU path's normwise errors on the same inputs (max over
    (b, h) of ||X - X_ref|| / ||X_ref||)."""
    import numpy as np
    import torch
    import oracle
    import paper_2604_16590_amd as la
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    xs = []
    for sid in range(4 if backward else 3):
        x = torch.empty(shape, dtype=tdt, device="cuda:0")
        la.gen_fill(x, seed=seed, stream_id=sid, std=std if sid < 3 else 1.0, grid=grid)
        xs.append(x)
    torch.cuda.synchronize()

    def host(x):
        x = x.cpu()
        return x.view(torch.int16).numpy().view(np.uint16) if dtype == "bf16" else x.numpy()

    hx = [host(x) for x in xs]
    oracle._load()
    t0 = time.perf_counter()
    o_ref = oracle.forward(*hx[:3])
    refs = oracle.backward(*hx) if backward else None
    dt = time.perf_counter() - t0
    plan = la.Plan(*xs[:3], dout=xs[3] if backward else None)
    plan.forward()
    if backward:
        plan.backward()
    torch.cuda.synchronize()
    lead = shape[0] * shape[1]

    def err(t, ref):
        a = t.float().cpu().numpy().astype(np.float64).reshape(lead, -1)
        r = ref.reshape(lead, -1)
        return float((np.linalg.norm(a - r, axis=1) / np.linalg.norm(r, axis=1)).max())

    errors = {"o": err(plan.o, o_ref)}
    if backward:
        for name, t, r in zip(("dq", "dk", "dv"), (plan.dq, plan.dk, plan.dv), refs):
            errors[name] = err(t, r)
    del plan, xs
    torch.cuda.empty_cache()
    return dt, errors


def cpu_baseline(n_tokens):
    """The FP64 oracle on a bounded sample of the bench workload (B1 H8
    n_tokens d128 bf16, forward + backward), with the GPU's errors on it."""
    import oracle
    w = WORKLOAD
    shape = (1, w["H"], n_tokens, w["d"])
    dt, errors = oracle_sample(shape, "bf16", 77, w["std_qkv"])
    return {
        "value": round(n_tokens / dt, 1), "unit": "tokens/s", "cores": oracle.threads(),
        "kind": "oracle", "cpu": cpu_model(),
        "sample": "fwd+bwd, B1 H8 N%d d128 bf16 N(0,0.5) inputs, FP64 oracle, %.1f s" % (n_tokens, dt),
    }, errors


def cpu_baseline_other_workloads():
    """The oracle on the other workload shapes (whole configurations where
    they take seconds, else a stated sample), tokens/s counting a token
    through all H heads, with the GPU's errors on the same inputs."""
    out = {}
    cases = (
        # name, shape run, heads of the configuration, dtype, backward, grid
        ("fwd_B1_H1_N4096_d64_fp32", (1, 1, 4096, 64), 1, "fp32", False, None),
        ("fwd_B4_H16_N16384_d64", (4, 16, 16384, 64), 16, "bf16", False, (8, 32, 64)),
        ("fwd_bwd_B2_H16_N262144_d64", (1, 2, 262144, 64), 16, "bf16", True, None),
    )
    for name, shape, H_all, dtype, bwd, grid in cases:
        dt, errors = oracle_sample(shape, dtype, 1001, 1.0, backward=bwd, grid=grid)
        tokens = shape[0] * shape[2] * shape[1] / H_all  # tokens through all heads
        out[name] = {"tokens_per_s": round(tokens / dt, 1), "oracle_s": round(dt, 3),
                     "sample": "B%d H%d N%d d%d %s%s" % (shape + (dtype, ", fwd+bwd" if bwd else "")),
                     "errors_vs_oracle": errors}
        log("oracle %s: %.2f s" % (name, dt))
    return out


# ---- profile summaries (host only) ----

# attention kernels of the long-context step, by the demangled name's start
PROFILE_KERNELS = (("la::summary_kernel<0, 128, 0>", "summary_fwd"),
                   ("la::combine_kernel<128, 0>", "combine"),
                   ("la::apply_kernel<0, 0, 128, false>", "apply"),
                   ("la::image_kernel<128>", "images"),
                   ("la::bwd_qds4_kernel<0>", "bwd_query_ds"),
                   ("la::combine_kernel<128, 1>", "combine_bwd"),
                   ("la::bwd_key_kernel<0, 0, 128, 3>", "bwd_key"))
COPY_KERNEL = "stream_copy_swept_kernel"


def profile_name(kernel_name):
    for key, name in PROFILE_KERNELS:
        if key in kernel_name:
            return name
    return None


def read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def find_one(directory, suffix):
    hits = []
    for base, _, files in os.walk(directory):
        hits += [os.path.join(base, f) for f in files if f.endswith(suffix)]
    if len(hits) != 1:
        raise SystemExit("expected one *%s under %s, found %d" % (suffix, directory, len(hits)))
    return hits[0]


def counter_means(directory, counter):
    """Mean value of `counter` per dispatch, by kernel name (rocprofv3
    counter collection CSV: one row per dispatch and counter)."""
    rows = read_csv(find_one(directory, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Kernel_Name"], r.get("Dispatch_Id") or r.get("Correlation_Id"))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in out.items()}


def summarize_profiles(top, prof=None):
    """profiles/kernel_stats_long_context_bf16.txt from a --kernel-trace
    --stats run and profiles/counters_long_context_bf16.{json,txt} from
    FETCH_SIZE and WRITE_SIZE runs, each scaled by what the counter reads
    for the library's plain 1 GiB copy.  The commands are the ones in
    the headers below (run from /tmp with TMPDIR=/tmp)."""
    prof = prof or os.path.join(ROOT, "profiles")
    cal = "rocprofv3 %s -f csv -d %s -o run -- python3 /root/repo/bench.py --copy-calibration"
    if os.path.isdir(os.path.join(top, "tiled_trace")):
        summarize_tiled(top, prof, cal)
    if not os.path.isdir(os.path.join(top, "trace")):
        return
    cmd = ("rocprofv3 %s -f csv -d %s -o run -- python3 /root/repo/bench.py "
           "--steps 5 --warmup 2 --no-fp32 --no-cpu-baseline --no-serve --no-others")
    # kernel statistics
    rows = read_csv(find_one(os.path.join(top, "trace"), "kernel_stats.csv"))
    lines = ["# rocprofv3 kernel statistics: long-context workload (B1 H8 N2097152 d128 bf16), "
             "fwd+bwd step",
             "# command: cd /tmp && TMPDIR=/tmp " + cmd % ("--kernel-trace --stats",
                                                          "DIR/trace"),
             "# (DIR: the rocprofv3 output directory later given to bench.py --summarize-profiles)",
             "# 2 warm-up + 5 timed steps, then 1 warm-up and 5 forward-only steps inside bench.py;",
             "# kernel = the name bench.py reports (its HIP-event averages cover the same launches)",
             "# median_ns: the median launch in the kernel trace (the first, cold launches count "
             "in avg_ns); bench_avg_ns: the same kernel's average over the timed steps by the "
             "bench's own HIP events in this run",
             "%-14s %-60s %6s %14s %12s %7s %12s %13s" % ("kernel", "name", "calls", "total_ns",
                                                         "avg_ns", "pct", "median_ns",
                                                         "bench_avg_ns")]
    durs = {}
    trace_csv = [os.path.join(b, f) for b, _, fs in os.walk(os.path.join(top, "trace"))
                 for f in fs if f.endswith("kernel_trace.csv")]
    if len(trace_csv) == 1:
        for r in read_csv(trace_csv[0]):
            durs.setdefault(r["Kernel_Name"], []).append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    def median(v):
        v = sorted(v)
        return v[len(v) // 2] if v else None
    events = {}
    trace_out = os.path.join(top, "trace.out")
    if os.path.isfile(trace_out):
        events = {k: v["avg_ms"] * 1e6 for k, v in last_json_line(trace_out)["kernels"].items()}
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        pname = profile_name(r["Name"])
        ev = events.get(pname if pname != "combine_bwd" else "", None)
        med = median(durs.get(r["Name"], []))
        lines.append("%-14s %-60s %6s %14s %12.0f %7.2f %12s %13s" % (
            pname or "-", r["Name"][:60], r["Calls"], r["TotalDurationNs"],
            float(r["AverageNs"]), float(r["Percentage"]), "%d" % med if med else "-",
            "%.0f" % ev if ev else "-"))
    with open(os.path.join(prof, "kernel_stats_long_context_bf16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    # HBM traffic
    fetch = counter_means(os.path.join(top, "fetch"), "FETCH_SIZE")
    write = counter_means(os.path.join(top, "write"), "WRITE_SIZE")
    cf = counter_means(os.path.join(top, "copy_fetch"), "FETCH_SIZE")
    cw = counter_means(os.path.join(top, "copy_write"), "WRITE_SIZE")
    copy_f = [v for k, v in cf.items() if COPY_KERNEL in k]
    copy_w = [v for k, v in cw.items() if COPY_KERNEL in k]
    if len(copy_f) != 1 or len(copy_w) != 1:
        raise SystemExit("copy calibration kernel not found")
    gib_kib = float(1 << 20)
    f_fac, w_fac = gib_kib / copy_f[0][0], gib_kib / copy_w[0][0]
    w = WORKLOAD
    elems = w["B"] * w["H"] * w["N"] * w["d"]
    kern = {}
    for name in set(fetch) | set(write):
        pname = profile_name(name)
        if pname is None:
            continue
        fk = fetch.get(name, (0.0, 0))[0]
        wk = write.get(name, (0.0, 0))[0]
        base = pname if pname != "combine_bwd" else "combine"
        kern[pname] = {"fetch_kib": fk, "write_kib": wk,
                       "hbm_bytes_per_launch": (fk * f_fac + wk * w_fac) * 1024.0,
                       "alg_bytes_per_launch": KERNEL_PASSES.get(base, 0) * elems * 2,
                       "dispatches": fetch.get(name, (0.0, 0))[1]}
    # the digest of the sources the counted runs used (their bench lines
    # carry it), so that counters taken on other sources never pass for
    # the current ones
    run_digests = set()
    for name in ("trace.out", "fetch.out", "write.out"):
        path = os.path.join(top, name)
        if os.path.isfile(path):
            run_digests.add(last_json_line(path).get("source_digest"))
    if len(run_digests) != 1 or None in run_digests:
        raise SystemExit("the profiled runs carry no common source digest: %s" % sorted(map(str, run_digests)))
    run_digest = run_digests.pop()
    if run_digest != source_digest():
        print("note: the profiled runs used other kernel sources than these; the bench will "
              "report traffic null until the counters are taken again", file=sys.stderr)
    rec = {"source_digest": run_digest, "copy_factor_fetch": f_fac, "copy_factor_write": w_fac,
           "kernels": kern}
    with open(os.path.join(prof, "counters_long_context_bf16.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# HBM traffic per launch from rocprofv3 counters (FETCH_SIZE, WRITE_SIZE in KiB per "
             "dispatch)",
             "# long-context workload, bf16 fwd+bwd; each counter scaled by what it reads for the "
             "library's plain 1 GiB device copy",
             "# commands: cd /tmp && TMPDIR=/tmp " + cmd % ("--pmc FETCH_SIZE",
                                                            "DIR/fetch"),
             "#           cd /tmp && TMPDIR=/tmp " + cmd % ("--pmc WRITE_SIZE",
                                                            "DIR/write"),
             "#           cd /tmp && TMPDIR=/tmp " + cal % ("--pmc FETCH_SIZE",
                                                            "DIR/copy_fetch"),
             "#           cd /tmp && TMPDIR=/tmp " + cal % ("--pmc WRITE_SIZE",
                                                            "DIR/copy_write"),
             "# (DIR: the rocprofv3 output directory later given to bench.py --summarize-profiles)",
             "# copy of 1 GiB: FETCH_SIZE %.0f KiB (factor %.4f), WRITE_SIZE %.0f KiB (factor %.4f)"
             % (copy_f[0][0], f_fac, copy_w[0][0], w_fac),
             "%-14s %12s %12s %14s %14s" % ("kernel", "fetch_KiB", "write_KiB", "hbm_GB/launch",
                                           "alg_GB/launch")]
    for _, pname in PROFILE_KERNELS:
        if pname in kern:
            k = kern[pname]
            lines.append("%-14s %12.0f %12.0f %14.3f %14.3f" % (
                pname, k["fetch_kib"], k["write_kib"], k["hbm_bytes_per_launch"] / 1e9,
                k["alg_bytes_per_launch"] / 1e9))
    with open(os.path.join(prof, "counters_long_context_bf16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    avg_ms = {profile_name(r["Name"]): float(r["AverageNs"]) / 1e6 for r in rows
              if profile_name(r["Name"])}
    if os.path.isdir(os.path.join(top, "mfma")):
        summarize_mfma(os.path.join(top, "mfma"), prof, cmd, avg_ms)
    if os.path.isfile(os.path.join(top, "bench.json")):
        summarize_bench(os.path.join(top, "bench.json"), prof)
    if os.path.isfile(os.path.join(top, "serve2000.json")):
        summarize_serving(os.path.join(top, "serve2000.json"), prof)
    print("wrote profiles/ summaries (source digest %s)" % rec["source_digest"])


# the fused tiled step's kernels (d = 64) and their algorithmic field
# passes: K and V read by the column walks, Q read and O written by the
# apply; the slot pass moves workspace only
TILED_KERNELS = (("tile_cols_kernel<64>", "tile_cols", 2), ("tile_slot_kernel<64>", "tile_slots", 0),
                 ("tile_apply_kernel<64>", "tile_apply", 2))


def summarize_tiled(top, prof, cal):
    """profiles/tiled_step_T256_Y64_X128_H16_d64.txt: kernel statistics
    and HBM traffic per launch of the fused tiled step, from a kernel trace
    and FETCH_SIZE / WRITE_SIZE runs of bench.py --tiled-step, the counters
    scaled by the same plain-copy calibration as the long-context ones."""
    cmd = ("rocprofv3 %s -f csv -d %s -o run -- python3 /root/repo/bench.py --tiled-step "
           "--steps 10 --warmup 2")
    digests = set()
    for name in ("tiled_trace.out", "tiled_fetch.out", "tiled_write.out"):
        path = os.path.join(top, name)
        if os.path.isfile(path):
            digests.add(last_json_line(path).get("tiled_source_digest"))
    if len(digests) != 1 or None in digests:
        raise SystemExit("the tiled runs carry no common source digest: %s" % sorted(map(str, digests)))
    digest = digests.pop()
    events = last_json_line(os.path.join(top, "tiled_trace.out"))["kernels_ms"]
    rows = read_csv(find_one(os.path.join(top, "tiled_trace"), "kernel_stats.csv"))
    durs = {}
    for r in read_csv(find_one(os.path.join(top, "tiled_trace"), "kernel_trace.csv")):
        durs.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    fetch = counter_means(os.path.join(top, "tiled_fetch"), "FETCH_SIZE")
    write = counter_means(os.path.join(top, "tiled_write"), "WRITE_SIZE")
    cf = [v for k, v in counter_means(os.path.join(top, "copy_fetch"), "FETCH_SIZE").items()
          if COPY_KERNEL in k]
    cw = [v for k, v in counter_means(os.path.join(top, "copy_write"), "WRITE_SIZE").items()
          if COPY_KERNEL in k]
    if len(cf) != 1 or len(cw) != 1:
        raise SystemExit("copy calibration kernel not found")
    f_fac, w_fac = float(1 << 20) / cf[0][0], float(1 << 20) / cw[0][0]
    t = TILED_STEP
    field = t["dims"][0] * t["dims"][1] * t["dims"][2] * t["H"] * t["d"] * 2
    lines = ["# rocprofv3 on the fused tiled step: T256 x 64 x 128 grid, cores 8 x 16 x 16, halos "
             "2 x 4 x 4, 16 heads of d = 64, bf16",
             "# commands: cd /tmp && TMPDIR=/tmp " + cmd % ("--kernel-trace --stats", "DIR/tiled_trace"),
             "#           cd /tmp && TMPDIR=/tmp " + cmd % ("--pmc FETCH_SIZE", "DIR/tiled_fetch"),
             "#           cd /tmp && TMPDIR=/tmp " + cmd % ("--pmc WRITE_SIZE", "DIR/tiled_write"),
             "#           cd /tmp && TMPDIR=/tmp " + cal % ("--pmc FETCH_SIZE", "DIR/copy_fetch"),
             "#           cd /tmp && TMPDIR=/tmp " + cal % ("--pmc WRITE_SIZE", "DIR/copy_write"),
             "# (DIR: the rocprofv3 output directory later given to bench.py --summarize-profiles)",
             "# sources of the tiled kernels: digest %s; counters scaled by the plain 1 GiB copy "
             "(FETCH_SIZE factor %.4f, WRITE_SIZE factor %.4f)" % (digest, f_fac, w_fac),
             "# alg_GB: the field passes the kernel must make (K, V read; Q read, O written); "
             "bench_avg_ms: the library's HIP-event timer in the traced run",
             "%-11s %6s %10s %10s %13s %12s %12s %13s %13s %9s" % (
                 "kernel", "calls", "avg_ms", "median_ms", "bench_avg_ms", "fetch_KiB", "write_KiB",
                 "hbm_GB/launch", "alg_GB/launch", "alg_GB/s")]
    total_ms = 0.0
    for key, pname, passes in TILED_KERNELS:
        row = [r for r in rows if key in r["Name"]]
        if len(row) != 1:
            raise SystemExit("kernel %s not found once in the tiled trace" % key)
        row = row[0]
        fk = [v for k, v in fetch.items() if key in k]
        wk = [v for k, v in write.items() if key in k]
        fk = fk[0][0] if fk else 0.0
        wk = wk[0][0] if wk else 0.0
        avg = float(row["AverageNs"]) / 1e6
        med = sorted(durs[row["Name"]])[len(durs[row["Name"]]) // 2] / 1e6
        total_ms += med
        alg = passes * field
        lines.append("%-11s %6s %10.4f %10.4f %13s %12.0f %12.0f %13.3f %13.3f %9s" % (
            pname, row["Calls"], avg, med, events.get(pname, "-"), fk, wk,
            (fk * f_fac + wk * w_fac) * 1024.0 / 1e9, alg / 1e9,
            "%.1f" % (alg / (med * 1e-3) / 1e9) if alg else "-"))
    lines.append("step (sum of medians) %.4f ms: %.2f GB of field passes, %.1f GB/s, %.4f of 8 TB/s"
                 % (total_ms, 4 * field / 1e9, 4 * field / (total_ms * 1e-3) / 1e9,
                    4 * field / (total_ms * 1e-3) / 1e9 / HBM_PEAK_GBS))
    with open(os.path.join(prof, "tiled_step_T256_Y64_X128_H16_d64.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


MFMA_COUNTERS = "SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES"


def summarize_mfma(directory, prof, cmd, avg_ms):
    """Matrix-core work per launch (SQ_INSTS_VALU_MFMA_MOPS_BF16 counts bf16
    matrix-core work in units of 512 FLOPs over the chip), over the
    kernel's average duration from the kernel trace."""
    mops = counter_means(directory, "SQ_INSTS_VALU_MFMA_MOPS_BF16")
    lines = ["# matrix-core work per launch from rocprofv3 counters: long-context workload, bf16 "
             "fwd+bwd",
             "# command: cd /tmp && TMPDIR=/tmp " + cmd % ("--pmc " + MFMA_COUNTERS,
                                                          "DIR/mfma"),
             "# (DIR: the rocprofv3 output directory later given to bench.py --summarize-profiles)",
             "# SQ_INSTS_VALU_MFMA_MOPS_BF16 counts bf16 matrix-core work in units of 512 FLOPs "
             "(summed over the chip);",
             "# TFLOP/s uses the kernel's average duration from kernel_stats_long_context_bf16.txt; "
             "peak 2500 TFLOP/s dense bf16",
             "%-14s %14s %12s %10s %10s %14s" % ("kernel", "MOPS/launch", "TFLOP/launch", "avg_ms",
                                                "TFLOP/s", "frac_of_2.5PF")]
    by = {}
    for name, (v, _) in mops.items():
        pname = profile_name(name)
        if pname:
            by[pname] = v
    for _, pname in PROFILE_KERNELS:
        if pname in by and pname in avg_ms:
            tf = by[pname] * 512 / 1e12
            rate = tf / (avg_ms[pname] * 1e-3)
            lines.append("%-14s %14.4g %12.4f %10.4f %10.1f %14.4f" % (
                pname, by[pname], tf, avg_ms[pname], rate, rate / 2500.0))
    with open(os.path.join(prof, "mfma_long_context_bf16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def last_json_line(path):
    with open(path) as f:
        return json.loads([l for l in f if l.startswith("{")][-1])


def summarize_bench(path, prof):
    """The bench line of a default run, with its headline figures first."""
    j = last_json_line(path)
    lines = ["# bench.py on one MI355X: long-context workload, bf16 fwd+bwd (plus bf16 forward, "
             "fp32 fwd+bwd, other shapes, serving, oracle on the host)",
             "# command: python bench.py   (20 timed steps after 3 warm-up; per-kernel times from "
             "the library's HIP-event timer)",
             "value %.1f tokens/s, %.3f ms/step; forward alone %.1f tokens/s (%.3f ms)" % (
                 j["value"], j["ms_per_step"], j["fwd_tokens_per_s"], j["fwd_ms"]),
             "roofline: " + json.dumps(j["roofline"]),
             "%-14s %8s %10s %8s %8s" % ("kernel", "launches", "avg_ms", "alg_GB", "GB_s")]
    for name, k in j["kernels"].items():
        lines.append("%-14s %8.1f %10.4f %8s %8s" % (name, k["launches_per_step"], k["avg_ms"],
                                                     k.get("alg_GB", "-"), k.get("GB_s", "-")))
    for key in ("fp32", "cpu_baseline", "errors_vs_oracle_on_sample"):
        lines.append("%s: %s" % (key, json.dumps(j.get(key))))
    lines += ["# full JSON line", json.dumps(j)]
    with open(os.path.join(prof, "bench_long_context_bf16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_serving(path, prof):
    """The serving block of a run with --serve-window 2000."""
    j = last_json_line(path)
    sv = j["serve"]
    lines = ["# serving, 2,000 Poisson arrivals per point: 64-member requests, N log-uniform "
             "[4096, 1048576], H16 d64 bf16",
             "# command: python bench.py --serve-window 2000 --no-fp32 --no-others "
             "--no-cpu-baseline",
             "%-34s %8s %10s %10s %10s %12s %10s" % ("point", "req/s", "p50_ms", "p99_ms",
                                                    "p999_ms", "Mtok/s", "attn_TB/s")]

    def row(name, r):
        return "%-34s %8.2f %10.1f %10.1f %10.1f %12.1f %10.3f" % (
            name, r["req_per_s"], r["p50_ms"], r["p99_ms"], r["p999_ms"], r["tokens_per_s"] / 1e6,
            r.get("attention_TB_s") or 0.0)
    lines.append(row("generated inputs, 200 req/s", sv["saturated_200rps"]))
    lines.append(row("generated inputs, 0.7x capacity", sv["sub_saturation"]))
    ao = sv.get("attention_only")
    if ao:
        lines.append(row("caller-owned inputs, 200 req/s", ao["saturated_200rps"]))
        lines.append(row("caller-owned inputs, 0.7x capacity", ao["sub_saturation"]))
    lines += ["# full serve block", json.dumps(sv)]
    with open(os.path.join(prof, "serving_poisson_2000_arrivals.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(token shards would exchange one (S, z) sum per pass); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_16590_amd as la

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.tiled_step:
        tiled_step_only(args.steps, args.warmup)
        return

    if args.copy_calibration:
        # the library's plain copy (stream_copy_swept_kernel): reads and
        # writes exactly 1 GiB per launch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        la.stream_probe("write", a, pattern=0x01010101)
        for _ in range(3):
            la.stream_probe("copy", b, a)
        torch.cuda.synchronize()
        log("copied 1 GiB x3")
        return

    w = WORKLOAD
    elems = w["B"] * w["H"] * w["N"] * w["d"]
    tokens = w["B"] * w["N"]

    # ---- bf16: the timed step (forward + backward) ----
    log("generating bf16 inputs")
    xs = make_inputs(torch.bfloat16)
    plan = la.Plan(*xs[:3], dout=xs[3])

    def step():
        plan.forward()
        plan.backward()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    la.profile_enable(True)
    t_step = time_steps(step, args.steps, 0)
    stats = la.profile_read()
    la.profile_enable(False)
    log("bf16 fwd+bwd %.3f ms/step" % (t_step * 1e3))
    t_fwd = time_steps(plan.forward, args.steps, 1)
    log("bf16 fwd %.3f ms" % (t_fwd * 1e3))

    kernels = kernel_table(stats, args.steps, elems, 2)
    timed = {k: v for k, v in kernels.items() if k in KERNEL_PASSES}
    dominant = max(timed, key=lambda k: timed[k]["avg_ms"] * timed[k]["launches_per_step"])
    dk = kernels[dominant]
    achieved = dk["GB_s"]
    traffic = traffic_for(dominant)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic}
    # what the kernels that ran must move and multiply, per step
    mma_flops = mma_flops_per_step(kernels, "bf16", elems, w["d"])
    step_bytes = sum(KERNEL_PASSES[k] * kernels[k]["launches_per_step"] * elems * 2
                     for k in KERNEL_PASSES if k in kernels)
    del plan, xs
    torch.cuda.empty_cache()

    peak_bytes = torch.cuda.max_memory_allocated()

    # ceilings measured the same way: plain streams over one tensor's bytes
    streams = stream_ceilings(elems * 2)
    roofline["stream_GB_s"] = streams
    mix = KERNEL_STREAM.get(dominant)
    # a reference, not a ceiling: kernels that issue fewer instructions per
    # byte than the probe's plain stream can exceed it
    roofline["rel_to_stream"] = ({"stream": mix, "ratio": round(achieved / streams[mix], 4),
                                  "note": "dominant kernel's rate / the library's plain stream "
                                          "of the same read:write mix; a reference, not a bound"}
                                 if mix else None)
    log("streams %s" % streams)

    # ---- the other workload shapes (context for the same kernels) ----
    others = None
    if not args.no_others:
        others = other_workloads(args.steps)

    # ---- fp32: the same step in plain fp32 ----
    fp32 = None
    if not args.no_fp32:
        log("generating fp32 inputs")
        xs = make_inputs(torch.float32)
        p32 = la.Plan(*xs[:3], dout=xs[3])

        def step32():
            p32.forward()
            p32.backward()

        n32 = max(2, args.steps // 4)
        step32()
        torch.cuda.synchronize()
        la.profile_enable(True)
        t32 = time_steps(step32, n32, 0)
        k32 = kernel_table(la.profile_read(), n32, elems, 4)
        la.profile_enable(False)
        t32f = time_steps(p32.forward, n32, 1)
        mma32 = mma_flops_per_step(k32, "fp32", elems, w["d"])
        fp32 = {"fwd_bwd_tokens_per_s": round(tokens / t32, 1), "fwd_tokens_per_s": round(tokens / t32f, 1),
                "ms_per_step": round(t32 * 1e3, 3), "fwd_ms": round(t32f * 1e3, 3),
                "kernels_ms": {k: v["avg_ms"] for k, v in k32.items()},
                "mma_frac_of_fp32_peak": round(mma32 / t32 / 1e12 / FP32_PEAK_TFLOPS, 4)}
        log("fp32 fwd+bwd %.3f ms" % (t32 * 1e3))
        del p32, xs
        torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            # the fp32 path against the oracle on a sample of the workload
            # (2 of the 8 heads, 65,536 tokens, the same distributions)
            _, fp32["errors_vs_oracle_on_sample"] = oracle_sample(
                (1, 2, 65536, w["d"]), "fp32", 78, w["std_qkv"])
            fp32["errors_sample"] = "fwd+bwd, B1 H2 N65536 d128 fp32 N(0,0.5) inputs"

    # ---- serving (ensemble-member requests, continuous batching) ----
    serve = None
    if not args.no_serve:
        from paper_2604_16590_amd import serve as serve_mod
        log("serving: Poisson stream of ensemble requests")
        try:
            serve = serve_mod.bench_summary(n_requests=args.serve_window, log=log)
        except Exception as ex:  # reported, not hidden: the line says what failed
            serve = {"error": "%s: %s" % (type(ex).__name__, ex)}
        torch.cuda.empty_cache()

    # ---- oracle on the host cores, plus the GPU's error on that sample ----
    cpu = None
    errors = None
    cpu_others = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        cpu, errors = cpu_baseline(args.cpu_tokens)
        if not args.no_others:
            cpu_others = cpu_baseline_other_workloads()

    result = {
        "metric": METRIC,
        "value": round(tokens / t_step, 1),
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "long-context shard fwd+bwd: T256 x 64 x 128 = 2,097,152 tokens, "
                               "B1 H8 d128, bf16 N(0,0.5) Q/K/V, upstream grad N(0,1)",
                   "global_batch": w["B"], "seq_len": w["N"], "heads": w["H"], "head_dim": w["d"],
                   "parallelism": "single GPU"},
        "fwd_tokens_per_s": round(tokens / t_fwd, 1),
        "fwd_ms": round(t_fwd * 1e3, 4),
        "step_alg_GB": round(step_bytes / 1e9, 3),
        "step_GB_s": round(step_bytes / t_step / 1e9, 1),
        "step_mma_TFLOP_s": round(mma_flops / t_step / 1e12, 2),
        "roofline": roofline,
        "kernels": kernels,
        "peak_device_bytes": peak_bytes,
        "other_workloads": others,
        "fp32": fp32,
        "serve": serve,
        "cpu_baseline": cpu,
        "errors_vs_oracle_on_sample": errors,
        "cpu_baseline_other_workloads": cpu_others,
        # the step's kernel sources this line was measured with
        "source_digest": source_digest(),
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
