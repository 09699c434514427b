"""Benchmark: SpMSpV GTEPS and HBM bandwidth on one MI355X.

Workload (one "step" = one y <- A x through the whole hot path: scan,
bucket scatter, LDS merge + compaction): A = R-MAT scale 22, edge factor 16,
symmetrised, duplicates and self loops removed, vertices relabelled, fp32
values uniform on (0, 1]; x = 1% of n (41,943 distinct uniform indices,
fp32 values on (0, 1]); 64 different x vectors are generated up front and
used in rotation so every step reads cold columns of the 1 GB matrix.
All inputs are resident in HBM before timing starts.

Printed: one JSON line with the headline metric (GTEPS = products / s, the
products being the sum of the selected column lengths), the dominant
kernel's achieved HBM bandwidth against the 8 TB/s peak (each kernel's own
start and end timestamps in HIP events on the launch stream), the CPU oracle's rate on a bounded sample
of the same workload, and side measurements (density sweep, min-select2nd,
BFS from 16 roots).
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

PEAK_HBM_GBS = 8000.0
METRIC = "SpMSpV GTEPS + HBM GB/s (% peak), plain vs batched+learned, 1 MI355X"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(phase, semiring, f, fnz, W, nnz_y):
    """Bytes each phase must move (per launch), from the method's data flow."""
    vbytes = 4 if semiring == 0 else 0      # plus-times reads A's values
    xbytes = 4 if semiring in (0, 1) else 1
    if phase == "scan":     # x idx + x val + colptr pair; compacted column triples
        return f * (4 + xbytes + 8) + 12 * fnz
    if phase == "scatter":  # column triples, row ids (+ values), bucket pairs written
        return 12 * fnz + W * (4 + vbytes) + 8 * W
    if phase == "merge":    # bucket pairs read, y (index + value) written
        return 8 * W + nnz_y * (4 + xbytes)
    if phase == "one_launch":   # the three phases' data flow in one kernel
        return sum(algorithmic_bytes(p, semiring, f, fnz, W, nnz_y) for p in ("scan", "scatter", "merge"))
    raise ValueError(phase)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--density", type=float, default=1e-2)
    ap.add_argument("--nx", type=int, default=64, help="distinct x vectors used in rotation")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="only the timed headline loop (for rocprofv3)")
    ap.add_argument("--schedules", action="store_true", help="also time a grid of launch schedules")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 256 MiB device copies (HBM counter calibration)")
    ap.add_argument("--batch-only", action="store_true", help="only the batched workload (R-MAT scale 20)")
    ap.add_argument("--no-msbfs", action="store_true", help="skip the 64-source BFS of the batched workload")
    ap.add_argument("--selector-only", action="store_true", help="only the learned-selector evaluation")
    ap.add_argument("--grid-only", action="store_true", help="only the 3-D grid BFS (256^3)")
    ap.add_argument("--formats-only", action="store_true",
                    help="only the format variants, masked multiplies, connected components and the deterministic mode on the headline graph")
    ap.add_argument("--no-selector-eval", action="store_true", help="skip the learned-selector evaluation")
    ap.add_argument("--selector-scale", type=int, default=24, help="R-MAT scale of the held-out graph")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the density sweep (push and pull) on the headline graph (for rocprofv3)")
    ap.add_argument("--bfs-profile", choices=("learned_graph", "learned", "diropt", "push"),
                    help="only BFS from 4 roots of the held-out graph in one level-loop mode (for rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is designed, not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import synth
    import paper_1610_07902_amd as spv

    spv.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batch_only:
        print(json.dumps(batch_bench(spv, dev, msbfs=not args.no_msbfs)))
        return
    if args.selector_only:
        print(json.dumps(selector_eval(spv, dev, args.selector_scale)))
        return
    if args.grid_only:
        print(json.dumps(grid_bfs_bench(spv, dev)))
        return
    if args.bfs_profile:
        print(json.dumps(bfs_profile(spv, dev, args.bfs_profile, args.selector_scale)))
        return

    t0 = time.time()
    A = synth.rmat(args.scale, 16, seed=1, symmetrize=True)
    log(f"generated {A.name}: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    M = spv.Matrix.from_csc(A, device=dev, flags=spv.WITH_TRANSPOSE)
    deg = A.degrees()
    if args.sweep_only:
        print(json.dumps({"sweep": sweep(spv, M, A, deg, dev, torch.cuda.current_stream())}))
        return
    if args.formats_only:
        print(json.dumps({"formats": formats_bench(spv, M, A, dev), "masked": masked_bench(spv, M, A, dev),
                          "cc": cc_bench(spv, M, A, dev), "deterministic": det_bench(spv, A, dev)}))
        return
    f = synth.density_f(A.n, args.density)
    xs = [synth.sparse_x(A.n, f, seed=1000 + r) for r in range(args.nx)]
    W = np.array([int(deg[x[0]].sum()) for x in xs], np.int64)
    fnz = np.array([int((deg[x[0]] > 0).sum()) for x in xs], np.int64)
    xi_d = [torch.as_tensor(x[0]).to(dev) for x in xs]
    xv_d = [torch.as_tensor(x[1]).to(dev) for x in xs]
    y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
    y_val = torch.empty(A.m, dtype=torch.float32, device=dev)
    d_nnz = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    log(f"f={f} mean W={W.mean():.0f} uploaded in {time.time() - t0:.1f}s; schedule {M.schedule.as_dict()}")

    def step(i, flags=0):
        r = i % args.nx
        spv.spmspv_run(M.handle, spv.PLUS_TIMES_F32, flags, f, xi_d[r], xv_d[r], y_idx, y_val, A.m, d_nnz,
                       sync=False, stream=stream)

    # nnz(y) of each x (one synchronous pass; also a sanity check of W)
    nnz_y = np.zeros(args.nx, np.int64)
    for r in range(args.nx):
        nnz_y[r] = spv.spmspv_run(M.handle, 0, 0, f, xi_d[r], xv_d[r], y_idx, y_val, A.m, d_nnz, sync=True)
        st = M.last_stats()
        assert st["W"] == W[r] and st["err"] == 0, st

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    steps_idx = np.arange(args.steps) % args.nx
    products = int(W[steps_idx].sum())
    gteps = products / (ms * 1e-3) / 1e9
    log(f"headline: {args.steps} steps in {ms:.3f} ms -> {gteps:.2f} GTEPS")
    if args.profile_only:
        print(json.dumps({"metric": METRIC, "value": gteps, "unit": "GTEPS", "ms_per_step": ms / args.steps}))
        return

    eff = spv.spmspv_effective_schedule(M.handle, f)
    # The same loop with the schedule forced to the other launch mode, for comparison.
    other = 1 if eff.launch == 2 else 2
    s = M.schedule
    s.launch = other
    try:
        M.schedule = s
        for i in range(args.warmup):
            step(i)
        ev0.record(stream)
        for i in range(args.steps):
            step(i)
        ev1.record(stream)
        torch.cuda.synchronize()
        other_ms = ev0.elapsed_time(ev1) / args.steps
    except spv.SpmspvError:
        other_ms = None
    M.schedule = None
    log(f"launch {other}: {other_ms} ms per step")
    concurrent = None if args.profile_only else concurrent_bench(spv, M, A, f, xi_d, xv_d, W, dev)

    # Per-kernel durations: the same loop again with events around each kernel.
    for i in range(args.steps):
        step(i, spv.PROFILE)
    phase_ms, calls = spv.spmspv_profile_read(M.handle)
    phases = ["one_launch"] if eff.launch == 2 else ["scan", "scatter", "merge"]
    avg_ms = {p: phase_ms[k] / calls for k, p in enumerate(phases)}
    avg_bytes = {p: float(np.mean([algorithmic_bytes(p, 0, f, fnz[r], W[r], nnz_y[r]) for r in steps_idx]))
                 for p in phases}
    dom = max(phases, key=lambda p: avg_ms[p])
    achieved = avg_bytes[dom] / (avg_ms[dom] * 1e-3) / 1e9
    method_bytes = float(np.mean([24 * W[r] + 28 * f + 8 * nnz_y[r] for r in steps_idx]))
    log(f"per-kernel ms {avg_ms}; dominant {dom}: {achieved:.1f} GB/s")

    result = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SpMSpV plus-times fp32, R-MAT scale {args.scale} ef16 symmetrised (n={A.n}, "
                               f"nnz={A.nnz}), x density {args.density:g} (f={f}), {args.nx} rotating x",
                   "scale": args.scale, "nnz": A.nnz, "f": f, "mean_products": float(W.mean()),
                   "mean_nnz_y": float(nnz_y.mean()),
                   "schedule": eff.as_dict(),
                   "other_launch_mode": {"launch": other, "ms_per_step": other_ms},
                   "concurrent_streams": concurrent},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(dom, args),
                     "algorithmic_bytes_per_launch": round(avg_bytes[dom]),
                     "per_kernel_us": {p: round(avg_ms[p] * 1e3, 2) for p in phases},
                     "per_kernel_gbs": {p: round(avg_bytes[p] / (avg_ms[p] * 1e-3) / 1e9, 1) for p in phases},
                     "whole_step_method_gbs": round(method_bytes / (ms / args.steps * 1e-3) / 1e9, 1)},
    }

    # CPU oracle on a bounded sample of the same workload (single thread).
    import oracle
    oracle.build(force=False)
    t_start = time.perf_counter()
    done, prod = 0, 0
    while True:
        r = done % args.nx
        oracle.spmspv(A, xs[r][0], xs[r][1])
        prod += int(W[r])
        done += 1
        if time.perf_counter() - t_start >= args.cpu_seconds:
            break
    cpu_s = time.perf_counter() - t_start
    result["cpu_baseline"] = {"value": round(prod / cpu_s / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                              "sample": f"{done} SpMSpV calls (rotating the same {args.nx} x vectors) in {cpu_s:.1f}s, "
                                        f"fp64 dense-accumulator oracle, one host thread",
                              "host": host_info()}
    log(f"cpu oracle: {result['cpu_baseline']['value']} GTEPS over {done} calls")

    if args.schedules:
        result["schedules"] = schedule_sweep(spv, M, A, deg, dev, stream)
    if not args.no_extras:
        result["sweep"] = sweep(spv, M, A, deg, dev, stream)
        result["bfs"] = bfs_bench(spv, M, A, dev)
        result["formats"] = formats_bench(spv, M, A, dev)
        result["masked"] = masked_bench(spv, M, A, dev)
        result["cc"] = cc_bench(spv, M, A, dev)
        M.close()
        result["deterministic"] = det_bench(spv, A, dev)
        del M, xi_d, xv_d
        torch.cuda.empty_cache()
        result["batched"] = batch_bench(spv, dev, msbfs=not args.no_msbfs)
        torch.cuda.empty_cache()
        result["grid_bfs"] = grid_bfs_bench(spv, dev)
        torch.cuda.empty_cache()
        if not args.no_selector_eval:
            result["learned_selector"] = selector_eval(spv, dev, args.selector_scale)
    print(json.dumps(result))


def concurrent_bench(spv, M, A, f, xi_d, xv_d, W, dev, nstreams=4, steps=256):
    """The headline multiplies issued round-robin on several streams, one
    handle (workspace) per stream over the same matrix arrays: independent
    multiplies overlap their latency-bound phases.  Reported beside the
    headline, which runs one multiply at a time."""
    import torch
    nx = len(xi_d)
    handles = [M] + [spv.Matrix(A.m, A.n, M.colptr, M.rowids, M.values, device=dev) for _ in range(nstreams - 1)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    ys = [(torch.empty(A.m, dtype=torch.int32, device=dev), torch.empty(A.m, dtype=torch.float32, device=dev))
          for _ in range(nstreams)]

    def run(n):
        for i in range(n):
            k = i % nstreams
            r = i % nx
            spv.spmspv_run(handles[k].handle, 0, 0, f, xi_d[r], xv_d[r], ys[k][0], ys[k][1], A.m, sync=False,
                           stream=streams[k])

    run(4 * nstreams)
    torch.cuda.synchronize()
    t = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    products = int(W[np.arange(steps) % nx].sum())
    for h in handles[1:]:
        h.close()
    out = {"streams": nstreams, "steps": steps, "ms_per_step": round(dt * 1e3 / steps, 4),
           "GTEPS": round(products / dt / 1e9, 2)}
    log(f"concurrent streams: {out}")
    return out


def host_info():
    """The host the oracle ran on: logical CPUs, the ones this process may
    use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


COPY_BYTES = 256 << 20


def copy_calibration(torch):
    """Ten plain device-to-device copies of 256 MiB: each reads and writes
    exactly COPY_BYTES, so FETCH_SIZE / WRITE_SIZE per dispatch of this copy
    kernel convert the counters' units to bytes."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 10}))


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for name in ("spmspv_kernels.hip", "fused_kernels.hip", "device_ops.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1610_07902_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, args):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is missing, is for another workload, or was
    taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != kernel_source_digest() or rec.get("scale") != args.scale or \
            rec.get("density") != args.density:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def time_calls(spv, M, sr, f, xi, xv, y_idx, y_val, m, steps, stream):
    import torch
    nx = len(xi)
    for i in range(4):
        spv.spmspv_run(M.handle, sr, 0, f, xi[i % nx], xv[i % nx], y_idx, y_val, m, sync=False, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        spv.spmspv_run(M.handle, sr, 0, f, xi[i % nx], xv[i % nx], y_idx, y_val, m, sync=False, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def schedule_sweep(spv, M, A, deg, dev, stream):
    import torch
    import synth
    out = {}
    y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
    y_val = torch.empty(A.m, dtype=torch.float32, device=dev)
    for dens in (1e-3, 1e-2, 1e-1):
        f = synth.density_f(A.n, dens)
        xs = [synth.sparse_x(A.n, f, seed=4000 + r) for r in range(8)]
        W = float(np.mean([int(deg[x[0]].sum()) for x in xs]))
        xi = [torch.as_tensor(x[0]).to(dev) for x in xs]
        xv = [torch.as_tensor(x[1]).to(dev) for x in xs]
        for tl in (12, 13, 14, 15):
            for sb, si in ((1024, 8), (1024, 4), (512, 4)):
                for mb in (1024, 512):
                    try:
                        M.schedule = spv.Schedule(0, tl, sb, si, mb, 0)
                    except spv.SpmspvError:
                        continue
                    ms = time_calls(spv, M, 0, f, xi, xv, y_idx, y_val, A.m, 32, stream)
                    out[f"d{dens:g}/t{tl}/s{sb}x{si}/m{mb}"] = round(W / (ms * 1e-3) / 1e9, 2)
    M.schedule = None
    best = {}
    for k, v in out.items():
        d = k.split("/")[0]
        if d not in best or v > best[d][1]:
            best[d] = (k, v)
    log(f"schedule sweep best: {best}")
    return {"GTEPS": out, "best": best}


def sweep(spv, M, A, deg, dev, stream):
    import torch
    import synth
    out = {}
    for sr, name in ((0, "plus_times_f32"), (1, "min_select2nd_i32")):
        for dens in (1e-4, 1e-3, 1e-2, 1e-1):
            f = synth.density_f(A.n, dens)
            nx = 16
            xs = [synth.sparse_x(A.n, f, seed=3000 + r) for r in range(nx)]
            W = float(np.mean([int(deg[x[0]].sum()) for x in xs]))
            xi = [torch.as_tensor(x[0]).to(dev) for x in xs]
            xv = [torch.as_tensor(x[1] if sr == 0 else x[0]).to(dev) for x in xs]
            y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
            y_val = torch.empty(A.m, dtype=torch.float32 if sr == 0 else torch.int32, device=dev)
            rec = {"f": f, "push_launch": spv.spmspv_effective_schedule(M.handle, f, 0, sr).launch}
            # push with the default schedule (sized per call, launch mode by the
            # expected product count), push forced to each launch mode, pull
            for key, direction, launch in (("push", 0, 0), ("push_three", 0, 1), ("push_one", 0, 2),
                                           ("pull", 1, 0)):
                M.schedule = None
                if direction == 1 or launch:
                    s = M.schedule
                    s.direction = direction
                    s.launch = launch
                    M.schedule = s
                try:
                    ms = time_calls(spv, M, sr, f, xi, xv, y_idx, y_val, A.m, 64, stream)
                except spv.SpmspvError:
                    continue
                rec[key + "_us"] = round(ms * 1e3, 2)
                rec[key + "_GTEPS"] = round(W / (ms * 1e-3) / 1e9, 3)
            M.schedule = None
            out[f"{name}@{dens:g}"] = rec
            log(f"sweep {name} density {dens:g}: {rec}")
    return out


def timed_us(fn, reps=32):
    """Mean duration of `reps` back-to-back calls of fn() (enqueue only)
    between two events on the current stream, after 4 warm-up calls."""
    import torch
    for _ in range(4):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def formats_bench(spv, M, A, dev):
    """Format variants on the headline graph (R-MAT scale 22, 1 % x,
    plus-times): left multiplication y' = x'A against the right one; DCSC
    against CSC on the same matrix, as stored (43 % empty columns) and cut
    to one column in 16 (hypersparse); bitvector x / y against list x / y
    (conversions included)."""
    import torch
    import synth
    import oracle
    out = {}
    f = synth.density_f(A.n, 1e-2)
    xs = [synth.sparse_x(A.n, f, seed=7000 + r, sort=True) for r in range(8)]
    xi = [torch.as_tensor(x[0]).to(dev) for x in xs]
    xv = [torch.as_tensor(x[1]).to(dev) for x in xs]
    deg = A.degrees()
    rdeg = np.bincount(A.rowids, minlength=A.m)
    W = float(np.mean([int(deg[x[0]].sum()) for x in xs]))
    Wl = float(np.mean([int(rdeg[x[0]].sum()) for x in xs]))
    y_idx = torch.empty(max(A.m, A.n), dtype=torch.int32, device=dev)
    y_val = torch.empty(max(A.m, A.n), dtype=torch.float32, device=dev)
    k = [0]

    def call(handle, flags, m):
        r = k[0] % 8
        k[0] += 1
        spv.spmspv_run(handle, 0, flags, f, xi[r], xv[r], y_idx, y_val, m, sync=False)

    right = timed_us(lambda: call(M.handle, 0, A.m))
    left = timed_us(lambda: call(M.handle, spv.LEFT, A.n))
    out["left"] = {"right_us": round(right, 2), "left_us": round(left, 2),
                   "right_GTEPS": round(W / right / 1e3, 2), "left_GTEPS": round(Wl / left / 1e3, 2)}
    log(f"formats: left {out['left']}")
    # DCSC against CSC
    for name, B in (("as_stored", A), ("hypersparse_1_in_16",
                                        synth.column_subset(A, np.random.default_rng(3).random(A.n) < 1 / 16))):
        D = synth.csc_to_dcsc(B)
        Mc = M if B is A else spv.Matrix.from_csc(B, device=dev)
        Md = spv.Matrix.from_dcsc(D, device=dev)
        Wb = float(np.mean([int(np.diff(B.colptr.astype(np.int64))[x[0]].sum()) for x in xs]))
        tc = timed_us(lambda: call(Mc.handle, 0, B.m))
        td = timed_us(lambda: call(Md.handle, 0, B.m))
        out["dcsc_" + name] = {"nzc": D.nzc, "n": B.n, "nnz": B.nnz, "products": Wb,
                               "csc_matrix_bytes": 4 * (B.n + 1) + 8 * B.nnz,
                               "dcsc_matrix_bytes": 4 * (2 * D.nzc + 1) + 8 * B.nnz,
                               "csc_us": round(tc, 2), "dcsc_us": round(td, 2)}
        log(f"formats: dcsc {name} {out['dcsc_' + name]}")
        Md.close()
        if Mc is not M:
            Mc.close()
    # bitvector x / y against list x / y
    bits = [torch.as_tensor(oracle.to_bitvector(x[0], None, A.n)[0].view(np.int32)).to(dev) for x in xs]
    y_bits = torch.empty((A.m + 31) // 32, dtype=torch.int32, device=dev)

    def bv():
        r = k[0] % 8
        k[0] += 1
        spv.spmspv_run_bitvector(M.handle, 0, 0, bits[r], xv[r], y_bits, y_val, A.m, sync=False)

    tb = timed_us(bv)
    tl = timed_us(lambda: call(M.handle, 0, A.m))
    out["bitvector"] = {"list_us": round(tl, 2), "bitvector_us": round(tb, 2)}
    log(f"formats: bitvector {out['bitvector']}")
    return out


def masked_bench(spv, M, A, dev):
    """Masked multiplies on the headline graph (1 % x, plus-times) against
    the unmasked one: the bitmap mask (rows with a set bit dropped, half of
    them) and the GraphBLAS form w<mask> = w + A x with a structural mask
    list of half the rows and a w of m/8 entries, without and with replace.
    GTEPS counts the unmasked products (the work the call is asked for)."""
    import torch
    import synth
    f = synth.density_f(A.n, 1e-2)
    xs = [synth.sparse_x(A.n, f, seed=8000 + r) for r in range(8)]
    xi = [torch.as_tensor(x[0]).to(dev) for x in xs]
    xv = [torch.as_tensor(x[1]).to(dev) for x in xs]
    deg = A.degrees()
    W = float(np.mean([int(deg[x[0]].sum()) for x in xs]))
    rng = np.random.default_rng(11)
    drop = rng.random(A.m) < 0.5
    nwords = (A.m + 31) // 32
    packed = np.zeros(nwords * 4, np.uint8)
    packed[: (A.m + 7) // 8] = np.packbits(drop, bitorder="little")
    mask_bits = torch.as_tensor(packed.view(np.int32)).to(dev)
    mi = torch.as_tensor(np.sort(rng.permutation(A.m)[: A.m // 2]).astype(np.int32)).to(dev)
    wi_np = np.sort(rng.permutation(A.m)[: A.m // 8]).astype(np.int32)
    wi = torch.as_tensor(wi_np).to(dev)
    wv = torch.as_tensor(synth.values(wi_np.size, 5)).to(dev)
    y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
    y_val = torch.empty(A.m, dtype=torch.float32, device=dev)
    k = [0]

    def nxt():
        r = k[0] % 8
        k[0] += 1
        return r

    def plain():
        r = nxt()
        spv.spmspv_run(M.handle, 0, 0, f, xi[r], xv[r], y_idx, y_val, A.m, sync=False)

    def bitmap():
        r = nxt()
        spv.spmspv_run_masked(M.handle, 0, 0, f, xi[r], xv[r], mask_bits, y_idx, y_val, A.m, sync=False)

    def graphblas(mflags):
        r = nxt()
        spv.spmspv_run_graphblas(M.handle, 0, 0, f, xi[r], xv[r], mi, None, A.m // 2, mflags, spv.ACCUM_ADD,
                                 wi, wv, wi_np.size, y_idx, y_val, A.m, sync=False)

    out = {"products": W, "mask_rows": A.m // 2, "w_entries": int(wi_np.size)}
    for name, fn in (("unmasked", plain), ("bitmap_mask", bitmap),
                     ("graphblas_accum_add", lambda: graphblas(0)),
                     ("graphblas_accum_add_replace", lambda: graphblas(spv.MASK_REPLACE))):
        t = timed_us(fn)
        out[name] = {"us": round(t, 2), "GTEPS": round(W / t / 1e3, 2)}
    log(f"masked: {out}")
    return out


def det_bench(spv, A, dev):
    """The deterministic plus-times mode (sequential fp32 fold per row in
    product order) against the default multiply, on the headline graph."""
    import torch
    import synth
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC, device=dev)
    deg = A.degrees()
    y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
    y_val = torch.empty(A.m, dtype=torch.float32, device=dev)
    out = {}
    for dens in (1e-3, 1e-2, 1e-1):
        f = synth.density_f(A.n, dens)
        xs = [synth.sparse_x(A.n, f, seed=9000 + r) for r in range(4)]
        W = float(np.mean([int(deg[x[0]].sum()) for x in xs]))
        xi = [torch.as_tensor(x[0]).to(dev) for x in xs]
        xv = [torch.as_tensor(x[1]).to(dev) for x in xs]
        k = [0]

        def call(flags):
            r = k[0] % 4
            k[0] += 1
            spv.spmspv_run(M.handle, 0, flags, f, xi[r], xv[r], y_idx, y_val, A.m, sync=False)

        td = timed_us(lambda: call(0), reps=16)
        tt = timed_us(lambda: call(spv.DETERMINISTIC), reps=16)
        out[f"{dens:g}"] = {"products": W, "default_us": round(td, 2), "deterministic_us": round(tt, 2),
                            "deterministic_GTEPS": round(W / tt / 1e3, 2)}
        log(f"deterministic {dens:g}: {out[f'{dens:g}']}")
    M.close()
    return out


def cc_bench(spv, M, A, dev):
    """Connected components by label propagation (min-select2nd SpMSpV of
    the changed labels each step) on the headline graph."""
    import torch
    P = spv.Matrix(A.m, A.n, M.colptr, M.rowids, None, device=dev)
    P.connected_components()
    torch.cuda.synchronize()
    t = time.perf_counter()
    lab, steps = P.connected_components()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    ncomp = int(torch.unique(lab).numel())
    P.close()
    out = {"ms": round(ms, 2), "steps": int(steps), "components": ncomp}
    log(f"cc: {out}")
    return out


def bfs_bench(spv, M, A, dev):
    """BFS from 16 roots on the pattern of A: push only vs direction-optimizing."""
    import torch
    import synth
    P = spv.Matrix(A.m, A.n, M.colptr, M.rowids, None, flags=spv.SYMMETRIC, device=dev)
    roots = synth.roots(A, 16, seed=2000)
    deg = A.degrees()
    out = {"roots": 16}
    for name, flags in (("push", spv.USE_GRAPH), ("diropt", spv.USE_GRAPH | spv.DIRECTION_OPT)):
        P.bfs(int(roots[0]), spv.MIN_SELECT2ND_I32, flags=flags)   # warm (graph capture)
        total_ms, total_w, levels = 0.0, 0, []
        for r in roots:
            torch.cuda.synchronize()
            t = time.perf_counter()
            lev, par, nl = P.bfs(int(r), spv.MIN_SELECT2ND_I32, flags=flags)
            torch.cuda.synchronize()
            total_ms += (time.perf_counter() - t) * 1e3
            lv = lev.cpu().numpy()
            total_w += int(deg[lv >= 0].sum())
            levels.append(nl)
        out[name] = {"total_ms": round(total_ms, 2), "GTEPS": round(total_w / (total_ms * 1e-3) / 1e9, 3),
                     "levels": levels}
        log(f"bfs {name}: {out[name]}")
    out["note"] = ("GTEPS = sum over reached vertices of their column length (push-equivalent products) / time; "
                   "min-select2nd semiring (parents = smallest in-neighbour on the previous level)")
    P.close()
    return out


def batch_bench(spv, dev, msbfs=True, reps=5):
    """64 independent x against R-MAT scale 20 (ef16, symmetrised, fp32
    values) with f_i log-uniform in [1, n/4]: one batched call versus 64
    plain calls (each reading nnz(y) back, and without the read-back); then
    a 64-source BFS versus 64 single-source BFS runs."""
    import torch
    import synth
    t0 = time.time()
    A = synth.rmat(20, 16, seed=1, symmetrize=True)
    deg = A.degrees()
    M = spv.Matrix.from_csc(A, device=dev)
    sizes = synth.log_uniform_sizes(64, A.n / 4, seed=4100)
    xs = [synth.sparse_x(A.n, int(f), seed=5000 + k) for k, f in enumerate(sizes)]
    off = np.zeros(65, np.int64)
    off[1:] = np.cumsum(sizes)
    W = np.array([int(deg[x[0]].sum()) for x in xs], np.int64)
    Wt = int(W.sum())
    xi_d = [torch.as_tensor(x[0]).to(dev) for x in xs]
    xv_d = [torch.as_tensor(x[1]).to(dev) for x in xs]
    off_d = torch.as_tensor(off).to(dev)
    cat_i = torch.cat(xi_d)
    cat_v = torch.cat(xv_d)
    # room for nnz(A) products per vector: fixed slices, no counting pass (16 GB of HBM here)
    M.attach_batch(64, max_f=int(off[-1]), max_products=64 * A.nnz)
    y_idx = torch.empty(A.m, dtype=torch.int32, device=dev)
    y_val = torch.empty(A.m, dtype=torch.float32, device=dev)
    d_nnz = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    log(f"batched workload: n={A.n} nnz={A.nnz} sum f={int(off[-1])} products={Wt} (set-up {time.time() - t0:.1f}s)")

    def plain(sync):
        for k in range(64):
            spv.spmspv_run(M.handle, 0, 0, int(sizes[k]), xi_d[k], xv_d[k], y_idx, y_val, A.m, d_nnz, sync=sync,
                           stream=stream)

    total_nnz = [0]
    cap = int(min(64 * A.m, Wt)) + 1
    by_idx = torch.empty(cap, dtype=torch.int32, device=dev)
    by_val = torch.empty(cap, dtype=torch.float32, device=dev)
    by_off = torch.empty(65, dtype=torch.int64, device=dev)

    def batched(sync):
        total_nnz[0] = spv.spmspv_run_batch(M.handle, 0, 0, 64, off_d, cat_i, cat_v, by_off, by_idx, by_val, cap,
                                            sync=sync, stream=stream)

    def timed(fn, *a):
        best = []
        fn(*a)
        torch.cuda.synchronize()
        for _ in range(reps):
            t = time.perf_counter()
            fn(*a)
            torch.cuda.synchronize()
            best.append(time.perf_counter() - t)
        return float(np.median(best)), float(np.min(best))

    out = {"workload": "64 x, f_i log-uniform in [1, n/4], plus-times fp32, R-MAT scale 20 ef16 symmetrised",
           "n": A.n, "nnz": A.nnz, "sum_f": int(off[-1]), "products": Wt}
    med, mn = timed(batched, False)
    out["batched_untuned"] = {"ms": round(med * 1e3, 3), "GTEPS": round(Wt / med / 1e9, 3),
                              "schedule": spv.spmspv_get_batch_schedule(M.handle, 64).as_dict()}
    # the autotuner picks the batch's bucket count, workgroup shape and merge block on this batch
    tuned, tuned_us = spv.spmspv_autotune_batch(M.handle, 0, 0, 64, off_d, cat_i, cat_v, by_off, by_idx, by_val, cap,
                                                reps=3, stream=stream)
    log(f"batched workload: untuned {out['batched_untuned']}; tuned {tuned.as_dict()} {tuned_us:.1f} us")
    for name, fn, arg in (("plain_sync", plain, True), ("plain_nosync", plain, False),
                          ("batched", batched, False), ("batched_sync", batched, True)):
        med, mn = timed(fn, arg)
        out[name] = {"ms": round(med * 1e3, 3), "min_ms": round(mn * 1e3, 3), "GTEPS": round(Wt / med / 1e9, 3)}
        log(f"batched workload {name}: {out[name]}")
    out["batched_over_plain_sync"] = round(out["plain_sync"]["ms"] / out["batched"]["ms"], 3)
    out["batched_over_plain_nosync"] = round(out["plain_nosync"]["ms"] / out["batched"]["ms"], 3)
    out["batch_schedule"] = spv.spmspv_get_batch_schedule(M.handle, 64).as_dict()
    M.batch_ws = None
    if msbfs:
        roots = synth.roots(A, 64, seed=2000)
        P = spv.Matrix(A.m, A.n, M.colptr, M.rowids, None, flags=spv.SYMMETRIC, device=dev)
        P.attach_batch(64, msbfs=True)
        single = {}
        for name, fl in (("push", spv.USE_GRAPH), ("diropt", spv.USE_GRAPH | spv.DIRECTION_OPT)):
            P.bfs(int(roots[0]), spv.MIN_SELECT2ND_I32, flags=fl)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for r in roots:
                P.bfs(int(r), spv.MIN_SELECT2ND_I32, flags=fl)
            torch.cuda.synchronize()
            single[name] = round((time.perf_counter() - t) * 1e3, 2)
        multi = {}
        for name, fl in (("push", 0), ("diropt", spv.DIRECTION_OPT)):
            P.msbfs(roots, flags=fl)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lev, par, nl = P.msbfs(roots, flags=fl)
            torch.cuda.synchronize()
            multi[name] = round((time.perf_counter() - t) * 1e3, 2)
        out["msbfs64"] = {"batched_ms": multi["push"], "batched_diropt_ms": multi["diropt"],
                          "single_push_ms": single["push"], "single_diropt_ms": single["diropt"], "levels": nl,
                          "batched_over_single_push": round(single["push"] / multi["push"], 3),
                          "batched_diropt_over_single_diropt": round(single["diropt"] / multi["diropt"], 3)}
        log(f"64-source BFS: {out['msbfs64']}")
        P.close()
    M.close()
    return out


def grid_bfs_bench(spv, dev, side=256):
    """High-diameter BFS: 3-D 7-point grid side^3 with the diagonal, pattern,
    or-and, from the corner vertex 0 (3*(side-1)+1 levels of small
    frontiers): per-level launches versus the captured level graph, the
    persistent kernel, and the direction-optimising and learned variants;
    then the persistent kernel with min-select2nd and parents."""
    import torch
    import synth
    t0 = time.time()
    G = synth.grid(side, side, side)
    P = spv.Matrix.from_csc(G, flags=spv.SYMMETRIC, pattern=True, device=dev)
    nnz = G.nnz
    del G
    log(f"grid BFS: {side}^3 n={P.n} nnz={nnz} set-up {time.time() - t0:.1f}s")
    out = {"graph": f"3-D 7-point grid {side}^3 with diagonal", "n": P.n, "nnz": nnz}
    try:
        from paper_1610_07902_amd import selector
        params, mean, std, _ = selector.load_weights()
        P.load_selector(params, mean, std)
        variants = (("per_level_launch", 0), ("graph", spv.USE_GRAPH),
                    ("persistent", spv.USE_GRAPH | spv.PERSISTENT),
                    ("graph_direction_heuristic", spv.USE_GRAPH | spv.DIRECTION_OPT),
                    ("graph_learned", spv.USE_GRAPH | spv.USE_SELECTOR))
    except OSError:
        variants = (("per_level_launch", 0), ("graph", spv.USE_GRAPH),
                    ("persistent", spv.USE_GRAPH | spv.PERSISTENT),
                    ("graph_direction_heuristic", spv.USE_GRAPH | spv.DIRECTION_OPT))
    variants += (("persistent_min_parents", spv.USE_GRAPH | spv.PERSISTENT),)
    for name, fl in variants:
        sr, par = (spv.MIN_SELECT2ND_I32, True) if name.endswith("_parents") else (spv.OR_AND_BOOL, False)
        P.bfs(0, sr, parents=par, flags=fl)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lev, _, nl = P.bfs(0, sr, parents=par, flags=fl)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        out[name] = {"ms": round(ms, 2), "levels": nl, "us_per_level": round(ms * 1e3 / nl, 2),
                     "GTEPS": round(nnz / (ms * 1e-3) / 1e9, 3)}
        log(f"grid BFS {name}: {out[name]}")
    out["note"] = "GTEPS = stored entries (every column is expanded once) / time"
    P.close()
    return out


def bfs_profile(spv, dev, mode, scale=24, nroots=4):
    """BFS (min-select2nd, parents) on the held-out R-MAT graph of the
    selector evaluation in one level-loop mode: one untimed run, then
    `nroots` timed ones.  Small enough to run under a kernel trace."""
    import torch
    import synth
    from paper_1610_07902_amd import selector
    A = synth.rmat(scale, 16, seed=24, symmetrize=True, with_values=False)
    P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True, device=dev)
    params, mean, std, _ = selector.load_weights()
    P.load_selector(params, mean, std)
    roots = synth.roots(A, nroots, seed=2000)
    del A
    fl = {"learned_graph": spv.USE_SELECTOR | spv.USE_GRAPH, "learned": spv.USE_SELECTOR,
          "diropt": spv.USE_GRAPH | spv.DIRECTION_OPT, "push": spv.USE_GRAPH}[mode]
    P.bfs(int(roots[0]), spv.MIN_SELECT2ND_I32, flags=fl)
    torch.cuda.synchronize()
    t = time.perf_counter()
    levels = []
    for r in roots:
        _, _, nl = P.bfs(int(r), spv.MIN_SELECT2ND_I32, flags=fl)
        levels.append(nl)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    out = {"mode": mode, "graph": f"R-MAT scale {scale} ef16 symmetrised", "roots": nroots, "ms": round(ms, 2),
           "levels": levels}
    if fl & spv.USE_SELECTOR:
        out["classes_last_root"] = P.selector_classes()
    P.close()
    return out


def selector_eval(spv, dev, scale=24, nroots=16, reps=2):
    """Held-out evaluation of the trained selector: R-MAT scale 24 (ef16,
    symmetrised; never seen in training).  BFS from 16 roots with the fixed
    default schedule (push), the frontier-edge direction heuristic, and the
    learned selector, against the best schedule in hindsight (every level
    timed under all ten classes; strict = per-level minimum, single = best
    one class for all levels).  Then data-driven PageRank (d 0.85, tol 1e-6)
    with the default schedule and with the selector."""
    import torch
    import synth
    from paper_1610_07902_amd import selector
    t0 = time.time()
    A = synth.rmat(scale, 16, seed=24, symmetrize=True, with_values=False)
    log(f"selector eval: generated R-MAT s{scale} n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True, device=dev)
    params, mean, std, meta = selector.load_weights()
    P.load_selector(params, mean, std)
    roots = synth.roots(A, nroots, seed=2000)
    del A
    out = {"graph": f"R-MAT scale {scale} ef16 symmetrised (held out)", "n": P.n, "nnz": P.nnz, "roots": nroots,
           "training": meta, "weights_match_kernels": selector.weights_current(meta)}

    def run_bfs(flags):
        P.bfs(int(roots[0]), spv.MIN_SELECT2ND_I32, parents=True, flags=flags)
        torch.cuda.synchronize()
        t = time.perf_counter()
        classes = []
        for r in roots:
            P.bfs(int(r), spv.MIN_SELECT2ND_I32, parents=True, flags=flags)
            if flags & spv.USE_SELECTOR:
                classes.append(P.selector_classes())
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, classes

    for name, fl in (("default_push", spv.USE_GRAPH), ("direction_heuristic", spv.USE_GRAPH | spv.DIRECTION_OPT),
                     ("learned", spv.USE_SELECTOR), ("learned_in_graph", spv.USE_SELECTOR | spv.USE_GRAPH)):
        ms, cls = run_bfs(fl)
        out[name + "_ms"] = round(ms, 2)
        if cls:
            out["learned_classes_root0"] = cls[0]
        log(f"selector eval BFS {name}: {ms:.2f} ms")
    samples = selector.bfs_samples(P, P.nnz, roots, reps=reps, tag=f"rmat{scale}")
    T = samples.T
    out["hindsight_strict_ms"] = round(float(T.min(1).sum()) * 1e-3, 2)
    single = [float(T[:, c].sum()) * 1e-3 for c in range(10)]
    out["hindsight_single_class"] = int(np.argmin(single))
    out["hindsight_single_ms"] = round(min(single), 2)
    pred = selector.predict(params, mean, std, samples.X)
    out["learned_choice_regret"] = round(selector.regret(T, pred), 4)
    # The hindsight-best class of every level replayed in the selector's own
    # loop (same scan, inference and host read per level as 'learned').
    best_seq = {}
    for k in range(len(samples.tags)):
        _, rtag, ltag = samples.tags[k].split("/")
        best_seq.setdefault(rtag, []).append((int(ltag[1:]), int(T[k].argmin())))
    t_replay = 0.0
    for r in roots:
        seq = [c for _, c in sorted(best_seq.get(f"r{r}", []))]
        spv.spmspv_force_classes(P.handle, seq)
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.bfs(int(r), spv.MIN_SELECT2ND_I32, parents=True, flags=spv.USE_SELECTOR)
        torch.cuda.synchronize()
        t_replay += time.perf_counter() - t
    spv.spmspv_force_classes(P.handle, [])
    out["hindsight_in_loop_ms"] = round(t_replay * 1e3, 2)
    out["learned_over_hindsight_in_loop"] = round(out["learned_ms"] / out["hindsight_in_loop_ms"], 3)
    log(f"selector eval hindsight replayed in the selector loop: {out['hindsight_in_loop_ms']} ms")
    out["levels_root0"] = [{"step": samples.tags[k].split("/")[-1], "f": int(samples.X[k, 0]),
                            "chosen": int(pred[k]), "best": int(T[k].argmin()),
                            "us": [round(float(v), 1) for v in T[k]]}
                           for k in range(len(pred)) if samples.tags[k].split("/")[1] == f"r{roots[0]}"]
    out["learned_over_hindsight"] = round(out["learned_ms"] / out["hindsight_strict_ms"], 3)
    out["learned_in_graph_over_hindsight"] = round(out["learned_in_graph_ms"] / out["hindsight_strict_ms"], 3)
    out["default_over_hindsight"] = round(out["default_push_ms"] / out["hindsight_strict_ms"], 3)
    log(f"selector eval hindsight strict {out['hindsight_strict_ms']} ms, single class "
        f"{out['hindsight_single_class']} {out['hindsight_single_ms']} ms, choice regret {out['learned_choice_regret']}")
    # PageRank's steps are standalone plus-times multiplies: the network
    # trained on those
    mparams, mmean, mstd, _ = selector.load_weights(kind="multiply")
    P.load_selector(mparams, mmean, mstd)
    for name, fl in (("pagerank_default", 0), ("pagerank_learned", spv.USE_SELECTOR),
                     ("pagerank_learned_on_device", spv.USE_SELECTOR | spv.USE_GRAPH)):
        P.pagerank(0.85, 1e-6, 100, flags=fl)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, it = P.pagerank(0.85, 1e-6, 100, flags=fl)
        torch.cuda.synchronize()
        out[name + "_ms"] = round((time.perf_counter() - t) * 1e3, 2)
        out[name + "_iters"] = it
        log(f"selector eval {name}: {out[name + '_ms']} ms, {it} multiplies")
    out["note"] = ("hindsight_strict / single are sums of per-level event-timed calls of each class (masked "
                   "SpMSpV steps, no decision cost); hindsight_in_loop replays the per-level best classes in the "
                   "selector's own host-driven loop; "
                   "learned and fixed BFS times are end-to-end host-timed runs; 'learned' reads each decision on the "
                   "host (bucket count and direction), 'learned_in_graph' consumes it on the device inside the "
                   "captured level graph (direction only)")
    P.close()
    return out


if __name__ == "__main__":
    main()
