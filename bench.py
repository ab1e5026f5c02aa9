#!/usr/bin/env python3
"""Throughput of the relaxation step on one MI355X: grid-point updates/s and HBM roofline.

Workload: the 256^3 periodic box [0, 2 pi)^3 holding the ABC Beltrami field (A = B = C = 1),
positions x0 = X + a seeded divergence-free Fourier displacement (|k| <= 3, max 0.1, seed 5).
A step is one accepted adaptive Cash-Karp RK5(4) step (six fused stage sweeps plus the
device step control; rejected attempts are redone inside and counted in the time).

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed|both] [--curl nn|nnn]

Prints one JSON line.  value = N * accepted steps / wall time of the timed relax_step
call (inputs resident in HBM), FP64.  The FP32-mixed figures are in "fp32_mixed".
"roofline" is the dominant kernel's algorithmic bytes per launch (the stage-fused step's
compulsory traffic per node, 72..192 B FP64 / 48..120 B FP32-mixed, times the nodes) over its
average launch duration (HIP events around each launch on the library's stream), against the
8 TB/s HBM3E peak; config.step_hbm_frac is the same for the whole step (792 / 480 B per node
per accepted step over the wall time per step, rejected attempts included in the time).
--curl nnn times the same step with the octilateral current of Sec. 2.3 (FP64 only; no
reverse-mode leg, which needs the nearest-neighbour current).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid-point updates/s (FP64 vs FP32-mixed) + % HBM roofline at 256^3"

# Algorithmic HBM bytes per node of the stage-fused Cash-Karp step (compulsory traffic, halo
# re-reads served by the caches): stage s = 1..5 reads x_n, k_1..k_{s-1} and B0 and writes
# k_s; stage 6 reads x_n, k_1..k_5 and B0 and writes x_{n+1}.  FP64: every vector 24 B;
# FP32-mixed: x in FP64 (24 B), B0 and the k_j in FP32 (12 B).  Per accepted step 792 / 480 B.
ALGO_FP64 = [72, 96, 120, 144, 168, 192]
ALGO_MIXED = [48, 60, 72, 84, 96, 120]
ALGO_STEP = {"fp64": sum(ALGO_FP64), "fp32-mixed": sum(ALGO_MIXED)}

# What this library's sweeps move per node (its own design, used only for the "design" keys).
# Every stage input is x_n plus one increment rounded once; a window holds at most two vectors:
#   stage 1: x_n, B0 -> k_1
#   stage 2: x_n, k_1, B0 -> k_2, y_3
#   stage 3: y_3, B0, k_1, k_2 at the node -> k_3, d_4
#   stage 4: x_n, d_4, B0, k_1..k_3 at the node -> y_5, P6, X, E
#   stage 5: y_5, B0, P6, E -> P6 (now d_6), E
#   stage 6: x_n, d_6, B0, X, E -> x_{n+1}
# FP64: every vector 24 B (864 B per attempt); FP32-mixed: x_n, y_3, y_5 and x_{n+1} 24 B, the
# k_j, d_4, the partial sums and B0 12 B (540 B per attempt).
DESIGN_FP64 = [72, 120, 144, 240, 144, 144]
DESIGN_MIXED = [48, 84, 84, 144, 84, 96]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(R, torch, w, precision, steps, warmup, tol, dt0, curl=0):
    cfg = R.make_config(w.grid, precision=precision, dt0=dt0, tol=tol, adaptive=True, curl=curl)
    x0 = torch.from_numpy(w.x0).cuda()
    B0 = torch.from_numpy(w.B0).cuda()
    N = w.grid.N
    tag = ("fp64" if precision == R.RELAX_FP64 else "fp32-mixed") + ("-octilateral" if curl else "")
    out = {}
    with R.Relaxation(cfg, x0, B0) as r:
        del x0, B0
        log(f"{tag}: warmup {warmup} steps")
        r.step(warmup, diag=False)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        log(f"{tag}: timed {steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(r.stream)
        diag = r.step(steps)
        stop.record(r.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms = start.elapsed_time(stop)
        rejects = sum(d["rejects"] for d in diag)
        # second pass with every launch bracketed by HIP events on the library's stream
        log(f"{tag}: profiled {steps} steps")
        r.profile(True)
        r.step(steps, diag=False)
        prof = r.profile(False)
    algo = ALGO_FP64 if precision == R.RELAX_FP64 else ALGO_MIXED
    design = DESIGN_FP64 if precision == R.RELAX_FP64 else DESIGN_MIXED
    kernels = {}
    for s in range(1, 7):
        ms, n = prof[f"stage{s}"]
        if n == 0:
            continue
        # stage 1 is skipped (an early exit) on retried attempts; its time is spread over the
        # accepted steps, which are the launches that do its work
        work = steps if s == 1 else n
        avg = ms / work
        kernels[f"stage{s}"] = {"avg_ms": avg, "launches": n, "working_launches": work, "total_ms": ms,
                                "algorithmic_GBs": algo[s - 1] * N / (avg * 1e-3) / 1e9,
                                "design_GBs": design[s - 1] * N / (avg * 1e-3) / 1e9}
    kernels["control"] = {"total_ms": prof["control"][0], "launches": prof["control"][1]}
    dom = max((k for k in kernels if "avg_ms" in kernels[k]), key=lambda k: kernels[k]["total_ms"])
    stage = int(dom[-1])
    achieved = kernels[dom]["algorithmic_GBs"]
    traffic = measured_traffic(stage, tag, w.name.replace("^3", ""))
    # whole step: the algorithmic bytes of one accepted step (rejected attempts are overhead)
    # over the wall time per accepted step; and what the design moves, rejected attempts included
    step_ms = wall * 1e3 / steps
    step_tag = "fp64" if precision == R.RELAX_FP64 else "fp32-mixed"
    design_bytes = sum(design[s - 1] * (prof[f"stage{s}"][1] if s > 1 else steps) for s in range(1, 7)) / steps * N
    out.update(
        value=N * steps / wall,
        ms_per_step=step_ms,
        event_ms_per_step=ev_ms / steps,
        rejects=rejects,
        dt_last=diag[-1]["dt"],
        xi_first=diag[0]["xi"],
        xi_last=diag[-1]["xi"],
        E_first=diag[0]["E_M"],
        E_last=diag[-1]["E_M"],
        step_algorithmic_GBs=ALGO_STEP[step_tag] * N / (step_ms * 1e-3) / 1e9,
        step_design_GBs=design_bytes / (step_ms * 1e-3) / 1e9,
        kernels=kernels,
        roofline={"bound": "hbm", "kernel": f"stage_kernel<{stage}> ({tag})",
                  "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "traffic": traffic, "algorithmic_bytes_per_node": algo[stage - 1],
                  "algorithmic_bytes": algo[stage - 1] * N, "design_bytes_per_node": design[stage - 1],
                  "design_GBs": kernels[dom]["design_GBs"]},
    )
    return out


def mixed_vs_fp64_fixed(R, torch, w, dt, K):
    """FP32-mixed against FP64 at identical t: both precisions take K steps of the same fixed
    dt from x0; E_M of every step, and the FP64 diagnostics sweep of both final states."""
    runs = {}
    for prec in (R.RELAX_FP64, R.RELAX_FP32_MIXED):
        cfg = R.make_config(w.grid, precision=prec, dt0=dt, adaptive=False)
        with R.Relaxation(cfg, torch.from_numpy(w.x0).cuda(), torch.from_numpy(w.B0).cuda()) as r:
            d = r.step(K)
            runs[prec] = ([x["E_M"] for x in d], r.diagnostics())
    (E64, f64), (E32, f32) = runs[R.RELAX_FP64], runs[R.RELAX_FP32_MIXED]

    def rel(a, b):
        return abs(a - b) / abs(b)
    return {"steps": K, "dt": dt, "E_M_t_max_rel": max(rel(a, b) for a, b in zip(E32, E64)),
            "final_E_M_rel": rel(f32["E_M"], f64["E_M"]), "final_xi_rel": rel(f32["xi"], f64["xi"]),
            "final_R2_rel": rel(f32["R2"], f64["R2"]), "final_xi_fp64": f64["xi"], "final_R2_fp64": f64["R2"]}


def measured_traffic(stage, tag, workload):
    """HBM bytes per launch of stage_kernel<stage> from the committed FETCH_SIZE / WRITE_SIZE
    summary of this workload, or None when there is none or the kernel source changed since."""
    from paper_1405_0942_amd import profiling
    rec = profiling.read_traffic(os.path.join(ROOT, "profiles", f"stage_kernel_{workload}_{tag}_traffic.txt"))
    if rec is None or rec.get("source_sha256") != profiling.kernel_source_hash():
        return None
    v = rec.get(f"stage{stage}_bytes_per_launch")
    return float(v) if v is not None else None


def stream_bandwidth(R, torch, mib=1024, reps=10):
    """GB/s (bytes moved) of the library's streaming reference kernel -- one FP64 element per
    lane, non-temporal loads and stores, the sweeps' element width -- on arrays of `mib` MiB:
    copy (1 read, 1 write), read only, 2 reads + 1 write, 4 reads + 1 write; plus torch's
    device-to-device copy (the runtime's blit kernel, the known-size kernel the HBM byte
    counters are calibrated on)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(4 * n, dtype=torch.float64, device="cuda")
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, name, moved in ((0, "copy", 2), (1, "read", 1), (2, "add_2r1w", 3), (3, "sum_4r1w", 5)):
        rc, ms = R.relax_stream_probe(kind, src.data_ptr(), dst.data_ptr(), n, reps, stream)
        if rc != R.RELAX_OK:
            raise R.RelaxError(rc, "relax_stream_probe")
        out[name] = moved * 8 * n / (ms * 1e-3) / 1e9
    a = src[:n]
    dst.copy_(a)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    out["torch_copy"] = 16 * n / (start.elapsed_time(stop) * 1e-3 / reps) / 1e9
    del src, dst, a
    # the best rate of a kernel that both reads and writes: what a sweep can hope for
    out["read_write_ceiling"] = max(out["copy"], out["add_2r1w"], out["sum_4r1w"])
    return out


def adjoint_cost(R, torch, W, steps=200, every=20):
    """Reverse-mode cost on the braid gradient workload (64x64x192, twist amplitudes
    U(0.5, 1.5) with seed 4): K adaptive FP64 steps recording dt and checkpoints every
    `every` steps, then relax_backward of E_M(x_K) (which recomputes each segment)."""
    w = W.braid(64, 192, seed=4)
    cfg = R.make_config(w.grid, precision=R.RELAX_FP64, dt0=w.dt0, tol=w.tol, adaptive=True, record=True,
                        checkpoint_every=every)
    x0 = torch.from_numpy(w.x0).cuda()
    B0 = torch.from_numpy(w.B0).cuda()
    with R.Relaxation(cfg, x0, B0, K_record=steps) as r:  # first use: code objects loaded
        r.step(every, diag=False)
        r.backward(1.0, 0.0)
    with R.Relaxation(cfg, x0, B0, K_record=steps) as r:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.step(steps, diag=False)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        r.backward(1.0, 0.0)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    return {"workload": f"{w.name}, twist amplitudes U(0.5,1.5) seed 4", "steps": steps,
            "checkpoint_every": every, "forward_ms_per_step": tf * 1e3 / steps,
            "backward_ms_per_step": tb * 1e3 / steps, "backward_over_forward": tb / tf}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_step_times(oracle, w, dt, steps):
    """Wall seconds of each of `steps` fixed-dt oracle steps after one warm-up step, chained
    from x0 (each call takes one step from the previous one's positions)."""
    x = w.x0
    times = []
    for i in range(steps + 1):
        t0 = time.perf_counter()
        x = oracle.run(w.grid, x, w.B0, 1, dt=dt, mode=oracle.MODE_FIXED)["x"]
        if i > 0:
            times.append(time.perf_counter() - t0)
    return times


def cpu_baseline(W, w5, dt5, steps=5):
    """The oracle as it stands (OpenMP, FP64) on this host: the median of `steps` fixed-dt
    steps after one warm-up step, on the 256^3 benchmark box (the value) and on the 16^3 twist
    and the 64x64x192 braid; all host threads, and one thread on the two smaller grids."""
    import statistics

    import oracle
    nthreads = oracle.threads()
    res = {}
    cases = [("abc_256^3", w5, dt5, [nthreads]), ("single_twist_16^3", W.single_twist_16(), 1e-3, [nthreads, 1]),
             ("braid_64x64x192", W.braid(64, 192), 1e-2, [nthreads, 1])]
    t_all = time.perf_counter()
    for name, w, dt, thread_counts in cases:
        for th in thread_counts:
            oracle.set_threads(th)
            log(f"cpu baseline: oracle on {name}, {th} thread(s), {steps} + 1 steps")
            ts = _oracle_step_times(oracle, w, dt, steps)
            med = statistics.median(ts)
            res[f"{name}, {th} thread{'s' if th > 1 else ''}"] = {
                "updates_per_s": w.grid.N / med, "median_step_s": med, "steps_timed": steps, "threads": th}
    oracle.set_threads(nthreads)
    main = res[f"abc_256^3, {nthreads} thread{'s' if nthreads > 1 else ''}"]
    return {"value": main["updates_per_s"], "unit": "grid-point updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"median of {steps} fixed-dt Cash-Karp steps (dt {dt5:.3g}) of the full abc_256^3 grid "
                      f"after one warm-up step; {os.cpu_count()} host CPUs ({_cpu_model()})",
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(), "by_config": res,
            "total_s": time.perf_counter() - t_all}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis of the ABC box")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--dt0", type=float, default=1e-3)
    ap.add_argument("--cpu-steps", type=int, default=5, help="timed oracle steps per configuration")
    ap.add_argument("--accuracy-steps", type=int, default=20,
                    help="fixed-dt steps of the FP32-mixed vs FP64 comparison at identical t")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode cost figure")
    ap.add_argument("--curl", choices=["nn", "nnn"], default="nn",
                    help="nearest-neighbour loops (Sec. 2.2) or the octilateral current (Sec. 2.3, FP64 only)")
    args = ap.parse_args()
    if args.curl == "nnn" and args.precision != "fp64":
        print("bench.py --curl nnn: the octilateral current is FP64 only; timing FP64", file=sys.stderr)
        args.precision = "fp64"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the relaxation step has no multi-GPU path in this build "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1405_0942_amd as R
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    R.lib()  # fail loudly if the HIP library is missing
    stream = stream_bandwidth(R, torch)
    log("device streaming GB/s: " + ", ".join(f"{k} {v:.0f}" for k, v in stream.items()))
    log(f"building inputs abc_{args.n}^3")
    w = W.abc_box(args.n)
    res = {}
    curl = R.RELAX_CURL_NNN if args.curl == "nnn" else R.RELAX_CURL_NN
    if args.precision in ("fp64", "both"):
        res["fp64"] = run_precision(R, torch, w, R.RELAX_FP64, args.steps, args.warmup, args.tol, args.dt0, curl)
    if args.precision in ("mixed", "both"):
        res["mixed"] = run_precision(R, torch, w, R.RELAX_FP32_MIXED, args.steps, args.warmup, args.tol, args.dt0)
    main_key = "fp64" if "fp64" in res else "mixed"
    m = res[main_key]
    tag = "fp64" if main_key == "fp64" else "fp32-mixed"
    ceiling = stream["read_write_ceiling"]
    line = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_key == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: ABC field A=B=C=1 on the periodic box [0,2pi)^3, x0 = X + "
                               f"divergence-free |k|<=3 displacement (max 0.1, seed 5)",
                   "grid": list(w.grid.n), "step": "one accepted adaptive Cash-Karp RK5(4) step",
                   "current": ("octilateral loops over the eight ring neighbours (Sec. 2.3)" if args.curl == "nnn"
                               else "loops over the four nearest neighbours (Sec. 2.2)"),
                   "tol": args.tol, "rejects_in_timed_steps": m["rejects"],
                   "step_algorithmic_bytes_per_node": ALGO_STEP[tag],
                   "step_hbm_GBs_algorithmic": m["step_algorithmic_GBs"],
                   "step_hbm_frac": m["step_algorithmic_GBs"] / HBM_PEAK_GBS,
                   "step_frac_of_stream_ceiling": m["step_algorithmic_GBs"] / ceiling,
                   "step_hbm_GBs_design": m["step_design_GBs"]},
        "roofline": m["roofline"],
        "kernels": m["kernels"],
        "stream_GBs": stream,
    }
    if main_key == "fp64" and "mixed" in res:
        mm = res["mixed"]
        log(f"FP32-mixed vs FP64: {args.accuracy_steps} steps at the same fixed dt")
        # 1e-4 at 256^3, just below the explicit stability limit there; the limit scales as h^2
        acc = mixed_vs_fp64_fixed(R, torch, w, dt=1e-4 * (256.0 / args.n) ** 2, K=args.accuracy_steps)
        line["fp32_mixed"] = {"value": mm["value"], "ms_per_step": mm["ms_per_step"], "dtype": "f64+f32",
                              "rejects_in_timed_steps": mm["rejects"], "roofline": mm["roofline"],
                              "step_algorithmic_bytes_per_node": ALGO_STEP["fp32-mixed"],
                              "step_hbm_GBs_algorithmic": mm["step_algorithmic_GBs"],
                              "step_hbm_frac": mm["step_algorithmic_GBs"] / HBM_PEAK_GBS,
                              "step_hbm_GBs_design": mm["step_design_GBs"], "kernels": mm["kernels"],
                              "accuracy_vs_fp64_fixed_dt": acc}
    if not args.no_adjoint and args.curl == "nn":
        log("adjoint cost: braid 64x64x192, 200 steps, checkpoints every 20")
        line["adjoint"] = adjoint_cost(R, torch, W)
    if not args.no_cpu_baseline:
        # fixed steps of the size the adaptive GPU run settled to (dt0 itself is above the
        # explicit stability limit of the 256^3 grid)
        import oracle
        with oracle.curl(oracle.CURL_NNN if args.curl == "nnn" else oracle.CURL_NN):
            line["cpu_baseline"] = cpu_baseline(W, w, m["dt_last"], steps=args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
