#!/usr/bin/env python3
"""Throughput of the relaxation step on one MI355X: grid-point updates/s and HBM roofline.

Workload: the 256^3 periodic box [0, 2 pi)^3 holding the ABC Beltrami field (A = B = C = 1),
positions x0 = X + a seeded divergence-free Fourier displacement (|k| <= 3, max 0.1, seed 5).
A step is one accepted adaptive Cash-Karp RK5(4) step (six fused stage sweeps plus the
device step control; rejected attempts are redone inside and counted in the time).

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed|both]

Prints one JSON line.  value = N * accepted steps / wall time of the timed relax_step
call (inputs resident in HBM), FP64.  The FP32-mixed figures are in "fp32_mixed".
"roofline" is the dominant kernel's algorithmic bytes per launch over its average launch
duration (HIP events around each launch), against the 8 TB/s HBM3E peak.
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

# algorithmic HBM bytes per node of each stage sweep.  Both modes:
#   stage 1: x_n, B0 -> k_1
#   stage 2: x_n, k_1, B0, k_1 at the node -> k_2, y_3
#   stage 3: y_3, B0, k_1, k_2 at the node -> k_3, y_4
# FP64 (every vector 24 B):
#   stage 4: y_4, B0, k_1..k_3 at the node -> y_5 and the sums Y6, dX, E
#   stage 5: y_5, B0, Y6 and E at the node -> y_6, E
#   stage 6: y_6, B0, x_n, dX and E at the node -> x_{n+1}
# FP32-mixed (x_n, y_s in FP64; k_j and B0 in FP32):
#   stage s = 4, 5: y_s, B0, k_1..k_{s-1} at the node -> k_s, y_{s+1}
#   stage 6: y_6, B0, x_n, k_1, k_3, k_4, k_5 at the node -> x_{n+1}
BYTES_FP64 = [72, 144, 144, 216, 144, 144]
BYTES_MIXED = [48, 96, 96, 108, 120, 132]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(R, torch, w, precision, steps, warmup, tol, dt0):
    cfg = R.make_config(w.grid, precision=precision, dt0=dt0, tol=tol, adaptive=True)
    x0 = torch.from_numpy(w.x0).cuda()
    B0 = torch.from_numpy(w.B0).cuda()
    N = w.grid.N
    out = {}
    with R.Relaxation(cfg, x0, B0) as r:
        del x0, B0
        log(f"precision {precision}: warmup {warmup} steps")
        r.step(warmup, diag=False)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        log(f"precision {precision}: timed {steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(r.stream)
        diag = r.step(steps)
        stop.record(r.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms = start.elapsed_time(stop)
        rejects = sum(d["rejects"] for d in diag)
        # second pass with every launch bracketed by HIP events, for the per-kernel figures
        log(f"precision {precision}: profiled {steps} steps")
        r.profile(True)
        r.step(steps, diag=False)
        prof = r.profile(False)
        fin = r.diagnostics()
    bytes_node = BYTES_FP64 if precision == R.RELAX_FP64 else BYTES_MIXED
    kernels = {}
    for s in range(2, 7):  # stage 1 is skipped on retries, so its launch count overstates work
        ms, n = prof[f"stage{s}"]
        avg = ms / n
        gbs = bytes_node[s - 1] * N / (avg * 1e-3) / 1e9
        kernels[f"stage{s}"] = {"avg_ms": avg, "launches": n, "GB/s": gbs}
    ms1, n1 = prof["stage1"]
    kernels["stage1"] = {"total_ms": ms1, "launches": n1}
    kernels["control"] = {"total_ms": prof["control"][0], "launches": prof["control"][1]}
    dom = max((k for k in kernels if "avg_ms" in kernels[k]), key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    achieved = kernels[dom]["GB/s"]
    tag = "fp64" if precision == R.RELAX_FP64 else "fp32-mixed"
    traffic = measured_traffic(int(dom[-1]), tag, w.name.replace("^3", ""))
    # bytes per accepted step, rejected attempts included: each stage's bytes times its
    # launches per accepted step in the profiled pass (stage 1 runs once per accepted step)
    step_bytes = sum(bytes_node[s - 1] * (prof[f"stage{s}"][1] if s > 1 else steps) for s in range(1, 7)) / steps * N
    out.update(
        value=N * steps / wall,
        ms_per_step=wall * 1e3 / steps,
        event_ms_per_step=ev_ms / steps,
        rejects=rejects,
        dt_last=diag[-1]["dt"],
        xi_first=diag[0]["xi"],
        xi_last=diag[-1]["xi"],
        E_first=diag[0]["E_M"],
        E_last=diag[-1]["E_M"],
        fp64_final_xi=fin["xi"],
        step_GBs=step_bytes * steps / wall / 1e9,
        kernels=kernels,
        roofline={"bound": "hbm", "kernel": f"stage_kernel<{dom[-1]}> ({tag})",
                  "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "traffic": traffic, "algorithmic_bytes": bytes_node[int(dom[-1]) - 1] * N},
    )
    return out


def measured_traffic(stage, tag, workload):
    """HBM bytes per launch of stage_kernel<stage> from the committed FETCH_SIZE / WRITE_SIZE
    summary of this workload, or None when there is none or the kernel source changed since."""
    from paper_1405_0942_amd import profiling
    rec = profiling.read_traffic(os.path.join(ROOT, "profiles", f"stage_kernel_{workload}_{tag}_traffic.txt"))
    if rec is None or rec.get("source_sha256") != profiling.kernel_source_hash():
        return None
    v = rec.get(f"stage{stage}_bytes_per_launch")
    return float(v) if v is not None else None


def stream_bandwidth(torch, mib=1024, reps=5):
    """What plain streaming kernels reach on this device, GB/s of bytes moved: a device-to-
    device copy of `mib` MiB (the runtime's blit kernel, also the known-size kernel the HBM
    byte counters are calibrated on), a read-only sum and a two-read one-write add."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            fn()
        stop.record()
        torch.cuda.synchronize()
        return nbytes / (start.elapsed_time(stop) * 1e-3 / reps) / 1e9

    out = {"copy": rate(lambda: c.copy_(a), 16 * n), "read": rate(lambda: a.sum(), 8 * n),
           "add_2r1w": rate(lambda: torch.add(a, b, out=c), 24 * n)}
    del a, b, c
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


def cpu_baseline(w, steps, dt):
    import oracle
    log(f"cpu baseline: oracle, {steps} fixed-dt steps on the full grid, {oracle.threads()} threads")
    t0 = time.perf_counter()
    oracle.run(w.grid, w.x0, w.B0, steps, dt=dt, mode=oracle.MODE_FIXED)
    sec = time.perf_counter() - t0
    return {"value": w.grid.N * steps / sec, "unit": "grid-point updates/s", "cores": oracle.threads(),
            "kind": "oracle", "sample": f"{steps} fixed-dt Cash-Karp steps (dt {dt:.3g}) of the full "
                                        f"{w.name} grid ({sec:.1f} s wall)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis of the ABC box")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--dt0", type=float, default=1e-3)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode cost figure")
    args = ap.parse_args()

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
    stream = stream_bandwidth(torch)
    copy_gbs = stream["copy"]
    log("device streaming GB/s: " + ", ".join(f"{k} {v:.0f}" for k, v in stream.items()))
    log(f"building inputs abc_{args.n}^3")
    w = W.abc_box(args.n)
    res = {}
    if args.precision in ("fp64", "both"):
        res["fp64"] = run_precision(R, torch, w, R.RELAX_FP64, args.steps, args.warmup, args.tol, args.dt0)
    if args.precision in ("mixed", "both"):
        res["mixed"] = run_precision(R, torch, w, R.RELAX_FP32_MIXED, args.steps, args.warmup, args.tol, args.dt0)
    main_key = "fp64" if "fp64" in res else "mixed"
    m = res[main_key]
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
                   "tol": args.tol, "rejects_in_timed_steps": m["rejects"],
                   "step_hbm_GBs_algorithmic": m["step_GBs"],
                   "step_hbm_frac": m["step_GBs"] / HBM_PEAK_GBS},
        "roofline": m["roofline"],
        "kernels": m["kernels"],
        "copy_GBs": copy_gbs,
        "stream_GBs": stream,
    }
    if main_key == "fp64" and "mixed" in res:
        mm = res["mixed"]
        line["fp32_mixed"] = {"value": mm["value"], "ms_per_step": mm["ms_per_step"], "dtype": "f64+f32",
                              "rejects_in_timed_steps": mm["rejects"], "roofline": mm["roofline"],
                              "step_hbm_GBs_algorithmic": mm["step_GBs"], "kernels": mm["kernels"],
                              "E_last_rel_diff_vs_fp64": abs(mm["E_last"] - m["E_last"]) / abs(m["E_last"])}
    if not args.no_adjoint:
        log("adjoint cost: braid 64x64x192, 200 steps, checkpoints every 20")
        line["adjoint"] = adjoint_cost(R, torch, W)
    if not args.no_cpu_baseline:
        # the oracle takes fixed steps of the size the adaptive GPU run settled to (dt0 itself
        # is above the explicit stability limit of the 256^3 grid)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, dt=m["dt_last"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
