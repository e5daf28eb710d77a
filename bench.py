"""Benchmark of one S2O4 step of the high-order isothermal GKS (HIP library, one MI355X).

Default workload: the channel-like flow, 192 x 96 x 96 cells, no-slip walls in y, periodic x and z,
constant pressure-gradient body force, FP32 storage and arithmetic with density stored as its
deviation from rho_ref. A step = ghost cells, CFL dt on the device, both S2O4 stages (reconstruction,
gas-kinetic flux, divergence, combination) and the body-force update. Inputs are resident in HBM
when the timed region starts. The FP64 run of the same case is timed too, and the FP32 result is
compared with it after the same number of steps.

Prints ONE JSON line (last line of stdout).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point operations (add, sub, mul = 1, FMA = 2, div / sqrt / exp / erf = 1) per
# cell and face direction, counted from the textbook formulation of the scheme (Jiang-Shu closed-form
# smoothness indicators shared by the two faces of a cell, one normalisation per evaluation point, the
# closed-form flux): reconstruction of the four variables (normal 111, t1 215, t2 430 per variable),
# flux at four Gauss points, divergence. It is a fixed unit of work: kernels that evaluate the same
# quantities with fewer operations do not change it.
FLOP_STAGE1_PER_CELL_DIR = 3692
FLOP_STAGE2_PER_CELL_DIR = 3592
FLOP_PER_CELL_STEP = 3 * (FLOP_STAGE1_PER_CELL_DIR + FLOP_STAGE2_PER_CELL_DIR) + 56
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # MI355X published vector peaks
PEAK_HBM_GBS = 8000.0

# HBM bytes per stage-1 face-pass launch (mean over the x, y, z launches) of the FP32 channel workload,
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
# "bench.py [--order 2] --steps 4 --warmup 2 --repeats 1 --no-fp64 --no-cpu-baseline --no-adjoint --no-bodies",
# each scaled by what the same counter reads for a plain 1 GiB device copy ("bench.py --calibrate-copy 1024":
# FETCH_SIZE x 2.0, WRITE_SIZE x 1.0). A figure belongs to the kernel sources it was measured on; bench
# reports null once they differ.
TRAFFIC = {
    5: {"sources": ("gks_stage.hip", "gks_device.h", "gks_internal.h"),
         "sources_sha256": "231c17131be534ff89f16fca6c5dd7cd445b185a47cac350e12eab1dbd2df8be",
         "fetch_bytes": 197_497_908, "write_bytes": 84_954_526},
    2: {"sources": ("gks_stage2.hip", "gks_device.h", "gks_internal.h"),
         "sources_sha256": "8d5906e99bf19247d8bea11a23e4b01fef46cdf6bf5fbb341931ecfb6df876bf",
         "fetch_bytes": 102_163_699, "write_bytes": 77_066_262},
}


def kernel_sources_sha256(order=5):
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC[order]["sources"]:
        with open(os.path.join(ROOT, "paper_2603_11102_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(case, precision, order=5):
    t = TRAFFIC[order]
    if case != "channel" or precision != "fp32" or t["sources_sha256"] != kernel_sources_sha256(order):
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def _time_steps(s, steps):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def _time_graph(s, steps, side):
    """Capture `steps` steps in one HIP graph and time a replay of it on the solver's stream."""
    import torch
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.step(steps)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(side):  # a replay runs on the current stream
        e0.record(side)
        g.replay()
        e1.record(side)
    e1.synchronize()
    return e0.elapsed_time(e1)


def stage1_launch_ms(timing):
    """Mean duration of one stage-1 face launch (x, y and z passes) from the per-launch event timing."""
    s1_ms = sum(timing[k][0] for k in ("s1x", "s1y", "s1z"))
    return s1_ms / max(1, sum(timing[k][1] for k in ("s1x", "s1y", "s1z")))


def run_gpu(cfg, precision, steps, warmup, graph=False, repeats=5):
    """Warm up, then time `repeats` windows of `steps` steps; returns the solver, the median window time,
    every window time (ms), the per-launch timing of one more window and the forces."""
    import statistics
    import torch
    from paper_2603_11102_amd import GksSolver
    side = torch.cuda.Stream() if graph else None
    if graph:
        with torch.cuda.stream(side):
            s = GksSolver(cfg, precision=precision)
    else:
        s = GksSolver(cfg, precision=precision)
    s.step(warmup)
    torch.cuda.synchronize()
    windows = [(_time_graph(s, steps, side) if graph else _time_steps(s, steps)) for _ in range(max(1, repeats))]
    ms = statistics.median(windows)
    torch.cuda.synchronize()
    s.set_timing(True)
    _time_steps(s, steps)
    timing = s.read_timing()
    s.set_timing(False)
    f = s.forces(check=False)
    return s, ms, windows, timing, f


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, planes):
    """Time the FP64 CPU oracle for one step on a bounded sample: the first `planes` z-planes of the same
    initial field, periodic in z (same spacing, same physics)."""
    import torch
    from oracle import Oracle
    sub = cfg if planes >= cfg.nz else cfg.with_(nz=planes, lz=cfg.dz * planes, q0=cfg.q0[:, :planes].copy())
    o = Oracle(sub)
    t0 = time.perf_counter()
    o.step()
    dt = time.perf_counter() - t0
    return {"value": sub.n_cells / dt, "unit": "cell-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model(),
            "sample": (f"1 S2O4 step of the FP64 oracle on the whole {sub.nx}x{sub.ny}x{sub.nz} field, {dt:.1f} s"
                       if sub is cfg else
                       f"1 S2O4 step of the FP64 oracle on {sub.nx}x{sub.ny}x{sub.nz} cells (first {planes} "
                       f"z-planes of the same field, periodic in z), {dt:.1f} s")}


def adjoint_ratio(steps_override=None):
    """Time of the discrete adjoint over the rotor-gradient window (recompute included) divided by the time
    of the FP64 forward window that stores the checkpoints, on the 128^3 rotor box."""
    import numpy as np
    import torch
    from paper_2603_11102_amd import GksSolver
    from synth import make_case
    cfg = make_case("adjoint")
    nsteps = steps_override or cfg.steps
    ones = torch.ones(cfg.rotor.n_act, dtype=torch.float64, device="cuda")
    w = GksSolver(cfg, precision="fp64")  # warm-up of every kernel of the forward and adjoint windows
    w.set_rotor(cfg.rotor, ones)
    w.set_checkpoints(1)
    w.step(1)
    w.adjoint(1, (1.0, 0.5))
    w.close()
    s = GksSolver(cfg, precision="fp64")
    s.set_rotor(cfg.rotor, ones)
    s.set_checkpoints(nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    g, _ = s.adjoint(nsteps, (1.0, 0.5))
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    ok = bool(torch.isfinite(g).all())
    return {"metric": "adjoint/forward time ratio", "value": t_adj / t_fwd, "unit": "ratio",
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"rotor box {cfg.nx}x{cfg.ny}x{cfg.nz}, {cfg.rotor.n_act} actuator points, "
                                   f"{nsteps} steps, gradient of mean power and thrust w.r.t. the point scalings"},
            "forward_s": t_fwd, "adjoint_s": t_adj, "gradient_finite": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--case", default="channel")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--accuracy-steps", type=int, default=100,
                    help="steps after which the FP32 field is compared with the FP64 one (at least the timed ones)")
    ap.add_argument("--cpu-planes", type=int, default=64,
                    help="z-planes of the field (from z = 0, periodic in z) the CPU oracle steps once")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--order", type=int, default=5, choices=(2, 5),
                    help="5: the high-order GKS (default); 2: the second-order variant (own JSON line)")
    ap.add_argument("--graph", action="store_true",
                    help="time the steps as one captured HIP graph replay (launch overheads removed)")
    ap.add_argument("--ibm-yaw", type=float, default=0.0, metavar="OMEGA",
                    help="turn the immersed tower and nacelle about the tower axis at OMEGA rad per unit time "
                         "(their supports are then rebuilt on the device every step)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio of the rotor-gradient window in the default line")
    ap.add_argument("--repeats", type=int, default=5, help="timed windows of --steps steps; value is their median")
    ap.add_argument("--no-bodies", action="store_true",
                    help="skip the companion timing of the rotor + tower/nacelle workload in the default line")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time the adjoint against its checkpointed forward window and print that line")
    args = ap.parse_args()
    if args.adjoint:
        r = adjoint_ratio()
        print(f"[bench] adjoint/forward: {r['value']:.3f} (forward {r['forward_s']:.3f} s, adjoint "
              f"{r['adjoint_s']:.3f} s)", flush=True)
        print(json.dumps(r), flush=True)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": n * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the x-slab multi-GPU "
              "decomposition is a design note only, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from synth import make_case
    cfg = make_case(args.case).with_(order=args.order)
    if args.ibm_yaw:
        if cfg.ibm is None or cfg.rotor is None:
            sys.exit("--ibm-yaw needs a workload with a rotor and immersed bodies (alm_ibm)")
        from synth.cases import IbmMotion, IbmSpec
        hub = cfg.rotor.hub
        axis = (hub[0] + 0.16 * 2.0 * cfg.rotor.radius, hub[1], 0.0)  # tower axis 0.16 D behind the rotor plane
        cfg = cfg.with_(ibm=IbmSpec(xyz=cfg.ibm.xyz, dS=cfg.ibm.dS,
                                    motion=IbmMotion(center=axis, omega=(0.0, 0.0, args.ibm_yaw))))
    print(f"[bench] case={args.case} order={args.order} grid={cfg.nx}x{cfg.ny}x{cfg.nz} precision={args.precision} "
          f"steps={args.steps} warmup={args.warmup}", flush=True)
    stretched = any(f is not None for f in (cfg.faces or ()))
    s, ms, windows, timing, f = run_gpu(cfg, args.precision, args.steps, args.warmup, graph=args.graph,
                                        repeats=args.repeats)
    n = cfg.n_cells
    value = n * args.steps / (ms * 1e-3)
    print(f"[bench] {args.precision}: {ms / args.steps:.3f} ms/step, {value:.4e} cell-updates/s", flush=True)
    print("[bench] per-category ms/step: " + ", ".join(f"{k}={v[0] / args.steps:.3f}" for k, v in timing.items()),
          flush=True)
    avg_launch_ms = stage1_launch_ms(timing)
    flops_launch = FLOP_STAGE1_PER_CELL_DIR * n
    achieved = flops_launch / (avg_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    es = 4 if args.precision == "fp32" else 8
    result = {
        "metric": "cell-updates/s per S2O4 step",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "timing": f"median of {len(windows)} timed windows of {args.steps} steps",
        "window_ms_per_step": [w / args.steps for w in windows],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.case} {cfg.nx}x{cfg.ny}x{cfg.nz} ({n} cells), "
                               f"{'FP32, density as deviation from rho_ref' if args.precision == 'fp32' else 'FP64'}",
                   "cells": n, "bc": list(cfg.bc), "ma": cfg.ma,
                   "launch": "one HIP graph replay of the timed steps" if args.graph else "eager",
                   **({"ibm_yaw_rad_per_time": args.ibm_yaw} if args.ibm_yaw else {})},
        "roofline": {"bound": "alu", "kernel": f"face_kernel<{'float' if args.precision == 'fp32' else 'double'}, 1, "
                                                f"3 | 0 | 4, {str(stretched).lower()}> (stage 1: mean over the x, y, z "
                                                "launches)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(args.case, args.precision, 5), "avg_launch_ms": avg_launch_ms,
                     "algorithmic_flop_per_launch": flops_launch},
        "per_category_ms_per_step": {k: v[0] / args.steps for k, v in timing.items()},
        "flop_per_cell_step": FLOP_PER_CELL_STEP,
    }
    if args.order == 2:
        # second-order variant: a few hundred flops per cell and direction against the same memory
        # traffic as the high-order pass, so the HBM roofline is the reference. Algorithmic bytes per
        # cell of a stage-1 launch (FP32): x and y read the field (16) and write L, L_t (32); z reads
        # the field, both residuals (64), Q^n and its low-order part (32) and writes Q*, S and their
        # low-order parts (64); FP64 has no low-order parts.
        per_cell = ((48 + 48 + 176) / 3.0) if args.precision == "fp32" else ((96 + 96 + 288) / 3.0)
        bytes_launch = per_cell * n
        result["metric"] = "cell-updates/s per S2O4 step (second-order variant)"
        result["config"]["workload"] += ", second-order GKS"
        result["roofline"] = {"bound": "hbm", "kernel": f"face2_kernel<{'float' if es == 4 else 'double'}, 1, "
                                                        f"3 | 0 | 4, {str(stretched).lower()}> (stage 1: mean over "
                                                        "the x, y, z launches)",
                              "achieved": bytes_launch / (avg_launch_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                              "unit": "GB/s", "frac": bytes_launch / (avg_launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                              "traffic": measured_traffic(args.case, args.precision, 2),
                              "avg_launch_ms": avg_launch_ms, "algorithmic_bytes_per_launch": bytes_launch}
    if args.precision == "fp32" and not args.no_fp64:
        s64, ms64, win64, timing64, _ = run_gpu(cfg, "fp64", args.steps, args.warmup, repeats=args.repeats)
        s64.close()
        del s64
        l64 = stage1_launch_ms(timing64)
        a64_tf = flops_launch / (l64 * 1e-3) / 1e12
        # accuracy: fresh FP32 and FP64 runs of exactly accuracy_steps steps from the same start
        from paper_2603_11102_amd import GksSolver
        a32, a64 = GksSolver(cfg, precision="fp32"), GksSolver(cfg, precision="fp64")
        a32.step(args.accuracy_steps)
        a64.step(args.accuracy_steps)
        done = args.accuracy_steps
        q32, q64 = a32.interior(), a64.interior()
        a32.close()
        a64.close()
        rl2 = [float(torch.linalg.vector_norm(q32[v] - q64[v]) / torch.linalg.vector_norm(q64[v])) for v in range(4)]
        result["fp64"] = {"value": n * args.steps / (ms64 * 1e-3), "ms_per_step": ms64 / args.steps,
                          "window_ms_per_step": [w / args.steps for w in win64],
                          "roofline": {"bound": "alu", "kernel": f"face_kernel<double, 1, 3 | 0 | 4, "
                                                                 f"{str(stretched).lower()}> (stage 1: mean over "
                                                                 "the x, y, z launches)",
                                       "achieved": a64_tf, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                       "frac": a64_tf / PEAK_TFLOPS["fp64"], "avg_launch_ms": l64}}
        result["fp32_vs_fp64_rel_l2"] = {"after_steps": done, "per_variable": rl2}
        print(f"[bench] fp64: {ms64 / args.steps:.3f} ms/step; fp32 vs fp64 rel L2 {rl2}", flush=True)
    s.close()
    del s
    if not args.no_bodies and args.case == "channel" and args.order == 5 and args.precision == "fp32":
        # companion line: the rotor and tower/nacelle workload, 512 x 256 x 256 cells, 192 actuator points
        # and 24,139 Lagrangian points, FP32 field with FP64 load reductions
        bcfg = make_case("alm_ibm")
        sb, msb, winb, timingb, fb = run_gpu(bcfg, "fp32", 10, 3, repeats=3)
        sb.close()
        del sb
        result["alm_ibm"] = {"workload": f"alm_ibm {bcfg.nx}x{bcfg.ny}x{bcfg.nz} ({bcfg.n_cells} cells), "
                                         f"{bcfg.rotor.n_act} actuator points, {bcfg.ibm.n} Lagrangian points, FP32",
                             "value": bcfg.n_cells * 10 / (msb * 1e-3), "unit": "cell-updates/s",
                             "ms_per_step": msb / 10, "window_ms_per_step": [w / 10 for w in winb],
                             "per_category_ms_per_step": {k: v[0] / 10 for k, v in timingb.items()},
                             "thrust": fb["thrust"], "power": fb["power"], "ibm_force": fb["ibm_force"]}
        print(f"[bench] alm_ibm fp32: {msb / 10:.3f} ms/step, alm {timingb['alm'][0] / 10:.3f} ms, "
              f"ibm {timingb['ibm'][0] / 10:.3f} ms", flush=True)
    if not args.no_adjoint and args.case == "channel" and args.order == 5 and args.precision == "fp32":
        # the third part of the metric: adjoint/forward time of the 128^3 rotor-gradient window (FP64)
        r = adjoint_ratio()
        result["adjoint_forward_ratio"] = {"value": r["value"], "forward_s": r["forward_s"],
                                           "adjoint_s": r["adjoint_s"], "workload": r["config"]["workload"]}
        print(f"[bench] adjoint/forward: {r['value']:.3f}", flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample ...", flush=True)
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_planes)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
