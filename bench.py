"""Benchmark of the CDUGKS time step on one MI355X.

Default workload: 2D Kelvin-Helmholtz layer, 256^2 cells x 28^2 velocities,
FP64 storage (the configuration the throughput metric is quoted on).  Prints
ONE JSON line: phase-space updates/s (one update = g and b advanced at one
(cell, velocity), Sec. 4 scaling figure), the dominant kernel against the
HBM roofline, the FP32-storage rate of the same workload, and the FP64 CPU
oracle timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config kh|sod|shear3d]
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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
# Algorithmic bytes per phase-space update: read g and b, write g and b.
ALGO_BYTES = {"f64": 32.0, "f32": 16.0}
# Per kernel: face sums read g, b; the update reads g, b and writes g, b.
KERNEL_BYTES = {"face_sums": {"f64": 16.0, "f32": 8.0}, "update": {"f64": 32.0, "f32": 16.0}}
PHASES = ["face_sums", "face_close", "cell_close", "update"]


def workload(name: str, storage: str):
    from paper_2208_09132_amd import workloads as wl
    if name == "kh":
        return "kh2d_256x256_v28x28", wl.kelvin_helmholtz(storage=storage)
    if name == "sod":
        return "sod1d_128_v64", wl.sod(storage=storage)
    if name == "shear3d":
        return "shear3d_64cube_v16cube_kn1e-3", wl.shear3d(storage=storage)
    raise SystemExit(f"unknown config {name}")


def time_gpu(prob, steps: int, warmup: int):
    import torch
    from paper_2208_09132_amd import cdugks as cd

    s = cd.Solver(prob, use_torch=True)
    N, V = s.N, s.V
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel durations from HIP events on the context's stream
    phase_ms = s.profile_phases(max(3, min(steps, 10)))
    s.close()
    return N, V, wall, phase_ms


def cpu_baseline(prob, budget_s: float = 20.0):
    """The FP64 oracle on the host cores: one step of the same workload (a
    smaller tile of cells when one full step would exceed the budget)."""
    from oracle import oracle as orc
    from tests.helpers import oracle_problem

    orc.build(force=False)
    q = oracle_problem(prob)
    o = orc.Oracle(q)
    o.init(prob["rho"], prob["u"], prob["T"])
    t0 = time.perf_counter()
    o.step(1)
    dt = time.perf_counter() - t0
    N = o.N * o.V
    return {"value": N / dt, "unit": "phase-space updates/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"1 step of the full {prob['n']} x {prob['nv']} workload, FP64, {dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="kh")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is a design note, "
              "not a code path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)

    name, prob = workload(args.config, "f64")
    N, V, wall, phase_ms = time_gpu(prob, args.steps, args.warmup)
    ups = N * V * args.steps / wall
    ms_step = 1e3 * wall / args.steps

    # dominant kernel: the update (reads and writes g, b)
    dom = int(np.argmax(phase_ms))
    dom_name = PHASES[dom]
    kb = KERNEL_BYTES.get(dom_name, {"f64": 0.0})["f64"]
    achieved = kb * N * V / (phase_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel_ms": float(phase_ms[dom]), "phase_ms": {k: float(v) for k, v in zip(PHASES, phase_ms)},
                "algorithmic_bytes_per_update": kb,
                "step_algorithmic_frac": ALGO_BYTES["f64"] * ups / 1e9 / HBM_PEAK_GBS}

    out = {"metric": "phase-space updates/s", "value": ups, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "cells": list(prob["n"]), "velocities": list(prob["nv"]),
                      "storage": "f64", "gamma": prob["gamma"], "Pr": prob["Pr"], "Kn": prob["Kn"]},
           "roofline": roofline}

    if not args.no_fp32:
        _, p32 = workload(args.config, "f32")
        N2, V2, wall2, ph2 = time_gpu(p32, args.steps, args.warmup)
        ups32 = N2 * V2 * args.steps / wall2
        out["fp32_store"] = {"value": ups32, "unit": "updates/s", "ms_per_step": 1e3 * wall2 / args.steps,
                             "speedup_vs_fp64": ups32 / ups,
                             "phase_ms": {k: float(v) for k, v in zip(PHASES, ph2)},
                             "step_algorithmic_frac": ALGO_BYTES["f32"] * ups32 / 1e9 / HBM_PEAK_GBS}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
