"""Benchmark of the CDUGKS time step on one MI355X.

Default workload: 2D Kelvin-Helmholtz layer, 256^2 cells x 28^2 velocities,
FP64 storage (the configuration the throughput metric is quoted on).  Prints
ONE JSON line: phase-space updates/s (one update = g and b advanced at one
(cell, velocity), Sec. 4 scaling figure), the dominant kernel against the
HBM roofline, the FP32-storage rate of the same workload, and the FP64 CPU
oracle timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config kh|sod|shear3d]

The default run also times the 3-D shear workload (64^3 cells x 16^3
velocities, FP32 storage) for a few steps, with its own roofline block.
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


# committed rocprofv3 traffic summaries, by (workload, storage, kernel)
TRAFFIC_PROFILES = {
    ("kh", "f64", "face_sums"): "hbm_traffic_face_sums_kh2d_256_v28_fp64.md",
    ("kh", "f64", "update"): "hbm_traffic_update_kh2d_256_v28_fp64.md",
    ("shear3d", "f32", "face_sums"): "hbm_traffic_face_sums_shear3d_64_v16_fp32.md",
    ("shear3d", "f32", "update"): "hbm_traffic_update_shear3d_64_v16_fp32.md",
    ("shear3d", "f64", "face_sums"): "hbm_traffic_face_sums_shear3d_64_v16_fp64.md",
    ("shear3d", "f64", "update"): "hbm_traffic_update_shear3d_64_v16_fp64.md",
}


def profiled_traffic(config: str, storage: str, kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel), or None
    when there is none for this workload, storage and kernel, or it was taken
    from other kernel sources."""
    from paper_2208_09132_amd import profiling as pf
    name = TRAFFIC_PROFILES.get((config, storage, kernel))
    rec = pf.load_record(os.path.join(ROOT, "profiles", name)) if name else None
    if rec is None or rec.get("digest") != pf.source_digest():
        return None
    return rec


def roofline_block(config: str, storage: str, N: int, V: int, phase_ms, ups: float):
    """The dominant kernel (longest average duration per step, from HIP events
    on the context's stream) against the HBM roofline: its algorithmic bytes
    per launch (the scheme's minimum share of that kernel: g, b read by the
    face sums; read and written by the update) over its duration."""
    dom = int(np.argmax(phase_ms))
    dom_name = PHASES[dom]
    kb = KERNEL_BYTES.get(dom_name, {storage: 0.0})[storage]
    achieved = kb * N * V / (phase_ms[dom] * 1e-3) / 1e9
    rec = profiled_traffic(config, storage, dom_name)
    return {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": rec["traffic_bytes"] if rec else None,
            "traffic_unit": "bytes per launch",
            "traffic_per_update": rec["traffic_bytes"] / (N * V) if rec else None,
            "kernel_ms": float(phase_ms[dom]), "phase_ms": {k: float(v) for k, v in zip(PHASES, phase_ms)},
            "algorithmic_bytes_per_update": kb, "units_per_launch": N * V,
            # the measured HBM traffic of the kernel over its duration
            "traffic_GBps": rec["traffic_bytes"] / (phase_ms[dom] * 1e-3) / 1e9 if rec else None,
            "traffic_frac": rec["traffic_bytes"] / (phase_ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS if rec else None,
            "step_algorithmic_frac": ALGO_BYTES[storage] * ups / 1e9 / HBM_PEAK_GBS}


def workload(name: str, storage: str):
    from paper_2208_09132_amd import workloads as wl
    if name == "kh":
        return "kh2d_256x256_v28x28", wl.kelvin_helmholtz(storage=storage)
    if name == "sod":
        return "sod1d_128_v64", wl.sod(storage=storage)
    if name == "shear3d":
        return "shear3d_64cube_v16cube_kn1e-3", wl.shear3d(storage=storage)
    raise SystemExit(f"unknown config {name}")


def workload_sized(name: str, storage: str, n: int):
    """The 3-D workload on n^3 cells (the baseline sample of the oracle)."""
    from paper_2208_09132_amd import workloads as wl
    if name != "shear3d":
        raise ValueError(name)
    return wl.shear3d(n=n, storage=storage)


def time_gpu(prob, steps: int, warmup: int, copy_calibration: bool = False):
    import torch
    from paper_2208_09132_amd import cdugks as cd

    torch.cuda.synchronize()
    t_init0 = time.perf_counter()
    s = cd.Solver(prob, use_torch=True)
    s.sync()
    t_init = time.perf_counter() - t_init0
    N, V = s.N, s.V
    bf16_rows = s.storage_info()[0]
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_read0 = time.perf_counter()
    s.moments()  # host copies of rho, u, T
    t_read = time.perf_counter() - t_read0
    # per-kernel durations from HIP events on the context's stream
    phase_ms = s.profile_phases(max(3, min(steps, 10)))
    if copy_calibration:
        # two dispatches of the library's storage-to-FP64 copy (N V values
        # each): a plain copy of known size for calibrating HBM counters
        s.distributions()
    s.close()
    # hand the arena back to the device, so that the next leg gets a fresh
    # allocation rather than a piece of this one's cached block (the 3-D FP32
    # face sums ran 1.9x slower in the reused block)
    torch.cuda.empty_cache()
    return N, V, wall, phase_ms, {"init_s": t_init, "moments_readback_s": t_read, "bf16_rows": bf16_rows}


def copy_ceiling(nbytes: int = 1 << 32):
    """Streaming bandwidth of a plain elementwise kernel (y = 1 * x over 4 GiB;
    read + write bytes / time): the practical HBM ceiling next to the 8 TB/s
    published peak."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def batched_run(count: int, chunk: int, warm_chunks: int = 1, timed_chunks: int = 1):
    """The uneven batch (1D and 2D random-Fourier problems, FP32), advanced as
    one batch: persistent launches per phase, HIP-graph chunks."""
    from paper_2208_09132_amd import cdugks as cd
    from paper_2208_09132_amd import workloads as wl

    probs = wl.batched(count=count)
    solvers = [cd.Solver(p) for p in probs]
    updates = sum(s.N * s.V for s in solvers)
    b = cd.Batch(solvers, chunk_steps=chunk)
    b.step(chunk * warm_chunks)
    for s in solvers:
        s.sync()
    t0 = time.perf_counter()
    b.step(chunk * timed_chunks)
    solvers[0].sync()
    wall = time.perf_counter() - t0
    b.close()
    for s in solvers:
        s.close()
    steps = chunk * timed_chunks
    return {"value": updates * steps / wall, "unit": "updates/s", "problems": count, "steps": steps,
            "updates_per_step": updates, "ms_per_step": 1e3 * wall / steps, "storage": "f32",
            "dims": {"1d": sum(p["dim"] == 1 for p in probs), "2d": sum(p["dim"] == 2 for p in probs)}}


def sequential_run(count: int, storage: str, steps: int = 50):
    """The same uneven problems as the batched leg, each advanced on its own
    with the plain single-problem step (one problem after another, the GPU
    synchronised in between): the per-problem execution that batching
    replaces."""
    from paper_2208_09132_amd import cdugks as cd
    from paper_2208_09132_amd import workloads as wl

    probs = wl.batched(count=count)
    total, updates = 0.0, 0
    for p in probs:
        q = dict(p)
        q["storage"] = storage
        s = cd.Solver(q)
        s.step(steps)  # warm-up (captures the step graph)
        s.sync()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        total += time.perf_counter() - t0
        updates += s.N * s.V * steps
        s.close()
    return {"value": updates / total, "unit": "updates/s", "problems": count, "steps": steps, "storage": storage}


def served_run(nreq: int, budget_gb: float = 200.0, max_active: int = 64, chunk: int = 100):
    """A prefix of the seeded Poisson stream (lambda = 50/s) submitted at its
    arrival times to the continuous-batching server."""
    from paper_2208_09132_amd import cdugks as cd
    from paper_2208_09132_amd import workloads as wl

    stream = wl.served_stream()[:nreq]
    srv = cd.Server(int(budget_gb * 1e9), max_active=max_active, chunk_steps=chunk)
    t0 = time.perf_counter()
    tickets, upd = [], 0
    for arrival, p in stream:
        while time.perf_counter() - t0 < arrival:
            time.sleep(min(0.001, max(0.0, arrival - (time.perf_counter() - t0))))
        tickets.append((srv.submit(p, p["steps"]), p))
        upd += int(np.prod(p["n"])) * int(np.prod(p["nv"])) * p["steps"]
    lat, qs, ss = [], [], []
    pending = dict(tickets)
    last = time.perf_counter()
    while pending:
        for t in list(pending):
            r = srv.poll(t)
            if r is not None:
                _, _, _, tq, ts = r
                qs.append(tq)
                ss.append(ts)
                lat.append(tq + ts)
                del pending[t]
        if time.perf_counter() - last > 30.0:  # progress for long streams
            last = time.perf_counter()
            print(f"served: {nreq - len(pending)}/{nreq} done after {last - t0:.0f} s", file=sys.stderr, flush=True)
        time.sleep(0.002)
    makespan = time.perf_counter() - t0
    srv.close()
    pct = lambda a, q: float(np.percentile(np.array(a), q))
    span = stream[-1][0] if stream else 0.0
    return {"requests": nreq, "throughput": upd / makespan, "unit": "updates/s", "makespan_s": makespan,
            "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99),
            "p50_queue_s": pct(qs, 50), "p99_queue_s": pct(qs, 99),
            "p50_service_s": pct(ss, 50), "p99_service_s": pct(ss, 99),
            "offered_updates_per_s": upd / span if span > 0 else None,
            "arrival_rate_per_s": 50.0, "budget_gb": budget_gb, "storage": "f32"}


# phase-space points the oracle's baseline may hold (its ghost-extended
# slope arrays grow as D^3 per point; the 2-D benchmark workload is 5.1e7)
CPU_SAMPLE_POINTS = 6.0e7
# timed oracle steps after one untimed warm-up step, cut short once the timed
# steps have taken CPU_SAMPLE_SECONDS (never fewer than CPU_MIN_STEPS)
CPU_TIMED_STEPS = 10
CPU_MIN_STEPS = 3
CPU_SAMPLE_SECONDS = 25.0


def cpu_baseline(config: str, prob):
    """The FP64 oracle on the host cores, timed over CPU_TIMED_STEPS steps
    after one warm-up step, on the same workload, or, when that is larger
    than CPU_SAMPLE_POINTS phase-space points, on the same workload with fewer
    cells (same velocity grid), halving the cells per axis."""
    from oracle import oracle as orc
    from tests.helpers import oracle_problem

    orc.build(force=False)
    sample = prob
    n = list(prob["n"])
    V = int(np.prod(prob["nv"]))
    while int(np.prod(n)) * V > CPU_SAMPLE_POINTS and max(n) > 4:
        n = [max(4, k // 2) for k in n]
        if config == "shear3d":
            sample = workload_sized(config, prob["storage"], n[0])
        else:
            break
    q = oracle_problem(sample)
    o = orc.Oracle(q)
    o.init(sample["rho"], sample["u"], sample["T"])
    o.step(1)  # warm-up: first touch of the arrays, thread start-up
    t0 = time.perf_counter()
    steps = 0
    while steps < CPU_TIMED_STEPS:
        if o.step(1) != 0:
            break
        steps += 1
        if steps >= CPU_MIN_STEPS and time.perf_counter() - t0 > CPU_SAMPLE_SECONDS:
            break
    dt = time.perf_counter() - t0
    N = o.N * o.V
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": N * steps / dt, "unit": "phase-space updates/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps (after 1 warm-up step) of the {'full ' if sample is prob else ''}"
                      f"{sample['n']} x {sample['nv']} workload, FP64, {dt:.2f} s wall",
            "steps": steps, "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": model, "host_cpus": os.cpu_count()}


def shear3d_leg(steps: int, warmup: int):
    """The 3-D shear workload (64^3 cells x 16^3 velocities, Kn 1e-3) in its
    own storage form, FP32 g and b with FP64 moments: updates/s and its
    dominant kernel against the roofline."""
    name, p = workload("shear3d", "f32")
    N, V, wall, ph, _ = time_gpu(p, steps, warmup)
    ups = N * V * steps / wall
    return {"workload": name, "value": ups, "unit": "updates/s", "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * wall / steps, "storage": "f32",
            "roofline": roofline_block("shear3d", "f32", N, V, ph, ups)}


def refit_leg(steps: int = 20, nv_to: int = 32):
    """Velocity-grid refit (cdugks_regrid, an adaptive velocity grid) of the
    KH state after a few steps, from 28^2 to nv_to^2 velocities on the same
    box, FP64: wall time of the call (a new context: allocation, set-up,
    the carried W and the refit kernels) and its algorithmic bytes (old g, b
    read once, new g, b written once)."""
    import torch
    name, p = workload("kh", "f64")
    s = _solver(p)
    s.step(steps)
    s.sync()
    q = dict(p, nv=[nv_to, nv_to])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.regrid(q)
    wall = time.perf_counter() - t0
    N, Vo, Vn = s.N, s.V, r.V
    r.close()
    s.close()
    torch.cuda.empty_cache()
    return {"workload": f"{name} -> {nv_to}x{nv_to} velocities", "storage": "f64", "cells": N,
            "velocities_from": Vo, "velocities_to": Vn, "wall_ms": 1e3 * wall,
            "algorithmic_bytes": 16 * N * (Vo + Vn)}


def _solver(prob):
    from paper_2208_09132_amd import cdugks as cd
    return cd.Solver(prob, use_torch=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU clock settles over the first ~20 steps (kernel traces show it)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="kh")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--batched-problems", type=int, default=256)
    ap.add_argument("--served-requests", type=int, default=16)
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip running the batched leg's problems one by one with the plain step")
    ap.add_argument("--shear3d-steps", type=int, default=10,
                    help="timed steps of the 3-D shear leg (FP32, 64^3 x 16^3); 0 skips it")
    ap.add_argument("--shear3d-warmup", type=int, default=5)
    ap.add_argument("--no-refit", dest="refit", action="store_false",
                    help="skip the velocity-grid refit leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run the library's FP64 distribution copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library steps a problem on one GPU; sharding over several GPUs is "
              "described in the design notes but not implemented (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)

    # the batched workload's problems one by one with the single-problem step
    # (run first, so that the last dispatches of the single-problem kernels in
    # a kernel trace are the headline workload's per-phase timing pass)
    sequential = {}
    if args.batched_problems > 0 and not args.no_sequential:
        for st in ("f64", "f32"):
            sequential[st] = sequential_run(args.batched_problems, st)

    # the single-slope reconstruction option (not the paper's), FP64, also
    # before the headline legs
    single_slope = None
    if not args.no_fp32:
        _, pss = workload(args.config, "f64")
        pss["reconstruction"] = "single_slope"
        N4, V4, wall4, ph4, _ = time_gpu(pss, args.steps, args.warmup)
        single_slope = {"value": N4 * V4 * args.steps / wall4, "unit": "updates/s",
                        "ms_per_step": 1e3 * wall4 / args.steps,
                        "phase_ms": {k: float(v) for k, v in zip(PHASES, ph4)}}

    name, prob = workload(args.config, "f64")
    N, V, wall, phase_ms, io = time_gpu(prob, args.steps, args.warmup, args.copy_calibration)
    ups = N * V * args.steps / wall
    ms_step = 1e3 * wall / args.steps

    # dominant kernel: the phase with the longest average duration
    roofline = roofline_block(args.config, "f64", N, V, phase_ms, ups)
    achieved = roofline["achieved"]

    out = {"metric": "phase-space updates/s", "value": ups, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "cells": list(prob["n"]), "velocities": list(prob["nv"]),
                      "storage": "f64", "gamma": prob["gamma"], "Pr": prob["Pr"], "Kn": prob["Kn"]},
           "roofline": roofline,
           # the boundary takes host moments at init and returns host moments:
           # the same K steps with that traffic counted (never `value`)
           "host_boundary": dict(io, pcie_inclusive_updates_per_s=N * V * args.steps /
                                 (wall + io["init_s"] + io["moments_readback_s"]))}

    if not args.no_fp32:
        _, p32 = workload(args.config, "f32")
        N2, V2, wall2, ph2, _ = time_gpu(p32, args.steps, args.warmup)
        ups32 = N2 * V2 * args.steps / wall2
        out["fp32_store"] = {"value": ups32, "unit": "updates/s", "ms_per_step": 1e3 * wall2 / args.steps,
                             "speedup_vs_fp64": ups32 / ups,
                             "phase_ms": {k: float(v) for k, v in zip(PHASES, ph2)},
                             "step_algorithmic_frac": ALGO_BYTES["f32"] * ups32 / 1e9 / HBM_PEAK_GBS}
        # FP32 with the far velocity tails in BF16 (rows fixed at set-up)
        _, pt = workload(args.config, "f32_bf16tail")
        N3, V3, wall3, ph3, io3 = time_gpu(pt, args.steps, args.warmup)
        ups3 = N3 * V3 * args.steps / wall3
        out["fp32_bf16tail_store"] = {"value": ups3, "unit": "updates/s", "ms_per_step": 1e3 * wall3 / args.steps,
                                      "speedup_vs_fp64": ups3 / ups, "speedup_vs_fp32": ups3 / ups32,
                                      "bf16_rows": io3["bf16_rows"], "rows": V3,
                                      "phase_ms": {k: float(v) for k, v in zip(PHASES, ph3)}}
    if single_slope is not None:
        single_slope["speedup_vs_fp64"] = single_slope["value"] / ups
        out["single_slope_fp64"] = single_slope
    if args.batched_problems > 0:
        out["batched"] = batched_run(args.batched_problems, chunk=100)
        out["batched"]["speedup_vs_fp64_plain"] = out["batched"]["value"] / ups
        for st, seq in sequential.items():
            out["batched"][f"same_problems_one_by_one_{st}"] = seq
            out["batched"][f"speedup_vs_same_problems_one_by_one_{st}"] = out["batched"]["value"] / seq["value"]
    if args.served_requests > 0:
        out["served"] = served_run(args.served_requests)
    if args.config != "shear3d" and args.shear3d_steps > 0:
        out["shear3d_fp32"] = shear3d_leg(args.shear3d_steps, args.shear3d_warmup)
    if args.config == "kh" and args.refit:
        out["refit"] = refit_leg()
    out["copy_ceiling_GBps"] = copy_ceiling()
    out["roofline"]["frac_of_copy_ceiling"] = achieved / out["copy_ceiling_GBps"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.config, prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
