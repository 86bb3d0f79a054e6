"""Write the oracle's reference moments for the long parity checkpoints of the
benchmark workloads (test infrastructure; calls only the oracle and the
seeded workload generators).

  kh2d_256_v28      2-D Kelvin-Helmholtz layer, 256^2 cells x 28^2 velocities
                    (Kn 1e-4): moments after 50, 1000 and 2000 steps
  shear3d_16_v16_*  3-D sine-wave shear on 16^3 cells x 16^3 velocities,
                    Kn 1e-3, 1e-1 and 10: moments after 500 steps

Each file holds the moments (rho, u, T) of a seeded sample of cells (all
cells when there are at most 4096), the cell indices, the time step and the
step counts.  The GPU tests run the same workloads in the benchmark's launch
configuration and compare at those cells.

    python tests/golden/make_oracle_references.py [kh] [shear3d | shear3d:kn1e-3 ...] [--out DIR]
"""
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2208_09132_amd import workloads as wl  # noqa: E402
from tests.helpers import make_oracle, oracle_dt  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE = 4096


def _sample(N: int, seed: int) -> np.ndarray:
    if N <= SAMPLE:
        return np.arange(N)
    return np.sort(np.random.default_rng(seed).choice(N, SAMPLE, replace=False))


def run(name: str, prob: dict, checkpoints, seed: int, outdir: str = HERE) -> None:
    dt = oracle_dt(prob)
    o = make_oracle(prob, dt=dt)
    idx = _sample(o.N, seed)
    out = {"cells": idx, "dt": np.float64(dt), "checkpoints": np.array(checkpoints, dtype=np.int64)}
    done, t0 = 0, time.time()
    for k in checkpoints:
        while done < k:  # progress every 50 steps
            n = min(50, k - done)
            assert o.step(n) == 0
            done += n
            print(f"{name}: step {done} after {time.time() - t0:.0f} s", flush=True)
        rho, u, T = o.moments()
        out[f"rho_{k}"] = rho[idx]
        out[f"u_{k}"] = u[:, idx]
        out[f"T_{k}"] = T[idx]
        print(f"{name}: {k} steps after {time.time() - t0:.0f} s", flush=True)
        # partial file after each checkpoint (a long run can be resumed from scratch only)
        np.savez_compressed(os.path.join(outdir, f"oracle_{name}.npz"), **out,
                            complete=np.array(k == checkpoints[-1]))


SHEAR3D = {"kn1e-3": 1e-3, "kn1e-1": 1e-1, "kn10": 10.0}


def main(which, outdir=HERE):
    orc.build(force=False)
    if "kh" in which:
        run("kh2d_256_v28", wl.kelvin_helmholtz(), [50, 1000, 2000], seed=1, outdir=outdir)
    for tag, kn in SHEAR3D.items():
        if "shear3d" in which or f"shear3d:{tag}" in which:
            run(f"shear3d_16_v16_{tag}", wl.shear3d(n=16, nv=16, Kn=kn), [500], seed=2, outdir=outdir)


if __name__ == "__main__":
    args = sys.argv[1:]
    outdir = HERE
    if "--out" in args:
        k = args.index("--out")
        outdir = args[k + 1]
        del args[k:k + 2]
    main(args or ["kh", "shear3d"], outdir)
