"""GPU parity of the single-slope reconstruction option (the upwind cell's
limited slopes carried to the characteristic foot, without the slopes of the
slopes) against the FP64 oracle's same option, and the batched form with both
options in one batch (each problem bitwise equal to its solo run)."""
import sys

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle, moment_errors

pytestmark = pytest.mark.gpu
SS = "single_slope"


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _parity(prob, steps, tol):
    _log(f"single-slope parity: dim={prob['dim']} n={prob['n']} nv={prob['nv']} bc={prob['bc']} "
         f"storage={prob.get('storage')} steps={steps}")
    s = cd.Solver(prob)
    s.step(steps)
    got = s.moments()
    dt = s.dt
    s.close()
    o = make_oracle(prob, dt=dt_checked(prob, dt))
    assert o.step(steps) == 0
    errs = moment_errors(o.moments(), got, prob.get("gamma", 5.0 / 3.0), prob.get("R", 0.5))
    _log(f"  errors rho/u/T = {errs}")
    assert max(errs) <= tol, errs
    return got


def test_sod_full_run_fp64():
    _parity(wl.sod(reconstruction=SS), 1024, 1e-12)


def test_kelvin_helmholtz_reduced_fp64_and_fp32():
    p = wl.kelvin_helmholtz(n=40, nv=12, reconstruction=SS)
    got = _parity(p, 20, 1e-12)
    _parity(dict(p, storage="f32"), 20, 1e-5)
    # the option changes the answer (it is another reconstruction)
    ref = _parity(wl.kelvin_helmholtz(n=40, nv=12), 20, 1e-12)
    assert max(moment_errors(ref, got)) > 1e-8


def test_3d_ragged_outflow_fp64():
    rng = wl.SplitMix64(41)
    p = wl.random_fourier(3, [11, 9, 6], [6, 5, 6], rng, Kn=1e-2, reconstruction=SS)
    p["bc"] = ["periodic", "outflow", "periodic"]
    _parity(p, 5, 1e-12)


def test_dirichlet_sides_fp64():
    _parity(wl.sod(n=100, nv=24, boundary="dirichlet", reconstruction=SS), 200, 1e-12)


def test_kelvin_helmholtz_full_size_one_step_fp64():
    _parity(wl.kelvin_helmholtz(reconstruction=SS), 1, 1e-12)


def test_batched_mix_of_both_reconstructions_equals_alone_bitwise():
    rng = wl.SplitMix64(9)
    probs = [wl.random_fourier(2, [20, 18], [8, 8], rng, Kn=1e-2, reconstruction=SS),
             wl.random_fourier(2, [20, 18], [8, 8], rng, Kn=1e-2),
             wl.random_fourier(1, [130], [20], rng, Kn=1e-1, reconstruction=SS, storage="f32"),
             wl.sod(n=60, nv=16, boundary="dirichlet", reconstruction=SS)]
    steps = 7
    ref = []
    for p in probs:
        s = cd.Solver(p)
        s.step(steps)
        ref.append(s.moments())
        s.close()
    solvers = [cd.Solver(p) for p in probs]
    bt = cd.Batch(solvers, chunk_steps=3)
    bt.step(steps)
    bt.close()
    for k, (s, r) in enumerate(zip(solvers, ref)):
        got = s.moments()
        for a, c in zip(got, r):
            assert np.array_equal(a, c), f"problem {k} differs"
        s.close()
