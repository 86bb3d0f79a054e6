"""GPU tests of the BF16-tail storage form (FP32 storage whose far velocity
tails, fixed at set-up, hold BF16): moments against the FP64 oracle within
the FP32 form's 1e-5, tail rows present and stored as BF16, the same result
alone and in a batch, and rows kept in FP32 identical to the FP32 form at
set-up."""
import sys

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle, moment_errors

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bf16_representable(x):
    """FP64 values that are exact BF16 numbers (zero low 16 bits as FP32)."""
    f = x.astype(np.float32)
    return np.all(f.astype(np.float64) == x) and np.all((f.view(np.uint32) & 0xFFFF) == 0)


def _parity(prob, steps, tol=1e-5):
    _log(f"bf16-tail parity: dim={prob['dim']} n={prob['n']} nv={prob['nv']} steps={steps}")
    s = cd.Solver(prob)
    tails, nbytes = s.storage_info()
    s.step(steps)
    got = s.moments()
    dt = s.dt
    s.close()
    o = make_oracle(prob, dt=dt_checked(prob, dt))
    assert o.step(steps) == 0
    errs = moment_errors(o.moments(), got, prob.get("gamma", 5.0 / 3.0), prob.get("R", 0.5))
    _log(f"  {tails} of {s.V} rows in BF16, state array {nbytes} bytes; errors rho/u/T = {errs}")
    assert tails > 0
    assert max(errs) <= tol, errs
    return got


def test_kelvin_helmholtz_reduced_within_1e5():
    p = wl.kelvin_helmholtz(n=40, nv=12, storage="f32_bf16tail")
    got = _parity(p, 20)
    # differs from the FP32 form (the tails are rounded) but only slightly
    q = dict(p, storage="f32")
    s = cd.Solver(q)
    s.step(20)
    ref = s.moments()
    s.close()
    d = max(moment_errors(ref, got))
    assert 0.0 < d <= 1e-5, d


def test_3d_small_within_1e5():
    p = wl.shear3d(n=12, nv=8, Kn=1e-1, storage="f32_bf16tail")
    _parity(p, 10)


def test_kelvin_helmholtz_full_size_one_step():
    """The benchmark's Kelvin-Helmholtz size in the BF16-tail form, one step
    against the FP64 oracle."""
    p = wl.kelvin_helmholtz(storage="f32_bf16tail")
    _parity(p, 1)


def test_tail_rows_hold_bf16_and_core_rows_match_fp32_form():
    p = wl.kelvin_helmholtz(n=24, nv=14, storage="f32_bf16tail")
    s = cd.Solver(p)
    tails, nbytes = s.storage_info()
    g, b = s.distributions()
    s.close()
    s32 = cd.Solver(dict(p, storage="f32"))
    g32, b32 = s32.distributions()
    _, nbytes32 = s32.storage_info()
    s32.close()
    assert 0 < tails < g.shape[0]
    assert nbytes < nbytes32
    is_tail = np.array([not np.array_equal(g[i], g32[i]) for i in range(g.shape[0])])
    # a row either equals the FP32 form's or is its BF16 rounding
    for i in range(g.shape[0]):
        if is_tail[i]:
            assert _bf16_representable(g[i]) and _bf16_representable(b[i])
            assert np.max(np.abs(g[i] - g32[i]) / np.abs(g32[i])) <= 2.0 ** -8
        else:
            assert np.array_equal(b[i], b32[i])
    assert is_tail.sum() == tails
    # the documented rule: nodes more than 4 sqrt(R T_max) from the box of
    # initial bulk velocities
    xi = np.linspace(-8.0, 8.0, 14)
    X, Y = np.meshgrid(xi, xi, indexing="xy")  # velocity index x fastest
    u = np.asarray(p["u"])
    gap = [np.maximum(0.0, np.maximum(u[d].min() - V, V - u[d].max())) for d, V in enumerate((X.ravel(), Y.ravel()))]
    rule = gap[0] ** 2 + gap[1] ** 2 > 16.0 * 0.5 * float(np.max(p["T"]))
    assert np.array_equal(is_tail, rule)


def test_batched_equals_alone_bitwise():
    rng = wl.SplitMix64(5)
    probs = [wl.random_fourier(2, [20, 20], [10, 10], rng, Kn=1e-2, storage="f32_bf16tail"),
             wl.random_fourier(1, [150], [24], rng, Kn=1e-1, storage="f32_bf16tail"),
             wl.random_fourier(2, [17, 23], [8, 8], rng, Kn=1e-3, storage="f32")]
    steps = 7
    ref = []
    for p in probs:
        s = cd.Solver(p)
        s.step(steps)
        ref.append(s.moments())
        s.close()
    solvers = [cd.Solver(p) for p in probs]
    assert solvers[0].storage_info()[0] > 0
    bt = cd.Batch(solvers, chunk_steps=3)
    bt.step(steps)
    bt.close()
    for k, (s, r) in enumerate(zip(solvers, ref)):
        got = s.moments()
        for a, c in zip(got, r):
            assert np.array_equal(a, c), f"problem {k} differs"
        s.close()
