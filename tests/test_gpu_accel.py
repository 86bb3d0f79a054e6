"""GPU parity of the external acceleration (Sec. 2: eqs. gPDE, bPDE, the
sources of eqs. gsource and bsource, the face moments of eqs. rhoubar and
rhoEbar), through the C ABI, against the FP64 oracle: moments within 1e-12
(FP64 storage) and 1e-5 (FP32), and g, b element by element within 1e-12 of
each velocity row's largest value.  Cases: 1-D free fall and the isothermal
atmosphere with Dirichlet ends, 2-D random periodic states with several
tiles and ragged edges, a 2-D Dirichlet side, 3-D FP64 and FP32 (the 3-D
update stores the next quarter-step fields, which carry the acceleration's
source).  In batches, the server and after autotuning, problems with an
acceleration (in classes of their own, beside problems without one) give
bitwise their solo results; a batch member also matches the oracle."""
import math
import sys
import time

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle, moment_errors
from tests.test_gpu_distributions import row_errors

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def parity(prob, steps, tol, distributions=False):
    _log(f"accel parity: dim={prob['dim']} n={prob['n']} nv={prob['nv']} bc={prob['bc']} "
         f"a={prob['accel']} storage={prob.get('storage')} steps={steps}")
    s = cd.Solver(prob)
    o = make_oracle(prob, dt=dt_checked(prob, s.dt))
    s.step(steps)
    assert o.step(steps) == 0
    errs = moment_errors(o.moments(), s.moments(), prob.get("gamma", 5.0 / 3.0), prob.get("R", 0.5))
    _log(f"  errors rho/u/T = {errs}")
    assert max(errs) <= tol, errs
    if distributions:
        g, b = s.distributions()
        og, ob, _ = o.state()
        eg, eb = row_errors(og, g), row_errors(ob, b)
        _log(f"  per-row relative errors g, b = {eg:.2e}, {eb:.2e}")
        assert eg <= 1e-12 and eb <= 1e-12
    s.close()


def test_1d_free_fall_and_atmosphere():
    p = wl.random_fourier(1, [300], [33], wl.SplitMix64(41), amp=0.2, Kn=1e-2)
    p["accel"] = [0.8]
    parity(p, 30, 1e-12, distributions=True)
    n = 200
    q = wl.sod(n=n, nv=64, boundary="dirichlet")
    x = (np.arange(n) + 0.5) / n
    q["rho"], q["T"], q["u"] = np.exp(-2.0 * x), np.ones(n), np.zeros((1, n))
    q["vmin"], q["vmax"] = [-8.0], [8.0]
    q["relax"], q["mu_ref"], q["T_ref"] = "mu", 1e-3, 1.0
    q["dirichlet"] = [[[1.0, 0.0, 1.0], [math.exp(-2.0), 0.0, 1.0]]]
    q["accel"] = [-1.0]
    parity(q, 100, 1e-12, distributions=True)


def test_2d_periodic_fp64_and_fp32():
    p = wl.random_fourier(2, [37, 21], [9, 10], wl.SplitMix64(5), amp=0.2, Kn=3e-2)
    p["accel"] = [0.6, -0.9]
    parity(p, 15, 1e-12, distributions=True)
    q = dict(wl.kelvin_helmholtz(n=40, nv=12), accel=[0.0, -0.5])
    parity(q, 20, 1e-12)
    parity(dict(q, storage="f32"), 20, 1e-5)
    parity(dict(q, storage="f32_bf16tail"), 20, 1e-5)


def test_2d_dirichlet_side():
    p = wl.random_fourier(2, [21, 18], [7, 6], wl.SplitMix64(8), amp=0.2, Kn=1e-2)
    p["bc"] = ["periodic", "dirichlet"]
    p["dirichlet"] = [None, [[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]]]
    p["accel"] = [0.3, -1.1]
    parity(p, 12, 1e-12, distributions=True)


def test_3d_fp64_and_fp32():
    p = wl.random_fourier(3, [17, 9, 11], [5, 6, 5], wl.SplitMix64(21), amp=0.2, Kn=3e-2)
    p["bc"] = ["outflow", "periodic", "periodic"]
    p["accel"] = [0.3, 0.8, -1.1]
    parity(p, 5, 1e-12, distributions=True)
    parity(dict(p, storage="f32"), 5, 1e-5)


def test_uniform_free_fall_momentum_exact_on_gpu():
    """A uniform state under a uniform acceleration stays uniform, keeps its
    mass bitwise and gains momentum rho a t (to rounding) on the GPU too."""
    n = 24
    p = wl.random_fourier(2, [n, n], [12, 12], wl.SplitMix64(1), amp=0.0, Kn=1e-2)
    N = n * n
    p["rho"], p["T"] = np.full(N, 1.3), np.full(N, 0.9)
    p["u"] = np.stack([np.full(N, 0.1), np.full(N, 0.2)])
    p["accel"] = [0.3, -0.7]
    s = cd.Solver(p)
    W0 = s.conserved()
    steps = 40
    s.step(steps)
    W = s.conserved()
    dt = s.dt
    s.close()
    assert np.array_equal(W[:, 0], W0[:, 0])
    assert np.array_equal(W, np.repeat(W[:1], N, axis=0))
    for d, (u0, a) in enumerate(((0.1, 0.3), (0.2, -0.7))):
        want = 1.3 * (u0 + steps * dt * a)
        assert abs(W[0, 1 + d] - want) <= 1e-13 * 1.3


def _accel_mix():
    """Problems with and without an acceleration: 1-D FP64 with Dirichlet
    ends, 2-D FP64 and FP32 (the FP32 batched tile shape differs from the
    solo one), 2-D BF16 tails, 3-D FP32 (stored quarter-step fields), and two
    without an acceleration."""
    a = wl.random_fourier(1, [130], [17], wl.SplitMix64(61), amp=0.2, Kn=1e-2)
    a["accel"] = [0.7]
    d = wl.sod(n=90, nv=20, boundary="dirichlet")
    d["accel"] = [-0.4]
    b = wl.random_fourier(2, [37, 21], [9, 10], wl.SplitMix64(62), amp=0.2, Kn=3e-2)
    b["accel"] = [0.6, -0.9]
    c = dict(wl.kelvin_helmholtz(n=40, nv=12), accel=[0.0, -0.5], storage="f32")
    e = dict(c, storage="f32_bf16tail", accel=[0.2, -0.3])
    f = wl.random_fourier(3, [17, 9, 11], [5, 6, 5], wl.SplitMix64(63), amp=0.2, Kn=3e-2)
    f.update(bc=["outflow", "periodic", "periodic"], accel=[0.3, 0.8, -1.1], storage="f32")
    g = wl.random_fourier(2, [24, 24], [8, 8], wl.SplitMix64(64), amp=0.2, Kn=1e-2)
    h = dict(wl.random_fourier(1, [100], [12], wl.SplitMix64(65), amp=0.2, Kn=1e-1), storage="f32")
    return [a, d, b, c, e, f, g, h]


def _alone(prob, steps):
    s = cd.Solver(prob)
    s.step(steps)
    m = s.moments()
    gb = s.distributions()
    s.close()
    return m, gb


def test_batched_acceleration_equals_alone_and_matches_oracle():
    probs = _accel_mix()
    steps = 9  # one 4-step graph chunk, twice, and a remainder
    ref = [_alone(p, steps) for p in probs]
    solvers = [cd.Solver(p) for p in probs]
    bt = cd.Batch(solvers, chunk_steps=4)
    bt.step(steps)
    bt.close()
    for k, (s, (m, gb)) in enumerate(zip(solvers, ref)):
        got = s.moments()
        for x, y in zip(got, m):
            assert np.array_equal(x, y), f"problem {k} moments differ: {moment_errors(m, got)}"
        for x, y in zip(s.distributions(), gb):
            assert np.array_equal(x, y), f"problem {k} distributions differ"
    _log(f"batched acceleration: {len(probs)} problems bitwise equal to their solo runs")
    # a batch member against the oracle (the 2-D FP64 problem)
    p, s = probs[2], solvers[2]
    o = make_oracle(p, dt=dt_checked(p, s.dt))
    assert o.step(steps) == 0
    errs = moment_errors(o.moments(), s.moments())
    _log(f"  batched 2-D FP64 member vs oracle: {errs}")
    assert max(errs) <= 1e-12, errs
    for s in solvers:
        s.close()


def test_served_acceleration_equals_alone():
    probs = _accel_mix()
    steps = [7, 5, 9, 6, 8, 4, 5, 7]
    ref = [_alone(p, n)[0] for p, n in zip(probs, steps)]
    need = [cd.cdugks_required_bytes(p) for p in probs]
    srv = cd.Server(int(max(need) * 3.5), max_active=4, chunk_steps=3)  # forces queueing
    tickets = [srv.submit(p, n) for p, n in zip(probs, steps)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.005)
    srv.close()
    assert len(done) == len(tickets)
    for k, (t, r) in enumerate(zip(tickets, ref)):
        rho, u, T, tq, ts = done[t]
        assert np.array_equal(rho, r[0]) and np.array_equal(u, r[1]) and np.array_equal(T, r[2]), k
    _log(f"served acceleration: {len(probs)} requests bitwise equal to their solo runs")


def test_autotuned_acceleration_keeps_results():
    """The autotuner takes problems with an acceleration (its update and
    batched-grid trials run batches of one): a context created after tuning
    and the tuned context itself give bitwise the results of untuned runs."""
    p = dict(wl.kelvin_helmholtz(n=40, nv=12), accel=[0.0, -0.5])
    ref, _ = _alone(p, 6)  # before tuning
    t = cd.Solver(p)
    t.autotune(2)  # advances by its trial steps
    n = t.info()[2]
    t.step(6)
    got_t = t.moments()
    t.close()
    _log(f"autotuned acceleration problem after {n} trial steps")
    got, _ = _alone(p, 6)  # takes the tuned shapes of this class
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
    ref_t, _ = _alone(p, n + 6)
    for x, y in zip(got_t, ref_t):
        assert np.array_equal(x, y)
    with pytest.raises(cd.CdugksError):  # acceleration with the single-slope option
        cd.Solver(dict(p, reconstruction="single_slope"))
