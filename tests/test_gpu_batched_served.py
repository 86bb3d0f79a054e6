"""GPU tests of the batched and served forms: every problem gives bitwise the
same result alone and in a mix; sampled problems (the batched workload's and
the served stream's own) match the oracle; the server admits by memory budget,
refuses invalid requests at submit and retires a request that fails on the
device without disturbing the others."""
import ctypes
import math
import sys
import time

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle, moment_errors

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def mixed_problems(seed=77, count=6):
    rng = wl.SplitMix64(seed)
    probs = []
    for k in range(count):
        if k % 2 == 0:
            p = wl.random_fourier(1, [rng.integer(40, 300)], [rng.integer(8, 33)], rng, Kn=10 ** rng.uniform(-3, 0),
                                  Pr=[0.5, 2.0 / 3.0, 1.0, 2.0][k % 4])
        else:
            n, m = rng.integer(12, 40), rng.integer(6, 12)
            p = wl.random_fourier(2, [n, n], [m, m], rng, Kn=10 ** rng.uniform(-3, 0), Pr=[2.0, 1.0, 0.5][k % 3])
        p["storage"] = "f32" if k % 3 == 1 else "f64"
        probs.append(p)
    return probs


def alone(prob, steps):
    s = cd.Solver(prob)
    s.step(steps)
    m = s.moments()
    s.close()
    return m


def test_batched_equals_alone_bitwise():
    probs = mixed_problems()
    steps = 13  # one 10-step graph chunk + an odd remainder
    ref = [alone(p, steps) for p in probs]
    solvers = [cd.Solver(p) for p in probs]
    b = cd.Batch(solvers, chunk_steps=10)
    b.step(steps)
    b.close()
    for k, (s, r) in enumerate(zip(solvers, ref)):
        got = s.moments()
        for a, c in zip(got, r):
            assert np.array_equal(a, c), f"problem {k} differs: {moment_errors(r, got)}"
        s.close()
    _log(f"batched: {len(probs)} problems bitwise equal to their solo runs")


def test_batched_with_dirichlet_problems_equals_alone_bitwise():
    """Problems with Dirichlet sides form their own class of the batch (the
    face-sum variant with boundary states); results stay bitwise equal."""
    probs = mixed_problems(seed=31, count=4)
    d1 = wl.sod(n=100, nv=24, boundary="dirichlet")
    d2 = wl.random_fourier(2, [20, 17], [6, 6], wl.SplitMix64(12), amp=0.2, Kn=1e-2)
    d2["bc"] = ["dirichlet", "periodic"]
    d2["dirichlet"] = [[[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]], None]
    d2["storage"] = "f32"
    probs += [d1, d2]
    steps = 7
    ref = [alone(p, steps) for p in probs]
    solvers = [cd.Solver(p) for p in probs]
    b = cd.Batch(solvers, chunk_steps=3)
    b.step(steps)
    b.close()
    for k, (s, r) in enumerate(zip(solvers, ref)):
        got = s.moments()
        for a, c in zip(got, r):
            assert np.array_equal(a, c), f"problem {k} differs"
        s.close()


def test_batched_sample_matches_oracle():
    probs = mixed_problems(seed=5, count=4)
    solvers = [cd.Solver(p) for p in probs]
    b = cd.Batch(solvers, chunk_steps=4)
    b.step(8)
    b.close()
    for p, s in zip(probs, solvers):
        got = s.moments()
        o = make_oracle(p, dt=dt_checked(p, s.dt))
        assert o.step(8) == 0
        errs = moment_errors(o.moments(), got)
        tol = 1e-12 if p["storage"] == "f64" else 1e-5
        _log(f"batched vs oracle: dim={p['dim']} storage={p['storage']} errs={errs}")
        assert max(errs) <= tol
        s.close()


def test_batched_workload_equals_alone_and_matches_oracle():
    """The benchmark's batched workload (256 uneven 1D/2D problems, FP32
    storage, one persistent launch per phase): every problem bitwise equal to
    its solo run after a 2-step graph chunk plus one step; 8 sampled problems
    (4 of each dimension, the cheapest for the CPU oracle) within 1e-5."""
    probs = wl.batched(count=256)
    steps = 3
    _log(f"batched workload: {len(probs)} problems, solo runs")
    ref = [alone(p, steps) for p in probs]
    solvers = [cd.Solver(p) for p in probs]
    b = cd.Batch(solvers, chunk_steps=2)
    b.step(steps)
    b.close()
    got = [s.moments() for s in solvers]
    dts = [s.dt for s in solvers]
    for s in solvers:
        s.close()
    for k, (g, r) in enumerate(zip(got, ref)):
        for a, c in zip(g, r):
            assert np.array_equal(a, c), f"problem {k} differs"
    cost = [int(np.prod(p["n"])) * int(np.prod(p["nv"])) for p in probs]
    sample = []
    for dim in (1, 2):
        idx = sorted((k for k, p in enumerate(probs) if p["dim"] == dim), key=lambda k: cost[k])
        sample += idx[:4]
    for k in sample:
        o = make_oracle(probs[k], dt=dt_checked(probs[k], dts[k]))
        assert o.step(steps) == 0
        errs = moment_errors(o.moments(), got[k])
        _log(f"batched workload vs oracle: problem {k} dim={probs[k]['dim']} errs={errs}")
        assert max(errs) <= 1e-5


def test_autotune_keeps_results():
    """The autotuner's choices (face-sum tile shape, update split, batched
    grid) change no result: a context created after tuning, which takes the
    tuned shapes, and the tuned context itself after its trial steps, give
    bitwise the results of untuned runs."""
    for p in (wl.kelvin_helmholtz(n=48, nv=10), wl.random_fourier(3, [20, 12, 12], [5, 5, 5], wl.SplitMix64(2),
                                                                    amp=0.2, Kn=1e-2, storage="f32")):
        a = cd.Solver(p)
        a.step(6)
        ref = a.moments()
        a.close()
        t = cd.Solver(p)
        t.autotune(2)  # advances by its trial steps
        _log(f"autotuned dim {p['dim']}: launch shape {t.launch_info()}")
        tuned_steps = t.info()[2]
        t.close()
        c = cd.Solver(p)  # picks the tuned shapes for this class
        c.step(6)
        got = c.moments()
        c.close()
        for x, y in zip(ref, got):
            assert np.array_equal(x, y)
        b = cd.Solver(p)
        b.step(tuned_steps + 6)
        ref2 = b.moments()
        b.close()
        t = cd.Solver(p)
        t.autotune(2)
        t.step(6)
        for x, y in zip(ref2, t.moments()):
            assert np.array_equal(x, y)
        t.close()
        # a batch whose update items take the split tuned for this class
        solvers = [cd.Solver(p), cd.Solver(mixed_problems(seed=5, count=2)[1])]
        ref3 = alone(solvers[1].prob, 6)
        b = cd.Batch(solvers, chunk_steps=4)
        b.step(6)
        b.close()
        for x, y in zip(ref, solvers[0].moments()):
            assert np.array_equal(x, y)
        for x, y in zip(ref3, solvers[1].moments()):
            assert np.array_equal(x, y)
        for sv in solvers:
            sv.close()


def test_server_results_equal_alone_and_budget_admission():
    probs = mixed_problems(seed=31, count=5)
    steps = [7, 12, 5, 9, 11]
    ref = [alone(p, n) for p, n in zip(probs, steps)]
    need = [cd.cdugks_required_bytes(p) for p in probs]
    budget = int(max(need) * 2.2)  # forces queueing: at most two or three at once
    srv = cd.Server(budget, max_active=3, chunk_steps=4)
    tickets = [srv.submit(p, n) for p, n in zip(probs, steps)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.005)
    assert len(done) == len(tickets)
    for t, r in zip(tickets, ref):
        rho, u, T, tq, ts = done[t]
        assert np.array_equal(rho, r[0]) and np.array_equal(u, r[1]) and np.array_equal(T, r[2])
        assert tq >= 0 and ts > 0
    # a request larger than the whole budget is refused up front
    big = wl.kelvin_helmholtz(n=128, nv=20)
    with pytest.raises(cd.CdugksError) as ei:
        srv.submit(big, 1)
    assert ei.value.code == cd.ERR_TOO_LARGE
    srv.close()


def _serve(srv, probs, steps, timeout=120.0):
    """Submit every problem, then poll until all are done; returns the poll
    results (or the CdugksError a failed request raised) by position."""
    tickets = [srv.submit(p, n) for p, n in zip(probs, steps)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < timeout:
        for k, t in enumerate(tickets):
            if k in done:
                continue
            try:
                r = srv.poll(t)
            except cd.CdugksError as e:
                r = e
            if r is not None:
                done[k] = r
        time.sleep(0.005)
    assert len(done) == len(tickets), f"{len(tickets) - len(done)} requests still pending"
    return [done[k] for k in range(len(tickets))]


def test_served_stream_requests_equal_alone_and_match_oracle():
    """The served workload's own requests: the first six of the seeded Poisson
    stream (Gresho vortices and random-Fourier states, 271^2..434^2 cells x
    16^2..30^2 velocities, FP32 storage), their step counts cut to 9..20 so
    that they end at different chunk boundaries, under a memory budget that
    admits only some at a time.  Each result is bitwise equal to the same
    request stepped alone, and the two cheapest (both vortices) match the FP64
    oracle within the FP32 tolerance, 1e-5."""
    stream = wl.served_stream(count=6)
    probs = [p for _, p in stream]
    steps = [20, 14, 17, 9, 12, 16]
    vortex = [k for k, p in enumerate(probs) if p["vmax"][0] == 10.0]
    assert len(vortex) >= 2
    need = [cd.cdugks_required_bytes(p) for p in probs]
    budget = int(max(need) * 1.5)  # the largest request fits, but never all at once
    assert sum(need) > budget
    _log(f"served stream prefix: {[p['n'][0] for p in probs]} cells per axis, budget {budget / 1e9:.1f} GB")
    solo, dts = [], []
    for p, n in zip(probs, steps):
        s = cd.Solver(p)
        s.step(n)
        solo.append(s.moments())
        dts.append(s.dt)
        s.close()
    srv = cd.Server(budget, max_active=4, chunk_steps=4)
    res = _serve(srv, probs, steps)
    srv.close()
    for k, (r, ref) in enumerate(zip(res, solo)):
        assert not isinstance(r, Exception), (k, r)
        rho, u, T, tq, ts = r
        assert np.array_equal(rho, ref[0]) and np.array_equal(u, ref[1]) and np.array_equal(T, ref[2]), k
        assert tq >= 0 and ts > 0
    cost = [int(np.prod(p["n"])) * int(np.prod(p["nv"])) * n for p, n in zip(probs, steps)]
    for k in sorted(range(len(probs)), key=lambda j: cost[j])[:2]:
        _log(f"  request {k}: oracle {probs[k]['n']} x {probs[k]['nv']}, {steps[k]} steps")
        o = make_oracle(probs[k], dt=dt_checked(probs[k], dts[k]))
        assert o.step(steps[k]) == 0
        errs = moment_errors(o.moments(), res[k][:3])
        _log(f"  request {k} ({'vortex' if k in vortex else 'random Fourier'}) vs oracle: errs={errs}")
        assert max(errs) <= 1e-5, (k, errs)


def _cold_request():
    """A state colder than the velocity grid resolves: every discrete
    equilibrium value underflows to zero, so the first step's face densities
    vanish and the step raises the non-physical flag on the device (the
    request is accepted at submit: its moments are valid)."""
    p = wl.random_fourier(2, [20, 20], [8, 8], wl.SplitMix64(3), amp=0.0, Kn=1e-2)
    p["T"] = np.full(400, 1e-4)
    p["u"] = np.stack([np.full(400, 0.3), np.full(400, 0.2)])
    return p


def test_server_isolates_a_request_failing_mid_run():
    """A request that turns non-physical on the device during its first chunk
    is retired with CDUGKS_ERR_NONPHYSICAL while the requests batched with it
    run on, bitwise equal to their solo runs."""
    good = mixed_problems(seed=9, count=3)
    bad = _cold_request()
    s = cd.Solver(bad)  # alone it fails the same way
    s.step(1)
    with pytest.raises(cd.CdugksError) as ei:
        s.sync()
    assert ei.value.code == cd.ERR_NONPHYSICAL
    s.close()
    probs = [good[0], bad, good[1], good[2]]
    steps = [9, 9, 6, 9]
    srv = cd.Server(1 << 34, max_active=4, chunk_steps=3)
    res = _serve(srv, probs, steps)
    srv.close()
    assert isinstance(res[1], cd.CdugksError) and res[1].code == cd.ERR_NONPHYSICAL, res[1]
    for k in (0, 2, 3):
        ref = alone(probs[k], steps[k])
        assert np.array_equal(res[k][0], ref[0]) and np.array_equal(res[k][2], ref[2]), k


def test_server_refuses_an_invalid_request_at_submit():
    good = mixed_problems(seed=9, count=3)
    bad = dict(good[0])
    bad["rho"] = good[0]["rho"].copy()
    bad["rho"][2] = -1.0
    srv = cd.Server(1 << 34, max_active=4, chunk_steps=3)
    tg = [srv.submit(p, 5) for p in good]
    with pytest.raises(cd.CdugksError) as ei:
        # the host validation refuses it at submit time
        srv.submit(bad, 5)
    assert ei.value.code == cd.ERR_INVALID
    for t, p in zip(tg, good):
        r = None
        t0 = time.time()
        while r is None and time.time() - t0 < 30:
            r = srv.poll(t)
            time.sleep(0.002)
        ref = alone(p, 5)
        assert np.array_equal(r[0], ref[0])
    srv.close()
