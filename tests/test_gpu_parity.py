"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative; u normwise, scaled by max(max|u|, sound speed at T=1)):
  FP64 storage  1e-12
  FP32 storage  1e-5
Cases span several tiles with ragged tails, odd velocity counts (a zero
velocity), outflow and periodic boundaries, Pr = 1, free streaming, and the
full Kelvin-Helmholtz size in the launch configuration the benchmark times.
"""
import math
import sys

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle, moment_errors, patch_problem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(prob, steps):
    s = cd.Solver(prob)
    s.step(steps)
    m = s.moments()
    dt = s.dt
    s.close()
    return m, dt


def oracle_run(prob, dt, steps):
    o = make_oracle(prob, dt=dt)
    assert o.step(steps) == 0
    return o.moments()


def check_parity(prob, steps, tol):
    _log(f"parity: dim={prob['dim']} n={prob['n']} nv={prob['nv']} bc={prob['bc']} storage={prob.get('storage')} steps={steps}")
    got, dt = gpu_run(prob, steps)
    # the oracle steps with its own CFL step, checked against the library's
    ref = oracle_run(prob, dt_checked(prob, dt), steps)
    errs = moment_errors(ref, got, prob.get("gamma", 5.0 / 3.0), prob.get("R", 0.5))
    _log(f"  errors rho/u/T = {errs}")
    assert max(errs) <= tol, errs
    return errs


def test_sod_full_run_fp64():
    p = wl.sod()
    check_parity(p, p["steps"], 1e-12)


def test_sod_dirichlet_full_run_fp64():
    """The paper's Sod set-up with Dirichlet ends, 1024 steps to t = 0.2."""
    check_parity(wl.sod(boundary="dirichlet"), 1024, 1e-12)


def test_dirichlet_sides_differing_from_the_interior():
    """Dirichlet states unlike the interior drive the boundary cells: a 1D
    free-streaming reservoir, 2D with a Dirichlet x axis beside periodic and
    outflow axes (ragged tiles, odd velocity count), FP32, and a 3D Dirichlet
    z axis."""
    p = wl.sod(n=300, nv=41, boundary="dirichlet")
    p["rho"], p["T"], p["u"] = np.ones(300), np.ones(300), np.zeros((1, 300))
    p["relax"], p["tau"] = "tau", math.inf
    p["dirichlet"] = [[[2.0, 0.0, 1.0], [0.7, -0.3, 1.4]]]
    check_parity(p, 150, 1e-12)
    q = wl.random_fourier(2, [21, 18], [7, 6], wl.SplitMix64(8), amp=0.2, Kn=1e-2)
    q["bc"] = ["dirichlet", "periodic"]
    q["dirichlet"] = [[[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]], None]
    check_parity(q, 20, 1e-12)
    r = wl.random_fourier(2, [19, 23], [6, 7], wl.SplitMix64(9), amp=0.2, Kn=1e-1)
    r["bc"] = ["outflow", "dirichlet"]
    r["dirichlet"] = [None, [[1.1, 0.0, 0.3, 1.0], [1.2, 0.1, -0.2, 1.3]]]
    check_parity(r, 15, 1e-12)
    r32 = dict(r, storage="f32")
    check_parity(r32, 15, 1e-5)
    t = wl.random_fourier(3, [9, 10, 11], [5, 5, 5], wl.SplitMix64(10), amp=0.2, Kn=1e-1)
    t["bc"] = ["periodic", "outflow", "dirichlet"]
    t["dirichlet"] = [None, None, [[1.2, 0.1, 0.0, 0.2, 1.1], [0.9, 0.0, -0.1, -0.2, 0.9]]]
    check_parity(t, 4, 1e-12)


def test_1d_periodic_ragged_odd_velocities():
    p = wl.random_fourier(1, [300], [33], wl.SplitMix64(41), amp=0.2, Kn=1e-2, Pr=2.0)
    check_parity(p, 30, 1e-12)


def test_2d_kelvin_helmholtz_reduced_fp64():
    p = wl.kelvin_helmholtz(n=40, nv=12)
    check_parity(p, 20, 1e-12)


def test_2d_outflow_rectangular_odd_velocities():
    p = wl.random_fourier(2, [37, 21], [9, 10], wl.SplitMix64(5), amp=0.2, Kn=3e-2)
    p["bc"] = ["outflow", "periodic"]
    check_parity(p, 15, 1e-12)


def test_2d_prandtl_one_and_free_streaming():
    p = wl.random_fourier(2, [20, 18], [10, 10], wl.SplitMix64(8), amp=0.2, Kn=1e-2, Pr=1.0)
    check_parity(p, 10, 1e-12)
    q = wl.random_fourier(2, [20, 18], [10, 10], wl.SplitMix64(8), amp=0.2, relax="tau", tau=math.inf)
    check_parity(q, 10, 1e-12)


def test_3d_small_fp64():
    p = wl.random_fourier(3, [10, 9, 12], [6, 6, 6], wl.SplitMix64(3), amp=0.2, Kn=1e-2)
    check_parity(p, 5, 1e-12)
    q = wl.random_fourier(3, [9, 9, 9], [5, 5, 5], wl.SplitMix64(4), amp=0.2, Kn=1e-1)
    q["bc"] = ["periodic", "outflow", "periodic"]
    check_parity(q, 4, 1e-12)


def test_3d_workload_velocity_grid_fp32():
    """The 3-D shear workload's 16^3 velocity grid on 16^3 cells (several
    tiles per axis), FP32 storage, Kn = 1e-3 and 1e-1, against the oracle."""
    p = wl.shear3d(n=16, nv=16, Kn=1e-3, storage="f32")
    check_parity(p, 30, 1e-5)
    q = wl.shear3d(n=16, nv=16, Kn=1e-1, storage="f32")
    check_parity(q, 10, 1e-5)


def test_3d_full_size_fp32_conservation_and_stationarity():
    """The 3-D workload at full size (64^3 cells x 16^3 velocities, FP32
    storage, the launch configuration the benchmark times): totals conserved
    to round-off; a uniform moving state leaves W bitwise unchanged."""
    p = wl.shear3d(storage="f32")
    _log("3-D full size: conservation")
    s = cd.Solver(p)
    W0 = s.conserved().sum(axis=0)
    s.step(3)
    W1 = s.conserved().sum(axis=0)
    s.close()
    assert np.max(np.abs(W1 - W0)) <= 1e-13 * np.max(np.abs(W0)) * math.sqrt(3) * 10
    u = dict(p)
    N = 64 ** 3
    u["rho"] = np.full(N, 1.2)
    u["T"] = np.full(N, 0.8)
    u["u"] = np.stack([np.full(N, 0.2), np.full(N, -0.1), np.full(N, 0.05)])
    _log("3-D full size: stationarity")
    s = cd.Solver(u)
    Wa = s.conserved()
    s.step(2)
    Wb = s.conserved()
    s.close()
    assert np.array_equal(Wa, Wb)


def test_3d_full_size_five_steps_at_a_cell():
    """The 3-D workload at full size (64^3 cells x 16^3 velocities) for 5
    steps, FP64, FP32 and BF16-tail storage, in the launch configuration the benchmark
    times, against the oracle at one cell: the oracle steps only the block of
    cells within 15 of it (the 5-step reach), with outflow ends, which gives
    that cell's full-grid result exactly (its CPU test pins this).  The cell
    sits where the shear gradient is largest, so the block wraps across the
    periodic y boundary."""
    p = wl.shear3d(storage="f64")
    centre = [37, 0, 21]
    steps = 5
    q, full_idx, local = patch_problem(p, centre, 3 * steps)
    _log(f"3-D full size at cell {centre}: oracle on a {q['n']} block, {steps} steps")
    ref = None
    for storage, tol in (("f64", 1e-12), ("f32", 1e-5), ("f32_bf16tail", 1e-5)):
        _log(f"  GPU {storage}, 64^3 x 16^3, {steps} steps")
        got, dt = gpu_run(dict(p, storage=storage), steps)
        if ref is None:
            # the block steps with the full problem's oracle-side step
            r = oracle_run(q, dt_checked(p, dt), steps)
            ref = (r[0][local], r[1][:, local], r[2][local])
        errs = moment_errors(ref, (got[0][full_idx], got[1][:, full_idx], got[2][full_idx]))
        _log(f"  {storage}: errors rho/u/T = {errs}")
        assert max(errs) <= tol, (storage, errs)


def test_3d_full_size_two_steps_at_sixteen_sampled_cells():
    """The 3-D workload at full size (64^3 x 16^3), 2 steps in the launch
    configuration the benchmark times, FP64 and FP32, against the oracle at 16
    seeded cells anywhere in the grid (periodic wraps included), each from the
    oracle on the 13^3 block within the 2-step reach of the cell."""
    p = wl.shear3d(storage="f64")
    steps = 2
    rng = wl.SplitMix64(3091)
    cells = [[rng.integer(0, 63) for _ in range(3)] for _ in range(16)]
    runs = {}
    for storage in ("f64", "f32"):
        _log(f"  GPU {storage}, 64^3 x 16^3, {steps} steps")
        runs[storage] = gpu_run(dict(p, storage=storage), steps)
    dt = dt_checked(p, runs["f64"][1])
    worst = {"f64": 0.0, "f32": 0.0}
    for centre in cells:
        q, full_idx, local = patch_problem(p, centre, 3 * steps)
        r = oracle_run(q, dt, steps)
        ref = (r[0][local], r[1][:, local], r[2][local])
        for storage, tol in (("f64", 1e-12), ("f32", 1e-5)):
            got = runs[storage][0]
            errs = moment_errors(ref, (got[0][full_idx], got[1][:, full_idx], got[2][full_idx]))
            worst[storage] = max(worst[storage], max(errs))
            assert max(errs) <= tol, (centre, storage, errs)
    _log(f"3-D full size at 16 sampled cells: largest errors {worst}")


@pytest.mark.parametrize("kn", [1e-1, 10.0])
def test_3d_full_size_other_knudsen_numbers_at_a_cell(kn):
    """The 3-D workload's other Knudsen numbers at full size (FP32 storage,
    2 steps) against the oracle on the 13^3 block within the 2-step reach of
    a corner cell (the block wraps across the periodic x and z ends)."""
    p = wl.shear3d(storage="f32", Kn=kn)
    centre, steps = [63, 31, 0], 2
    q, full_idx, local = patch_problem(p, centre, 3 * steps)
    _log(f"3-D full size, Kn {kn}, at cell {centre}: {steps} steps, oracle on a {q['n']} block")
    got, dt = gpu_run(p, steps)
    r = oracle_run(q, dt_checked(p, dt), steps)
    errs = moment_errors((r[0][local], r[1][:, local], r[2][local]),
                         (got[0][full_idx], got[1][:, full_idx], got[2][full_idx]))
    _log(f"  errors rho/u/T = {errs}")
    assert max(errs) <= 1e-5, errs


def test_fp32_storage_within_1e5():
    p = wl.kelvin_helmholtz(n=40, nv=12, storage="f32")
    check_parity(p, 20, 1e-5)
    q = wl.shear3d(n=12, nv=8, Kn=1e-1, storage="f32")
    check_parity(q, 10, 1e-5)


def test_velocity_slicing_does_not_change_results():
    p = wl.kelvin_helmholtz(n=32, nv=12)
    ms = []
    for sl in (1, 3, 16):
        q = dict(p, velocity_slices=sl)
        ms.append(gpu_run(q, 6)[0])
    for m in ms[1:]:
        assert max(moment_errors(ms[0], m)) <= 1e-13


def test_kelvin_helmholtz_full_size_one_step_fp64():
    """Benchmark configuration (256^2 cells x 28^2 velocities, FP64), same
    launch shape as bench.py: one step against the oracle."""
    p = wl.kelvin_helmholtz()
    check_parity(p, 1, 1e-12)


def test_kelvin_helmholtz_full_size_one_step_fp32():
    """The FP32-storage leg of the benchmark (same size), one step against the
    FP64 oracle."""
    p = wl.kelvin_helmholtz(storage="f32")
    check_parity(p, 1, 1e-5)


def test_kelvin_helmholtz_full_size_conservation_and_stationarity():
    p = wl.kelvin_helmholtz()
    s = cd.Solver(p)
    W0 = s.conserved().sum(axis=0)
    s.step(20)
    W1 = s.conserved().sum(axis=0)
    s.close()
    assert np.max(np.abs(W1 - W0)) <= 1e-13 * np.max(np.abs(W0)) * math.sqrt(20) * 10
    u = dict(p)
    N = 256 * 256
    u["rho"] = np.full(N, 1.5)
    u["T"] = np.full(N, 2.0)
    u["u"] = np.stack([np.full(N, 0.3), np.full(N, -0.2)])
    s = cd.Solver(u)
    Wa = s.conserved()
    s.step(4)
    Wb = s.conserved()
    s.close()
    assert np.array_equal(Wa, Wb)


def test_face_sum_tile_shapes_give_bitwise_equal_results():
    """Every face-sum tile shape a problem can use (cdugks_params.face_tile)
    gives bitwise the same result, on grids whose extents are not multiples
    of the tiles (ragged tiles in every shape); a non-default shape in a batch
    (which runs the default shape) too; and one non-default shape against
    the oracle."""
    cases = [(wl.kelvin_helmholtz(n=40, nv=12), 4, 5),
             (dict(wl.kelvin_helmholtz(n=40, nv=12), storage="f32"), 4, 5),
             (wl.random_fourier(3, [37, 9, 14], [5, 6, 5], wl.SplitMix64(6), amp=0.2, Kn=1e-2,
                                storage="f32"), 9, 3)]
    for p, nshapes, steps in cases:
        ref = None
        for k in range(1, nshapes + 1):
            q = dict(p, face_tile=k)
            try:
                s = cd.Solver(q)
            except cd.CdugksError as e:
                _log(f"  dim {p['dim']} {p['storage']}: shape {k} not available ({e})")
                continue
            assert s.launch_info()[0] == k
            s.step(steps)
            m = s.moments()
            s.close()
            _log(f"tile shape {k}: dim {p['dim']} {p['storage']} n={p['n']}")
            if ref is None:
                ref = m
            else:
                for a, b in zip(ref, m):
                    assert np.array_equal(a, b), (p["dim"], p["storage"], k)
    # a context with a non-default shape in a batch
    p = wl.kelvin_helmholtz(n=40, nv=12)
    solo = cd.Solver(dict(p, face_tile=2))
    solo.step(5)
    want = solo.moments()
    solo.close()
    a, b = cd.Solver(dict(p, face_tile=2)), cd.Solver(wl.sod(n=50, nv=16))
    bt = cd.Batch([a, b], chunk_steps=2)
    bt.step(5)
    bt.close()
    for x, y in zip(a.moments(), want):
        assert np.array_equal(x, y)
    a.close()
    b.close()
    check_parity(dict(p, face_tile=4), 5, 1e-12)


def _run_shape(p, shape, steps):
    s = cd.Solver(dict(p, face_tile=shape))
    assert s.launch_info()[0] == shape
    s.step(steps)
    m = s.moments()
    g, b = s.distributions()
    bf16 = s.storage_info()[0]
    s.close()
    return m, g, b, bf16


def test_zmarch_columns_equal_the_box_kernel_bitwise():
    """3-D face sums by z-marching columns (face values staged plane by plane,
    then their velocity sums in a second kernel) give bitwise the results of
    the box kernel that sums in registers: moments and distributions after a
    few steps, for FP64, FP32 and BF16-tail storage, ragged periodic and
    outflow grids, Dirichlet sides, the single-slope option and an external
    acceleration.  The default 3-D shape is a column; the other two columns
    take the problems without Dirichlet sides, acceleration or the option."""
    rng = wl.SplitMix64(44)
    base = wl.random_fourier(3, [21, 10, 13], [6, 5, 7], rng, amp=0.2, Kn=1e-2)
    out = dict(base, bc=["outflow", "periodic", "outflow"])
    bf = wl.random_fourier(3, [18, 9, 11], [10, 9, 10], rng, amp=0.2, Kn=1e-2, storage="f32_bf16tail")
    dirichlet = dict(base, bc=["periodic", "dirichlet", "dirichlet"],
                     dirichlet=[None, [[1.2, 0.1, -0.1, 0.05, 1.1], [0.9, -0.1, 0.05, 0.0, 0.8]],
                                [[1.0, 0.0, 0.1, -0.2, 1.3], [1.1, 0.05, 0.0, 0.1, 0.9]]])
    cases = [("periodic f64", base, (1, 7, 8, 9)), ("outflow f64", out, (1, 7, 8, 9)),
             ("outflow f32", dict(out, storage="f32"), (1, 7, 8, 9)), ("bf16 tails", bf, (1, 7, 9)),
             ("dirichlet f64", dirichlet, (1, 7)), ("dirichlet f32", dict(dirichlet, storage="f32"), (1, 7)),
             ("single slope", dict(out, reconstruction="single_slope"), (1, 7)),
             ("acceleration", dict(dirichlet, accel=[0.3, -0.8, 0.5]), (1, 7)),
             # one and two cells along z: the column's rings wrap or clamp
             # onto the same planes
             ("one plane", wl.random_fourier(3, [9, 7, 1], [5, 5, 4], rng, amp=0.2, Kn=1e-2), (1, 7, 8, 9)),
             ("two planes, outflow", dict(wl.random_fourier(3, [6, 11, 2], [4, 5, 5], rng, amp=0.2, Kn=1e-2),
                                          bc=["periodic", "outflow", "outflow"]), (1, 7, 8, 9))]
    for name, p, shapes in cases:
        ref = None
        for k in shapes:
            got = _run_shape(p, k, 4)
            _log(f"z-march vs box: {name} shape {k} n={p['n']} bf16 rows={got[3]}")
            if name == "bf16 tails":
                assert got[3] > 0
            if ref is None:
                ref = got
                continue
            for a, c in zip(ref[0], got[0]):
                assert np.array_equal(a, c), (name, k)
            assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2]), (name, k)
    # a column shape outside the default is refused for Dirichlet sides
    with pytest.raises(cd.CdugksError):
        cd.Solver(dict(dirichlet, face_tile=8))


def test_3d_one_and_two_cells_along_z():
    """3-D grids one and two cells thick along z (the z-marching column's
    rings then hold wrapped or clamped copies of the same planes) against the
    oracle."""
    rng = wl.SplitMix64(45)
    check_parity(wl.random_fourier(3, [9, 7, 1], [5, 5, 4], rng, amp=0.2, Kn=1e-2), 4, 1e-12)
    q = wl.random_fourier(3, [6, 11, 2], [4, 5, 5], rng, amp=0.2, Kn=1e-2)
    q["bc"] = ["periodic", "outflow", "outflow"]
    check_parity(q, 4, 1e-12)


def test_smallest_grids():
    """The smallest problems the library accepts: one cell (periodic, where
    every neighbour is the cell itself, and outflow), single-cell axes in 2-D
    and 3-D, two velocities per axis (on [-1.5, 1.5], so that the coarse
    velocity grids still carry transport).  Moments in FP64 against the
    oracle at 1e-12 and the FP32 form at 1e-5; a single cell has no gradient,
    so its moments stay put, and its g and b, which still relax, are compared
    element by element."""
    from tests.test_gpu_distributions import check_distributions

    rng = wl.SplitMix64(46)

    def small(dim, n, nv, bc, storage="f64"):
        p = wl.random_fourier(dim, n, nv, rng, amp=0.2, Kn=1e-1, storage=storage)
        p["bc"], p["vmin"], p["vmax"] = bc, [-1.5] * dim, [1.5] * dim
        return p

    for dim, n, nv, bc in [(1, [2], [2], ["periodic"]), (2, [1, 3], [2, 3], ["outflow", "periodic"]),
                           (2, [2, 1], [3, 2], ["periodic", "periodic"]),
                           (3, [2, 1, 3], [2, 3, 2], ["outflow", "periodic", "periodic"])]:
        check_parity(small(dim, n, nv, bc), 5, 1e-12)
    check_parity(small(2, [1, 3], [2, 3], ["periodic", "periodic"], "f32"), 5, 1e-5)
    for bc in ("periodic", "outflow"):
        p = small(1, [1], [3], [bc])
        start, _ = gpu_run(p, 0)
        got, _ = gpu_run(p, 5)
        for a, b in zip(got, start):
            assert np.array_equal(a, b)
        check_distributions(p)


def test_face_sum_tile_requests_outside_the_list_are_refused():
    p = wl.kelvin_helmholtz(n=24, nv=8)
    for bad in (-1, 5):
        with pytest.raises(cd.CdugksError) as ei:
            cd.Solver(dict(p, face_tile=bad))
        assert ei.value.code == cd.ERR_INVALID
    d = wl.sod(n=64, nv=16, boundary="dirichlet")  # 1-D has one shape
    with pytest.raises(cd.CdugksError):
        cd.Solver(dict(d, face_tile=2))
    q = wl.random_fourier(2, [21, 18], [7, 6], wl.SplitMix64(8), amp=0.2, Kn=1e-2)
    q["bc"] = ["dirichlet", "periodic"]
    q["dirichlet"] = [[[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]], None]
    with pytest.raises(cd.CdugksError) as ei:  # Dirichlet sides run the default shape only
        cd.Solver(dict(q, face_tile=2))
    assert "not available" in str(ei.value)
