"""The seeded workload generators against the recipes they state (CPU only).

Both the GPU path and the oracle take their inputs from these generators, so
a drift here would move every parity case and benchmark figure at once.  The
total update counts pinned below are the ones the benchmark's batched and
served legs report for these seeds.
"""
import math

import numpy as np
import pytest

from paper_2208_09132_amd import workloads as wl


def test_splitmix64_published_sequence():
    # the first outputs of SplitMix64 from state 0 (Steele, Lea & Flood 2014)
    r = wl.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_uniform_and_integer_ranges():
    r = wl.SplitMix64(7)
    u = np.array([r.uniform(-2.0, 3.0) for _ in range(20000)])
    assert u.min() >= -2.0 and u.max() < 3.0
    assert abs(u.mean() - 0.5) < 4 * 5.0 / math.sqrt(12 * 20000)
    k = np.array([r.integer(3, 9) for _ in range(20000)])
    assert set(k.tolist()) == set(range(3, 10))
    counts = np.bincount(k - 3)
    assert np.all(np.abs(counts - 20000 / 7) < 4 * math.sqrt(20000 / 7))


def test_kelvin_helmholtz_recipe():
    p = wl.kelvin_helmholtz()
    n = 256
    assert p["dim"] == 2 and p["n"] == [n, n] and p["nv"] == [28, 28]
    assert p["vmin"] == [-8.0, -8.0] and p["vmax"] == [8.0, 8.0] and p["bc"] == ["periodic"] * 2
    assert p["Kn"] == 1e-4 and p["cfl"] == 0.5 and p["steps"] == 2000
    x, y = wl.cell_centres(2, p["n"], p["lo"], p["hi"])
    inside = np.abs(y) < 0.25
    assert inside.sum() == n * n // 2
    np.testing.assert_array_equal(p["rho"], np.where(inside, 2.0, 1.0))
    np.testing.assert_array_equal(p["u"][0], np.where(inside, 0.5, -0.5))
    np.testing.assert_allclose(p["rho"] * p["R"] * p["T"], 2.0, rtol=1e-15)  # uniform pressure P = 2
    noise = p["u"][1] - 0.01 * np.sin(4.0 * math.pi * x)
    assert np.abs(noise).max() <= 1e-3 + 1e-17
    # one draw per cell in x-fastest order, from seed 2208
    r = wl.SplitMix64(2208)
    first = [r.uniform(-1e-3, 1e-3) for _ in range(3)]
    np.testing.assert_allclose(noise[:3], first, rtol=0, atol=1e-18)
    assert abs(noise.std() - 1e-3 / math.sqrt(3.0)) < 0.02 * 1e-3 / math.sqrt(3.0)


def test_random_fourier_field_is_normalised_and_periodic():
    r = wl.SplitMix64(3)
    coords = wl.cell_centres(2, [40, 40], [0.0, 0.0], [1.0, 1.0])
    s = wl.random_fourier_field(r, 2, coords)
    assert np.abs(s).max() <= 1.0
    # integer wave vectors: the field repeats with period 1 along each axis
    r2 = wl.SplitMix64(3)
    shifted = [coords[0] + 1.0, coords[1] - 2.0]
    np.testing.assert_allclose(wl.random_fourier_field(r2, 2, shifted), s, atol=1e-12)


def test_batched_workload_recipe():
    probs = wl.batched()
    assert len(probs) == 256
    ones = [p for p in probs if p["dim"] == 1]
    twos = [p for p in probs if p["dim"] == 2]
    assert len(ones) + len(twos) == 256
    assert abs(len(ones) - 128) < 4 * 8  # type is 1D with probability 1/2
    for p in ones:
        assert 64 <= p["n"][0] <= 1024 and 32 <= p["nv"][0] <= 128
    for p in twos:
        assert p["n"][0] == p["n"][1] and 32 <= p["n"][0] <= 256
        assert p["nv"][0] == p["nv"][1] and 16 <= p["nv"][0] <= 32
    for p in probs:
        D = p["dim"]
        assert 1e-4 <= p["Kn"] <= 10.0
        assert p["Pr"] in (0.5, 2.0 / 3.0, 1.0, 2.0)
        assert p["bc"] == ["periodic"] * D and p["vmin"] == [-6.0] * D and p["vmax"] == [6.0] * D
        assert p["storage"] == "f32"
        assert np.abs(p["rho"] - 1.0).max() <= 0.1 and np.abs(p["T"] - 1.0).max() <= 0.1
        assert np.abs(p["u"]).max() <= 0.1
    upd = sum(int(np.prod(p["n"])) * int(np.prod(p["nv"])) for p in probs)
    assert upd == 1_857_331_092
    # deterministic: the same seed gives the same problems
    again = wl.batched(count=4)
    for a, b in zip(probs[:4], again):
        np.testing.assert_array_equal(a["rho"], b["rho"])
        np.testing.assert_array_equal(a["u"], b["u"])


def test_served_stream_recipe():
    st = wl.served_stream()
    assert len(st) == 512
    t = np.array([a for a, _ in st])
    assert np.all(np.diff(t) > 0) and t[0] > 0
    # Poisson arrivals at 50/s: exponential gaps with mean 1/50
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.02) < 4 * 0.02 / math.sqrt(512)
    vortices = 0
    for _, p in st:
        assert p["dim"] == 2 and p["n"][0] == p["n"][1] and 64 <= p["n"][0] <= 512
        assert p["nv"][0] == p["nv"][1] and 16 <= p["nv"][0] <= 32
        assert 1e-4 <= p["Kn"] <= 1.0 and 200 <= p["steps"] <= 2000 and p["storage"] == "f32"
        if p["vmax"] == [10.0, 10.0]:  # Gresho vortex: rho = 1, peak speed 1
            vortices += 1
            np.testing.assert_array_equal(p["rho"], 1.0)
            assert np.hypot(p["u"][0], p["u"][1]).max() <= 1.0 + 1e-12
        else:
            assert p["vmax"] == [6.0, 6.0]
    assert abs(vortices - 256) < 4 * math.sqrt(128)
    upd = sum(int(np.prod(p["n"])) * int(np.prod(p["nv"])) * p["steps"] for _, p in st)
    assert upd == 29_936_943_442_053


@pytest.mark.parametrize("n,nv", [(16, 16), (64, 16)])
def test_shear3d_recipe(n, nv):
    p = wl.shear3d(n=n, nv=nv)
    x, y, z = wl.cell_centres(3, p["n"], p["lo"], p["hi"])
    assert p["vmin"] == [-6.0] * 3 and p["vmax"] == [6.0] * 3 and p["steps"] == 500
    np.testing.assert_array_equal(p["rho"], 1.0)
    np.testing.assert_array_equal(p["T"], 1.0)
    np.testing.assert_allclose(p["u"][0], 0.1 * np.sin(2.0 * math.pi * y), rtol=0, atol=0)
    assert not p["u"][1].any() and not p["u"][2].any()
