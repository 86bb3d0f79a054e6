"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, the ctypes structs match the C layout, and host validation
rejects bad problems before touching a GPU."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdugks.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cdugks_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = cd.load_library()
    names = declared_functions()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", cd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (cdugks_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cdugks.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(cdugks_space), '
                   'sizeof(cdugks_velocity), sizeof(cdugks_params), offsetof(cdugks_params, storage), '
                   'offsetof(cdugks_space, bc), offsetof(cdugks_velocity, quadrature)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    import ctypes
    assert vals == [ctypes.sizeof(cd.cdugks_space), ctypes.sizeof(cd.cdugks_velocity),
                    ctypes.sizeof(cd.cdugks_params), cd.cdugks_params.storage.offset,
                    cd.cdugks_space.bc.offset, cd.cdugks_velocity.quadrature.offset]


def test_required_bytes_scales_with_storage():
    p64 = wl.kelvin_helmholtz(n=64, nv=12)
    p32 = dict(p64, storage="f32")
    b64, b32 = cd.cdugks_required_bytes(p64), cd.cdugks_required_bytes(p32)
    NV = 64 * 64 * 144
    assert b64 >= 4 * NV * 8 and b32 >= 4 * NV * 4
    assert b64 - b32 >= 4 * NV * 4 * 0.99


@pytest.mark.parametrize("change,msg", [
    (dict(gamma=1.8), "gamma"), (dict(gamma=1.0), "gamma"), (dict(Pr=0.0), "Pr"), (dict(R=-1.0), "R"),
    (dict(quad="boole"), "Boole"), (dict(cfl=1.5), "cfl"), (dict(dt=1.0), "CFL"), (dict(Kn=0.0), "Kn"),
])
def test_validation_rejects_bad_parameters(change, msg):
    p = wl.sod(n=16, nv=10)
    p.update(change)
    with pytest.raises(cd.CdugksError) as ei:
        cd.cdugks_init(p)
    assert ei.value.code == cd.ERR_INVALID
    assert msg.lower() in str(ei.value).lower()


def test_validation_rejects_nonphysical_moments():
    p = wl.sod(n=16, nv=10)
    p["T"] = p["T"].copy()
    p["T"][3] = -1.0
    with pytest.raises(cd.CdugksError) as ei:
        cd.cdugks_init(p)
    assert ei.value.code == cd.ERR_INVALID
    p = wl.sod(n=16, nv=10)
    p["rho"] = p["rho"].copy()
    p["rho"][0] = math.nan
    with pytest.raises(cd.CdugksError):
        cd.cdugks_init(p)


def test_sizes_beyond_the_index_ranges_are_rejected():
    """Faces >= 2^31 or cells x velocities > 2^40 exceed the kernels' index
    arithmetic: refused before any allocation (the arrays here are never
    built; only the description is)."""
    for n, nv in (([1 << 16, 1 << 16], [4, 4]), ([1 << 12, 1 << 12], [1024, 1024])):
        p = {"dim": 2, "n": n, "lo": [0.0, 0.0], "hi": [1.0, 1.0], "bc": ["periodic", "periodic"],
             "nv": nv, "vmin": [-6.0, -6.0], "vmax": [6.0, 6.0], "relax": "mu", "mu_ref": 1e-3}
        with pytest.raises(cd.CdugksError) as ei:
            cd.cdugks_required_bytes(p)
        assert ei.value.code == cd.ERR_INVALID
        assert "too large" in str(ei.value)


def test_degenerate_descriptions_are_rejected():
    """Empty grids (no cells along an axis), fewer than two velocities on an
    axis, an empty domain or velocity box and an unsupported dimension are
    refused with ERR_INVALID before anything is allocated."""
    base = {"dim": 1, "n": [128], "lo": [0.0], "hi": [1.0], "bc": ["periodic"], "nv": [16], "vmin": [-6.0],
            "vmax": [6.0], "relax": "mu", "mu_ref": 1e-3}
    three = {"dim": 3, "n": [4, 4, 4], "lo": [0.0] * 3, "hi": [1.0] * 3, "bc": ["periodic"] * 3, "nv": [4, 4, 4],
             "vmin": [-6.0] * 3, "vmax": [6.0] * 3, "relax": "mu", "mu_ref": 1e-3}
    bad = [dict(base, n=[0]), dict(base, n=[-3]), dict(base, nv=[1]), dict(base, nv=[0]), dict(base, hi=[0.0]),
           dict(base, vmax=[-6.0]), dict(base, dim=0), dict(three, n=[4, 4, 0]), dict(three, nv=[4, 1, 4])]
    for p in bad:
        with pytest.raises(cd.CdugksError) as ei:
            cd.cdugks_required_bytes(p)
        assert ei.value.code == cd.ERR_INVALID
    # the smallest accepted: one cell, two velocities
    assert cd.cdugks_required_bytes(dict(base, n=[1], nv=[2])) > 0


def test_long_velocity_axes_are_accepted():
    """One axis may carry up to 2^24 - 1 velocities (the Sec. 3 sine-wave
    problem uses 16385); the total count and the product with the cells are
    what the index ranges bound."""
    base = {"dim": 1, "n": [128], "lo": [0.0], "hi": [1.0], "bc": ["periodic"], "vmin": [-6.0],
            "vmax": [6.0], "relax": "mu", "mu_ref": 1e-3, "quad": "boole"}
    assert cd.cdugks_required_bytes(dict(base, nv=[16385])) > 2 * 128 * 16385 * 8
    with pytest.raises(cd.CdugksError) as ei:
        cd.cdugks_required_bytes(dict(base, nv=[(1 << 24) + 1]))
    assert ei.value.code == cd.ERR_INVALID


def test_null_context_is_rejected():
    lib = cd.load_library()
    assert lib.cdugks_step(None, 1) == cd.ERR_INVALID
    assert lib.cdugks_sync(None) == cd.ERR_INVALID
    lib.cdugks_destroy(None)  # NULL-safe


def test_refit_and_grid_fit_validate_their_arguments():
    import ctypes
    lib = cd.load_library()
    p = wl.sod(n=16, nv=8)
    sp, ve, pa = cd.describe(p)
    out = ctypes.c_void_p()
    # no source context / no output pointer
    assert lib.cdugks_regrid(None, ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa), None, None, 0,
                             ctypes.byref(out)) == cd.ERR_INVALID
    assert lib.cdugks_regrid(None, ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa), None, None, 0,
                             None) == cd.ERR_INVALID
    # the grid fit is host arithmetic: a Boole grid has 4n + 1 nodes
    q = cd.fit_velocity(p, p["rho"], p["u"], p["T"], 1e-9, quad="boole")
    assert (q["nv"][0] - 1) % 4 == 0 and q["vmin"][0] < 0.0 < q["vmax"][0]
    with pytest.raises(cd.CdugksError) as ei:
        cd.fit_velocity(p, p["rho"], p["u"], p["T"], 2.0)
    assert ei.value.code == cd.ERR_INVALID


@pytest.mark.gpu
def test_destroying_a_batched_context_is_refused():
    """cdugks_destroy of a context that belongs to a live batch leaves it
    intact (the batch's graphs refer to its memory) and sets the error text;
    the batch still steps, and after the batch is gone the context gives the
    same result as a solo run of the same steps."""
    p = wl.kelvin_helmholtz(n=24, nv=8)
    q = wl.sod(n=64, nv=16)
    ref = cd.Solver(p)
    ref.step(6)
    want = ref.moments()
    ref.close()
    a, b = cd.Solver(p), cd.Solver(q)
    bt = cd.Batch([a, b], chunk_steps=2)
    lib = cd.load_library()
    lib.cdugks_destroy(a.ctx)  # refused
    assert "batch" in cd.last_error()
    with pytest.raises(cd.CdugksError) as ei:
        a.close()  # the binding refuses as well
    assert ei.value.code == cd.ERR_BUSY
    bt.step(4)
    bt.close()
    a.step(2)
    got = a.moments()
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_acceleration_validation():
    p = wl.sod(n=16, nv=10)
    for bad in ([math.nan], [math.inf]):
        with pytest.raises(cd.CdugksError) as ei:
            cd.cdugks_required_bytes(dict(p, accel=bad))
        assert ei.value.code == cd.ERR_INVALID
    with pytest.raises(cd.CdugksError) as ei:
        cd.cdugks_required_bytes(dict(p, accel=[1.0], reconstruction="single_slope"))
    assert "reconstruction" in str(ei.value)
    assert cd.cdugks_required_bytes(dict(p, accel=[1.0])) > 0
