"""The allocation-free variant of cdugks_distributions: the same FP64 copies
of g and b, staged through the library's fixed device array instead of a
temporary allocation, on two calls in a row (the second on a smaller
problem), and a problem whose velocity row exceeds the array refused."""
import os
import re
import sys

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(s):
    lib = cd.load_library()
    g = np.zeros(s.V * s.N)
    b = np.zeros(s.V * s.N)
    rc = lib.cdugks_distributions_noalloc(s.ctx, cd._ptr(g), cd._ptr(b))
    return rc, g.reshape(s.V, s.N), b.reshape(s.V, s.N)


def test_noalloc_distributions_match_the_allocating_entry_point():
    cases = [
        # larger first: KH 64^2 x 16^2 in FP32 storage (a row of 32 KB; many
        # rows per pass through the array), then a small FP64 Sod tube
        (wl.kelvin_helmholtz(n=64, nv=16, storage="f32"), 3),
        (wl.sod(n=40, nv=12), 2),
    ]
    for p, steps in cases:
        _log(f"no-alloc distributions: dim={p['dim']} n={p['n']} nv={p['nv']} storage={p['storage']}")
        s = cd.Solver(p)
        s.step(steps)
        g_ref, b_ref = s.distributions()
        rc, g, b = _noalloc(s)
        assert rc == cd.OK, cd.last_error()
        assert np.array_equal(g, g_ref) and np.array_equal(b, b_ref)
        s.close()


def scratch_bytes():
    """The array's size as the header states it."""
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cdugks.h")
    m = re.search(r"#define\s+CDUGKS_NOALLOC_SCRATCH_BYTES\s+\(\(size_t\)(\d+)\s*<<\s*(\d+)\)", open(hdr).read())
    return int(m.group(1)) << int(m.group(2))


def test_noalloc_distributions_refuse_rows_beyond_the_array():
    lib = cd.load_library()
    cap = scratch_bytes()
    n = cap // 8 + 1  # one cell more than an FP64 row the array holds
    p = wl.sod(n=n, nv=2)
    p["rho"] = np.ones(n)
    p["T"] = np.ones(n)
    p["u"] = np.zeros((1, n))
    _log(f"no-alloc distributions: row of {n} cells against an array of {cap} bytes")
    s = cd.Solver(p)
    g = np.zeros(2 * n)
    b = np.zeros(2 * n)
    rc = lib.cdugks_distributions_noalloc(s.ctx, cd._ptr(g), cd._ptr(b))
    assert rc == cd.ERR_TOO_LARGE
    assert "scratch" in cd.last_error()
    s.close()
