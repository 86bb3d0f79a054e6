"""GPU parity of the distributions themselves: g and b of every (cell,
velocity) after 1 and 5 steps against the oracle's, element by element.

The moment tests see the update kernel (eq. phiupdate) only through later
steps' moments; here g^{n+1} and b^{n+1} are compared directly, FP64 storage,
relative to the largest magnitude of each velocity row (1e-12), so an error
confined to the far tail rows is not hidden under the bulk.  Cases: the
Kelvin-Helmholtz layer at 40^2 x 12^2 (periodic, several tiles), a 3-D ragged
problem with outflow and periodic axes and an odd velocity count (a zero
velocity component), and a 2-D problem with Dirichlet sides unlike the
interior.  The library returns [V][N] (velocity-major), the oracle [N][V].
"""
import sys

import numpy as np
import pytest

from paper_2208_09132_amd import cdugks as cd
from paper_2208_09132_amd import workloads as wl
from tests.helpers import dt_checked, make_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def row_errors(ref_nv, got_vn):
    """max over velocities of max_c |got - ref| / max_c |ref| (per row)."""
    ref = np.asarray(ref_nv).T  # [V][N]
    scale = np.max(np.abs(ref), axis=1)
    assert np.all(scale > 0)
    return float(np.max(np.max(np.abs(np.asarray(got_vn) - ref), axis=1) / scale))


def check_distributions(prob, checkpoints=(1, 5)):
    _log(f"distributions: dim={prob['dim']} n={prob['n']} nv={prob['nv']} bc={prob['bc']}")
    s = cd.Solver(prob)
    o = make_oracle(prob, dt=dt_checked(prob, s.dt))
    g0, b0 = s.distributions()
    og, ob, _ = o.state()
    # the initial discrete equilibria (eqs. geq, beq) first
    errs = [(0, row_errors(og, g0), row_errors(ob, b0))]
    done = 0
    for n in checkpoints:
        s.step(n - done)
        assert o.step(n - done) == 0
        done = n
        g, b = s.distributions()
        og, ob, _ = o.state()
        errs.append((n, row_errors(og, g), row_errors(ob, b)))
    s.close()
    _log(f"  per-row relative errors (steps, g, b): {errs}")
    for n, eg, eb in errs:
        assert eg <= TOL and eb <= TOL, (n, eg, eb)


def test_kelvin_helmholtz_reduced_distributions():
    check_distributions(wl.kelvin_helmholtz(n=40, nv=12))


def test_3d_ragged_outflow_distributions():
    p = wl.random_fourier(3, [17, 9, 11], [5, 6, 5], wl.SplitMix64(21), amp=0.2, Kn=3e-2)
    p["bc"] = ["outflow", "periodic", "outflow"]
    check_distributions(p)


def test_dirichlet_distributions():
    p = wl.random_fourier(2, [21, 18], [7, 6], wl.SplitMix64(8), amp=0.2, Kn=1e-2)
    p["bc"] = ["dirichlet", "periodic"]
    p["dirichlet"] = [[[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]], None]
    check_distributions(p)
