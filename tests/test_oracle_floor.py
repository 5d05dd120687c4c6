"""The FP64 rounding floor of the 60x220x85 channelised workload.

The interface system (2.18) of this workload is badly conditioned in the
direction that shifts the pressure level (the gauge is fixed by one pinned
cell).  Rounding in the local solves, of a few units in the last place of the
MBFs, perturbs the interface matrix by about 1e-15 of its largest entry and
moves the pressure by about 1.7e-8 relative L2.  So the plain FP64 algorithm
cannot serve as the reference of a 1e-8 gate on this workload; the oracle
therefore refines every linear solve with an extended-precision residual
(``oracle.mrcm.refined_solve``).  These tests establish that floor on the CPU
and check that the refined oracle is converged.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from mrcm_inputs import config2
from oracle.geometry import Geometry
from oracle.mrcm import local_system, mrcm_solve, refined_solve
from oracle.norms import rel_l2

pytestmark = pytest.mark.slow

EXTENDED = np.finfo(np.longdouble).nmant >= 63


def _procs():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def cfg2_pair():
    c = config2()
    plain = mrcm_solve(c, extended=False, processes=_procs())
    ext = mrcm_solve(c, extended=True, processes=_procs())
    return c, plain, ext


@pytest.mark.skipif(not EXTENDED, reason="np.longdouble has no extended significand here")
def test_plain_fp64_floor_on_the_channelised_workload(cfg2_pair):
    """Same interface system to rounding, pressures 1e-8 apart."""
    c, plain, ext = cfg2_pair
    A0, A1 = plain.A_int, ext.A_int
    amax = abs(A1).max()
    assert abs(A1 - A0).max() <= 1e-14 * amax
    assert np.max(np.abs(ext.b_int - plain.b_int)) <= 1e-14 * np.max(np.abs(ext.b_int))
    e_p = rel_l2(plain.p, ext.p)
    e_u = rel_l2(plain.U, ext.U)
    # the floor of plain FP64 sits between 1e-10 and 1e-6 (measured 1.7e-8);
    # velocities, which the gauge does not shift, agree far better
    assert 1e-10 < e_p < 1e-6, e_p
    assert e_u < 1e-8, e_u
    print(f"plain FP64 vs refined oracle on 60x220x85: p {e_p:.3e}, U {e_u:.3e}, "
          f"interface matrix {abs(A1 - A0).max() / amax:.2e}")


@pytest.mark.skipif(not EXTENDED, reason="np.longdouble has no extended significand here")
def test_refined_oracle_is_converged(cfg2_pair):
    """Further refinement rounds change nothing beyond the last FP64 place:
    the refined MBFs of sampled subdomains, and the refined interface
    solution, are fixed points of one more round."""
    c, plain, ext = cfg2_pair
    geo = ext.geo
    rng = np.random.default_rng(0)
    for l in rng.choice(geo.n_sub, 12, replace=False):
        ls = local_system(c.problem, geo, int(l), c.alpha)
        X2 = refined_solve(ls.M, ls.R, True, steps=2)
        X4 = refined_solve(ls.M, ls.R, True, steps=4)
        assert np.max(np.abs(X4 - X2)) <= 4e-16 * np.max(np.abs(X4))
        assert np.array_equal(X2, ext.X[int(l)])
    # the extended residual itself is accurate only to about kappa times the
    # extended unit roundoff relative to |A||pi|, which bounds what further
    # rounds can settle (measured: 3e-14 between three and five rounds)
    pi5 = refined_solve(ext.A_int, ext.b_int, True, steps=5)
    assert rel_l2(pi5, ext.pi) < 1e-12
    # the plain sparse LU alone leaves the interface solution at ~1e-12
    pi0 = spla.splu(ext.A_int.tocsc()).solve(ext.b_int)
    assert rel_l2(pi0, ext.pi) < 1e-9
