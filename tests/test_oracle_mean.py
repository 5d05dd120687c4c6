"""Pins of the Mean post-processing oracle (oracle/mean.py), on the CPU.

* With one patch per fine face (the fine trace) the MRCM solution is the
  fine-grid solution (test T2), the two sides agree on every interface face,
  and the Neumann re-solves must return the fine-grid velocity.
* The result conserves mass cell by cell (except the pinned cells, which
  carry the compatibility defect, itself at the interface solve's rounding),
  is single-valued on every interface face, and keeps each patch's flux.
* The velocity does not depend on which cell fixes each subdomain's pressure.
* Wall faces keep the multiscale velocity (no-flow, Dirichlet and Neumann).
"""
import numpy as np
import pytest

from mrcm_inputs import small_case
from oracle.fine import face_area, fine_solve
from oracle.geometry import Geometry
from oracle.mean import cell_balance, mean_postprocess, unique_gamma_velocity
from oracle.mrcm import mrcm_solve


def _setup(case):
    pb = case.problem
    geo = Geometry(pb.dims, case.partition, case.iface)
    res = mrcm_solve(case)
    return pb, geo, res


def test_mean_on_the_fine_trace_returns_the_fine_velocity():
    case = small_case((12, 8, 6), (3, 2, 2), split=((0, 0), (0, 0), (0, 0)), seed=11)
    pb, geo, res = _setup(case)
    _, U_fine = fine_solve(pb)
    _, Ut = mean_postprocess(pb, geo, res.U)
    scale = np.max(np.abs(U_fine))
    assert np.max(np.abs(Ut - U_fine)) <= 1e-9 * scale


@pytest.mark.parametrize("split", [((1, 1), (1, 1), (1, 1)), ((2, 1), (1, 2), (2, 2))])
def test_mean_conserves_mass_and_is_single_valued(split):
    case = small_case((16, 12, 8), (2, 3, 2), split=split, seed=12)
    pb, geo, res = _setup(case)
    pt, Ut = mean_postprocess(pb, geo, res.U)
    A = np.repeat([face_area(pb.h, d) for d in range(3)], 2)
    flux_scale = np.max(np.abs(Ut * A[:, None]))
    bal = cell_balance(pb, Ut)
    pinned = np.array([geo.sub_cells(l)[0] for l in range(geo.n_sub)])
    free = np.ones(pb.n, dtype=bool)
    free[pinned] = False
    assert np.max(np.abs(bal[free])) <= 1e-11 * flux_scale
    assert np.max(np.abs(bal[pinned])) <= 1e-8 * flux_scale   # the compatibility defect
    for t, I in enumerate(geo.ifaces):
        d = I["d"]
        c, n, patch = geo.iface_faces(t)
        assert np.array_equal(Ut[2 * d + 1][c], -Ut[2 * d][n])
        # each patch transfers the mass the multiscale solution transfers
        for p in np.unique(patch):
            on = patch == p
            q_mean = Ut[2 * d + 1][c[on]].sum()
            q_lo = res.U.reshape(6, -1)[2 * d + 1][c[on]].sum()
            q_hi = -res.U.reshape(6, -1)[2 * d][n[on]].sum()
            s = max(abs(q_lo), abs(q_hi), 1e-300)
            assert abs(q_mean - q_lo) <= 1e-8 * max(s, flux_scale / face_area(pb.h, d))
            assert abs(q_mean - 0.5 * (q_lo + q_hi)) <= 1e-13 * max(s, 1.0)


def test_mean_velocity_does_not_depend_on_the_pinned_cell():
    case = small_case((16, 12, 8), (2, 3, 2), split=((2, 1), (1, 2), (2, 2)), seed=13)
    pb, geo, res = _setup(case)
    _, U0 = mean_postprocess(pb, geo, res.U)
    last = [len(geo.sub_cells(l)) - 1 for l in range(geo.n_sub)]
    _, U1 = mean_postprocess(pb, geo, res.U, pin=last)
    assert np.max(np.abs(U0 - U1)) <= 1e-8 * np.max(np.abs(U0))


def test_mean_keeps_the_wall_velocities():
    case = small_case((12, 10, 6), (2, 2, 2), split=((1, 1), (1, 1), (1, 1)), seed=14, pin=-1)
    pb = case.problem
    pb.wall_type = [1, 2, 0, 0, 0, 1]
    rng = np.random.default_rng(4)
    pb.wall_value = [rng.standard_normal(10 * 6), 0.01 * rng.standard_normal(10 * 6), None, None, None,
                     rng.standard_normal(12 * 10)]
    geo = Geometry(pb.dims, case.partition, case.iface)
    res = mrcm_solve(case)
    _, Ut = mean_postprocess(pb, geo, res.U)
    U = res.U.reshape(6, -1)
    from oracle.fine import wall_cells
    for f in range(6):
        cells = wall_cells(pb.dims, f)
        assert np.array_equal(Ut[f][cells], U[f][cells])


def test_unique_velocity_is_the_average_of_the_two_sides():
    case = small_case((10, 8, 6), (2, 2, 1), split=((1, 1), (2, 1), (1, 1)), seed=15)
    pb, geo, res = _setup(case)
    U = res.U.reshape(6, -1)
    Ub = unique_gamma_velocity(pb, geo, U)
    for t, I in enumerate(geo.ifaces):
        d = I["d"]
        c, n, _ = geo.iface_faces(t)
        assert np.allclose(Ub[2 * d + 1][c], 0.5 * (U[2 * d + 1][c] - U[2 * d][n]), rtol=0, atol=0)
    # faces off Gamma are untouched
    mask = np.ones_like(U, dtype=bool)
    for t, I in enumerate(geo.ifaces):
        d = I["d"]
        c, n, _ = geo.iface_faces(t)
        mask[2 * d + 1][c] = False
        mask[2 * d][n] = False
    assert np.array_equal(Ub[mask], U[mask])
