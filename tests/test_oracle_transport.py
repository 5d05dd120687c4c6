"""Pins of the saturation-step oracle (oracle/transport.py), on the CPU.

* A front of water under a uniform velocity at Courant number 1 moves exactly
  one cell per step, in the direction of the flow (signs, upwinding, walls).
* In 1D the scheme converges to the Buckley-Leverett solution built from the
  Welge tangent, with the error shrinking under refinement.
* A uniform saturation stays uniform under any velocity field (the
  divergence compensation).
* With a cell-conservative velocity (a fine solve with wells in a closed box)
  the water volume changes by exactly the injected water minus the water the
  producers take.
* Under the CFL step with cfl = 1/6 the saturation stays in [0, 1].
* From an all-oil state phi' vanishes and the CFL bound is infinite: the step
  is the caller's dt_max, and one step puts exactly dt q / V of water into
  the injector cell and nothing anywhere else (every phi is 0).
* phi' against central differences; the limits of phi and lambda.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from mrcm_inputs import small_case
from oracle.fine import fine_solve
from oracle.transport import (cfl_dt, frac_flow, frac_flow_deriv, mobility, transport_step,
                              water_volume)


def _uniform_x(n, u):
    """1D column of n cells with velocity u along x: outward values per cell."""
    U = np.zeros((6, n))
    U[1] = u     # +x face
    U[0] = -u    # -x face
    return U


@pytest.mark.parametrize("u", [1.0, -1.0])
def test_front_moves_one_cell_per_step_at_courant_one(u):
    n = 20
    U = _uniform_x(n, u)
    S = np.zeros(n)
    for k in range(1, 8):
        S = transport_step((n, 1, 1), (1.0, 1.0, 1.0), U, np.zeros(n), S, 1.0, 1.0, 3.0)
        expect = np.zeros(n)
        if u > 0:
            expect[:k] = 1.0
        else:
            expect[n - k:] = 1.0
        assert np.array_equal(S, expect), k


def _welge(M):
    """Front saturation of the Welge tangent: phi(s) / s = phi'(s)."""
    return brentq(lambda s: frac_flow(s, M) / s - frac_flow_deriv(s, M), 1e-6, 1.0 - 1e-9)


def _bl_exact(x, t, M):
    """Buckley-Leverett saturation for S = 0 initially, S = 1 injected at x = 0,
    unit velocity and porosity."""
    sf = _welge(M)
    xf = frac_flow_deriv(sf, M) * t
    S = np.zeros_like(x)
    behind = x < xf
    for i in np.nonzero(behind)[0]:
        # phi'(S) = x / t on the rarefaction S in [sf, 1]
        target = x[i] / t
        S[i] = 1.0 if target <= 0.0 else brentq(lambda s: frac_flow_deriv(s, M) - target, sf, 1.0 - 1e-12)
    return S


def test_buckley_leverett_convergence():
    M, T = 2.0, 0.4
    errs = []
    for n in (100, 400):
        h = 1.0 / n
        U = _uniform_x(n, 1.0)
        S = np.zeros(n)
        # the largest phi' over [0, 1] bounds the step for every state
        grid = np.linspace(0, 1, 10001)
        dt = 0.5 * h / frac_flow_deriv(grid, M).max()
        steps = int(np.ceil(T / dt))
        dt = T / steps
        for _ in range(steps):
            S = transport_step((n, 1, 1), (h, 1.0, 1.0), U, np.zeros(n), S, dt, 1.0, M)
        x = (np.arange(n) + 0.5) * h
        errs.append(np.mean(np.abs(S - _bl_exact(x, T, M))))
    assert errs[1] < 0.6 * errs[0], errs
    assert errs[1] < 0.02, errs


def test_uniform_saturation_is_unchanged_by_any_velocity():
    rng = np.random.default_rng(3)
    dims = (7, 5, 4)
    N = 7 * 5 * 4
    U = rng.standard_normal((6, N))
    # no flow across the domain walls (a wall inflow would bring water)
    X = np.stack(np.unravel_index(np.arange(N), (4, 5, 7)), axis=1)[:, ::-1]
    for f in range(6):
        d, up = f // 2, f % 2
        U[f][X[:, d] == (dims[d] - 1 if up else 0)] = 0.0
    S = np.full(N, 0.37)
    S1 = transport_step(dims, (2.0, 1.0, 0.5), U, np.zeros(N), S, 0.01, 1.0, 5.0)
    assert np.max(np.abs(S1 - S)) == 0.0


def _closed_box_with_wells(seed):
    case = small_case((10, 8, 5), (1, 1, 1), seed=seed)
    pb = case.problem
    p, U = fine_solve(pb)
    return pb, U.reshape(6, -1)


def test_water_balance_with_a_conservative_velocity():
    pb, U = _closed_box_with_wells(2)
    rng = np.random.default_rng(5)
    S = rng.uniform(0.0, 1.0, pb.n)
    mu_w, mu_o = 1.0, 4.0
    dt = cfl_dt(pb.dims, pb.h, U, S, mu_w, mu_o, cfl=1.0 / 6.0)
    S1 = transport_step(pb.dims, pb.h, U, pb.q, S, dt, mu_w, mu_o)
    q = np.asarray(pb.q)
    phi = frac_flow(S, mu_o / mu_w)
    water = dt * (q[q > 0].sum() + (phi[q < 0] * q[q < 0]).sum())
    change = water_volume(pb.h, S1) - water_volume(pb.h, S)
    assert abs(change - water) <= 1e-11 * max(abs(water), dt * np.abs(q).sum())


def test_saturation_stays_in_bounds_under_the_cfl_step():
    pb, U = _closed_box_with_wells(4)
    rng = np.random.default_rng(6)
    S = rng.uniform(0.0, 1.0, pb.n)
    for _ in range(40):
        dt = cfl_dt(pb.dims, pb.h, U, S, 1.0, 10.0, cfl=1.0 / 6.0)
        S = transport_step(pb.dims, pb.h, U, pb.q, S, dt, 1.0, 10.0)
        assert S.min() >= -1e-12 and S.max() <= 1.0 + 1e-12


def test_frac_flow_derivative_and_limits():
    M = 3.5
    s = np.linspace(0.01, 0.99, 50)
    e = 1e-6
    fd = (frac_flow(s + e, M) - frac_flow(s - e, M)) / (2 * e)
    assert np.max(np.abs(fd - frac_flow_deriv(s, M))) < 1e-7
    assert frac_flow(0.0, M) == 0.0 and frac_flow(1.0, M) == 1.0
    assert abs(frac_flow(0.5, M) - M / (M + 1.0)) < 1e-15
    assert mobility(0.0, 2.0, 5.0) == 1.0 / 5.0 and mobility(1.0, 2.0, 5.0) == 1.0 / 2.0


def test_all_oil_start_takes_the_callers_step_and_fills_the_injector_only():
    pb, U = _closed_box_with_wells(2)
    S = np.zeros(pb.n)
    assert cfl_dt(pb.dims, pb.h, U, S, 1.0, 5.0, cfl=1.0 / 6.0) == np.inf
    dt = cfl_dt(pb.dims, pb.h, U, S, 1.0, 5.0, cfl=1.0 / 6.0, dt_max=0.3)
    assert dt == 0.3
    S1 = transport_step(pb.dims, pb.h, U, pb.q, S, dt, 1.0, 5.0)
    q = np.asarray(pb.q)
    V = pb.h[0] * pb.h[1] * pb.h[2]
    expect = np.where(q > 0, dt * q / V, 0.0)
    assert np.array_equal(S1, expect)
    # a bound below the caller's step wins
    S = np.random.default_rng(1).uniform(0.0, 1.0, pb.n)
    b = cfl_dt(pb.dims, pb.h, U, S, 1.0, 5.0)
    assert cfl_dt(pb.dims, pb.h, U, S, 1.0, 5.0, dt_max=2 * b) == b
    assert cfl_dt(pb.dims, pb.h, U, S, 1.0, 5.0, dt_max=0.5 * b) == 0.5 * b
