"""Oracle of the IMPES saturation step (Sec. 5's two-phase model and the
fine-grid transport solver of the implementation section): the Buckley-
Leverett equation discretised by upwind finite volumes, eqs.
(transporte_discreto) and (flux_disc_up), with the divergence compensation
term, the CFL bound (eq. CFL), and the total mobility that scales the
permeability of each Darcy solve.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU baseline, never by the library.

Model (Sec. 5): water saturation S, viscosity ratio M = mu_o / mu_w,
  fractional flow  phi(S) = M S^2 / (M S^2 + (1 - S)^2),
  total mobility   lambda(S) = S^2 / mu_w + (1 - S)^2 / mu_o.
Velocities: U[6][N] per cell, outward normal, own side (the layout the
reconstruction and the Mean post-processing write), faces -x, +x, .., +z.

Readings (the printed scheme leaves them open):
* T1, signs and units.  The printed update adds the face terms and subtracts
  Dt phi_c D u with D u the plain sum of the six face values; taken as fluxes
  into the cell divided by the cell size along each face's normal, the step is
      S_c' = S_c - Dt sum_f (phi_f - phi(S_c)) U[f][c] / h_d(f),
  the upwind conservative update plus Dt phi(S_c) times the discrete
  divergence of the face velocities, which makes the scheme monotone and
  leaves a uniform S unchanged under any velocity field.
* T2, upwinding (eq. flux_disc_up): phi_f = phi(S_c) on an outflow face
  (U[f][c] >= 0), phi(S_n) of the neighbour across an inflow face; across a
  domain wall an inflow carries water (phi = 1).
* T3, wells.  The compensation removes phi_c div u, and div u = q / V in a
  source cell: a producer (q < 0) then loses water at phi_c |q| / V, as the
  physics asks; an injector (q > 0) injects water, so its cell gains
  Dt q (1 - phi(S_c)) / V.
* T4, CFL (eq. CFL): Dt = cfl * min(h) / max_c( |phi'(S_c)| max_f |U[f][c]| ),
  cfl = 1 the paper's bound; a cell with inflow on several faces keeps S in
  [0, 1] for cfl <= 1/6 (the sum over six faces).  The loop of the
  implementation section takes the step Dt_s as an input that satisfies the
  bound, and the text speaks of adapting it: the step is min(Dt_s, bound),
  with Dt_s = dt_max given by the caller.  The bound sees the face flows only
  (at S = 0 everywhere phi' vanishes and it is infinite); a source cell's own
  rate is the caller's to bound through dt_max.
"""
from __future__ import annotations

import numpy as np

from .fine import grid3


def frac_flow(S, M):
    S = np.asarray(S, dtype=np.float64)
    a = M * S * S
    return a / (a + (1.0 - S) ** 2)


def frac_flow_deriv(S, M):
    """d phi / dS = 2 M S (1 - S) / (M S^2 + (1 - S)^2)^2."""
    S = np.asarray(S, dtype=np.float64)
    den = M * S * S + (1.0 - S) ** 2
    return 2.0 * M * S * (1.0 - S) / (den * den)


def mobility(S, mu_w, mu_o):
    S = np.asarray(S, dtype=np.float64)
    return S * S / mu_w + (1.0 - S) ** 2 / mu_o


def transport_step(dims, h, U, q, S, dt, mu_w, mu_o):
    """One saturation step (readings T1-T3).  U[6][N] outward face velocities,
    q[N] total source rates (volume per time), S[N]; returns the new S."""
    nx, ny, nz = dims
    N = nx * ny * nz
    M = mu_o / mu_w
    V = h[0] * h[1] * h[2]
    U = np.asarray(U, dtype=np.float64).reshape(6, N)
    S = np.asarray(S, dtype=np.float64)
    phi = frac_flow(S, M)
    P = grid3(phi, dims)
    out = S.copy()
    Sg = grid3(out, dims)  # view for the update
    for f in range(6):
        d, side = f // 2, (1 if f % 2 else -1)
        ax = 2 - d
        u = grid3(U[f], dims)
        # phi of the neighbour across the face; water across a domain wall
        pn = np.ones_like(P)
        n = dims[d]
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        if side > 0:
            dst[ax], src[ax] = slice(0, n - 1), slice(1, n)
        else:
            dst[ax], src[ax] = slice(1, n), slice(0, n - 1)
        pn[tuple(dst)] = P[tuple(src)]
        phi_f = np.where(u >= 0.0, P, pn)
        Sg -= dt * (phi_f - P) * u / h[d]
    q = np.asarray(q, dtype=np.float64)
    inj = q > 0.0
    out[inj] += dt * q[inj] * (1.0 - phi[inj]) / V
    return out


def cfl_dt(dims, h, U, S, mu_w, mu_o, cfl=1.0, dt_max=np.inf):
    """Time step of reading T4 (eq. CFL): min(dt_max, the CFL bound); the
    bound is inf when nothing moves."""
    N = dims[0] * dims[1] * dims[2]
    U = np.asarray(U, dtype=np.float64).reshape(6, N)
    speed = np.abs(frac_flow_deriv(S, mu_o / mu_w)) * np.abs(U).max(axis=0)
    m = float(speed.max()) if N else 0.0
    bound = np.inf if m == 0.0 else cfl * min(h) / m
    return min(float(dt_max), bound)


def water_volume(h, S):
    return float(np.sum(S)) * h[0] * h[1] * h[2]
