"""Independent formulations of the MRCM used only as pins (oracle).

* ``mrcm_monolithic``: every local pressure and every interface unknown in one
  sparse system, with the Robin coupling written face by face.  No MBF is
  formed and nothing is superposed, so agreement with the MBF path
  (Algorithm 2) checks the superposition, the Gamma-flux blocks and the
  assembly of (2.18)-(2.22).
* ``dirichlet_local`` / ``neumann_local``: the two limits the paper describes
  for the Robin parameter (Introduction and Sec. 3.2.4): alpha -> 0 gives local
  problems with pressure data on Gamma and weak flux continuity (a mortar-type
  method); alpha -> infinity gives local problems with flux data on Gamma and
  weak pressure continuity (a hybrid-type method).

The trace pressure of a cell c at a Gamma face, in the flux-data limit, is
the half-cell value p_f = p_c - (Q_f / A) h / (2 K_d(c)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import Geometry
from .mrcm import local_system


def _blocks(pb, geo, alpha, beta_mode=0):
    return [local_system(pb, geo, l, alpha, beta_mode) for l in range(geo.n_sub)]


def mrcm_monolithic(case):
    """Solve the MRCM as one system in (p, pi^p, pi^u).  Returns (p, pi)."""
    pb, alpha = case.problem, case.alpha
    geo = Geometry(pb.dims, case.partition, case.iface)
    N, NV = pb.n, geo.n_patch
    rows, cols, vals = [], [], []
    rhs = np.zeros(N + 2 * NV)
    for ls in _blocks(pb, geo, alpha, getattr(case, "beta_mode", 0)):
        M = ls.M.tocoo()
        rows.append(ls.cells[M.row])
        cols.append(ls.cells[M.col])
        vals.append(M.data)
        rhs[ls.cells] = ls.R[:, 0]
        g = ls.gamma
        live = g.cell != ls.pin_local
        c = g.gcell[live]
        # cell rows:  - T (pi^p - sigma beta pi^u)
        rows += [c, c]
        cols += [N + g.patch[live], N + NV + g.patch[live]]
        vals += [-g.T[live], g.T[live] * g.sigma[live] * g.beta[live]]
        # P-rows: sum T (p_c - pi^p + sigma beta pi^u) = 0
        rows += [N + g.patch, N + g.patch, N + g.patch]
        cols += [g.gcell, N + g.patch, N + NV + g.patch]
        vals += [g.T, -g.T, g.T * g.sigma * g.beta]
        # U-rows: sum sigma beta T (p_c - pi^p + sigma beta pi^u) - sum A beta pi^u = 0
        sbt = g.sigma * g.beta * g.T
        rows += [N + NV + g.patch] * 4
        cols += [g.gcell, N + g.patch, N + NV + g.patch, N + NV + g.patch]
        vals += [sbt, -sbt, g.beta * g.beta * g.T, -g.area * g.beta]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N + 2 * NV, N + 2 * NV)).tocsc()
    x = spla.splu(A).solve(rhs)
    return x[:N], x[N:]


def dirichlet_local(case):
    """alpha -> 0 limit: Gamma data p = pi^p, flux Q = A (2K/h) (p_c - pi^p);
    rows: cells and weak flux continuity.  Returns (p, pi^p)."""
    pb = case.problem
    geo = Geometry(pb.dims, case.partition, case.iface)
    N, NV = pb.n, geo.n_patch
    rows, cols, vals = [], [], []
    rhs = np.zeros(N + NV)
    for ls in _blocks(pb, geo, 0.0):
        M = ls.M.tocoo()
        rows.append(ls.cells[M.row])
        cols.append(ls.cells[M.col])
        vals.append(M.data)
        rhs[ls.cells] = ls.R[:, 0]
        g = ls.gamma
        live = g.cell != ls.pin_local
        rows.append(g.gcell[live])
        cols.append(N + g.patch[live])
        vals.append(-g.T[live])
        rows += [N + g.patch, N + g.patch]
        cols += [g.gcell, N + g.patch]
        vals += [g.T, -g.T]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N + NV, N + NV)).tocsc()
    x = spla.splu(A).solve(rhs)
    return x[:N], x[N:]


def neumann_local(case):
    """alpha -> infinity limit: Gamma flux Q^s_f = sigma^s A pi^u_i;
    rows: cells and weak pressure continuity of the half-cell traces.
    Returns (p, pi^u)."""
    pb = case.problem
    geo = Geometry(pb.dims, case.partition, case.iface)
    N, NV = pb.n, geo.n_patch
    Ks = (pb.kx, pb.ky, pb.kz)
    rows, cols, vals = [], [], []
    rhs = np.zeros(N + NV)
    for ls in _blocks(pb, geo, 1.0):
        g = ls.gamma
        # remove the Robin diagonal: the local operator keeps TPFA + walls only
        M = ls.M.tolil()
        for c, t in zip(g.cell, g.T):
            if c != ls.pin_local:
                M[c, c] -= t
        M = M.tocoo()
        rows.append(ls.cells[M.row])
        cols.append(ls.cells[M.col])
        vals.append(M.data)
        rhs[ls.cells] = ls.R[:, 0]
        live = g.cell != ls.pin_local
        rows.append(g.gcell[live])
        cols.append(N + g.patch[live])
        vals.append(g.sigma[live] * g.area[live])
        d = g.face // 2
        h = np.asarray(pb.h)[d]
        K = np.array([Ks[dd][c] for dd, c in zip(d, g.gcell)])
        # sum_s sigma^s sum_f A (p_c - sigma pi^u h / (2K)) = 0
        rows += [N + g.patch, N + g.patch]
        cols += [g.gcell, N + g.patch]
        vals += [g.sigma * g.area, -g.area * h / (2.0 * K)]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N + NV, N + NV)).tocsc()
    x = spla.splu(A).solve(rhs)
    return x[:N], x[N:]
