"""Oracle of the "Mean" velocity post-processing (Sec. 6, the two-phase
experiment): a unique flux on the interfaces from the average of the two
sides' multiscale velocities, then one Neumann problem per subdomain, eq.
(locprob_submean), whose velocity is conservative cell by cell.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU baseline, never by the library.

Input: the multiscale velocity u_H as the reconstruction gives it, per cell
and face, outward, own side: U[6][N] (faces -x, +x, -y, +y, -z, +z).
* The unique interface velocity: on a fine face of Gamma between cell c (the
  lower side) and cell n (the upper side) along axis d, with the normal
  n^ = +e_d, the average of the two sides' normal velocities,
      ubar = (U[+d][c] - U[-d][n]) / 2,
  outward from c it is ubar, outward from n it is -ubar.
* Per subdomain: the TPFA matrix of (2.10) restricted to the subdomain's own
  cell pairs, and Neumann data on its whole boundary: A_d ubar on Gamma, the
  multiscale velocity's own value A_d U on the domain walls (the paper's
  boundary condition u_h.n = u_H.n there).  Row c reads
      sum over interior faces T (p_c - p_n) = q_c - sum over boundary faces A_d u_out.
* Reading M1 (the paper does not say how the singular Neumann problem is
  fixed): the pressure is set to zero at the subdomain's lowest-corner cell,
  whose row and column become the identity; that row's balance then carries
  the compatibility defect, which the multiscale solution's weak flux
  continuity keeps at the rounding of its interface solve.  The velocities do
  not depend on the choice of the cell beyond that defect.
* Output: the subdomain pressures pt (in that gauge) and the velocity
  Ut[6][N]: interior faces T (p_c - p_n) / A_d from pt, Gamma faces and walls
  from the data.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fine import face_area, grid3, interior_transmissibility
from .mrcm import refined_solve


def unique_gamma_velocity(pb, geo, U):
    """U with its Gamma faces replaced by the two sides' average (above)."""
    U = np.asarray(U, dtype=np.float64).reshape(6, pb.n)
    Ub = U.copy()
    for t, I in enumerate(geo.ifaces):
        d = I["d"]
        c, n, _ = geo.iface_faces(t)
        ub = 0.5 * (U[2 * d + 1][c] - U[2 * d][n])
        Ub[2 * d + 1][c] = ub
        Ub[2 * d][n] = -ub
    return Ub


def neumann_local(pb, geo, l, Ub, pin_local=0):
    """Matrix and right-hand side of subdomain l's Neumann problem with the
    boundary velocities Ub (unique on Gamma, multiscale on walls), the local
    cells in x-fastest order and local cell pin_local fixed at zero."""
    nx, ny, _ = pb.dims
    cells = geo.sub_cells(l)
    lo, hi = geo.sub_lo[l], geo.sub_hi[l]
    ext = hi - lo
    nl = len(cells)
    loc = np.arange(nl).reshape(ext[2], ext[1], ext[0])
    rows, cols, vals = [], [], []
    diag = np.zeros(nl)
    for d in range(3):
        T = interior_transmissibility(pb, d)  # global [nz][ny][nx] shrunk along d
        ax = 2 - d
        sl = [slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0])]
        sl[ax] = slice(lo[d], hi[d] - 1)     # pairs (c, c + e_d) inside the box
        t = T[tuple(sl)].reshape(-1)
        c = np.take(loc, np.arange(0, ext[d] - 1), axis=ax).reshape(-1)
        n = np.take(loc, np.arange(1, ext[d]), axis=ax).reshape(-1)
        np.add.at(diag, c, t)
        np.add.at(diag, n, t)
        rows += [c, n]
        cols += [n, c]
        vals += [-t, -t]
    rows.append(np.arange(nl))
    cols.append(np.arange(nl))
    vals.append(diag)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nl, nl)).tocsr()
    rhs = np.asarray(pb.q, dtype=np.float64)[cells].copy()
    # boundary faces of the box: data outflows move to the right-hand side
    X = np.stack(np.unravel_index(np.arange(nl), (ext[2], ext[1], ext[0])), axis=1)[:, ::-1] + lo
    for f in range(6):
        d, side = f // 2, (1 if f % 2 else -1)
        on = X[:, d] == (hi[d] - 1 if side > 0 else lo[d])
        rhs[on] -= face_area(pb.h, d) * Ub[f][cells[on]]
    M = M.tolil()
    M[pin_local, :] = 0.0
    M[:, pin_local] = 0.0
    M[pin_local, pin_local] = 1.0
    rhs[pin_local] = 0.0
    return M.tocsr(), rhs, cells


def mean_postprocess(pb, geo, U, pin=None, extended=True):
    """The Mean post-processing of the multiscale velocity U[6][N].  pin:
    per subdomain the local cell fixed at zero (default: 0, the lowest
    corner).  Returns (pt[N], Ut[6][N])."""
    Ub = unique_gamma_velocity(pb, geo, U)
    N = pb.n
    pt = np.zeros(N)
    for l in range(geo.n_sub):
        M, rhs, cells = neumann_local(pb, geo, l, Ub, 0 if pin is None else int(pin[l]))
        pt[cells] = refined_solve(M, rhs[:, None], extended)[:, 0]
    # interior faces of every subdomain from pt; Gamma faces and walls keep Ub
    Ut = Ub.copy().reshape(6, *reversed(pb.dims))
    P = grid3(pt, pb.dims)
    sub_of = [np.searchsorted(geo.cuts[d], np.arange(pb.dims[d]), side="right") - 1 for d in range(3)]
    for d in range(3):
        T = interior_transmissibility(pb, d)
        ax = 2 - d
        A = face_area(pb.h, d)
        plo = np.take(P, np.arange(0, P.shape[ax] - 1), axis=ax)
        phi = np.take(P, np.arange(1, P.shape[ax]), axis=ax)
        u = T * (plo - phi) / A
        same = sub_of[d][:-1] == sub_of[d][1:]  # the pair lies inside one subdomain
        shape = [1, 1, 1]
        shape[ax] = -1
        inside = np.broadcast_to(same.reshape(shape), u.shape)
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, P.shape[ax] - 1)
        sl_hi[ax] = slice(1, P.shape[ax])
        U_lo = Ut[2 * d + 1][tuple(sl_lo)]
        U_hi = Ut[2 * d][tuple(sl_hi)]
        U_lo[inside] = u[inside]
        U_hi[inside] = -u[inside]
    return pt, Ut.reshape(6, N)


def cell_balance(pb, Ut):
    """Per cell: sum over faces of A_d Ut - q (the conservation residual)."""
    Ut = np.asarray(Ut).reshape(6, pb.n)
    A = np.repeat([face_area(pb.h, d) for d in range(3)], 2)
    return (Ut * A[:, None]).sum(axis=0) - np.asarray(pb.q, dtype=np.float64)
