"""Two-point-flux finite volumes and the global fine-grid solve (oracle).

Follows Sec. 2.2.1: the 7-point system (2.9) with the harmonic-mean
coefficients (2.10), its global assembly (2.11) and the two-point velocity
recovery (2.12).

All quantities are written as total face rates Q (outward from a cell), with
face area A_d = V / h_d, so that a row reads  sum_faces Q = q_c  where
q_c = f_c V_c.  Dividing a row by V recovers (2.9)/(2.10): the interior
transmissibility T = A_d Ktilde / h_d is V times a_{ijk} = Ktilde / h_d^2.

Reading adopted for walls (the paper defers the boundary modification of
(2.10) to its reference [guiraldello2018]): the lowest-order Raviart-Thomas
scheme with trapezoidal quadrature, i.e. a half-cell transmissibility:
  Dirichlet wall  Q = A_d (2 K_d / h_d) (p_c - g_p)
  Neumann wall    Q = A_d g_u            (g_u = outward normal velocity)
  no-flow wall    Q = 0
Gauge: where no Dirichlet wall fixes the pressure, one pinned cell c* has its
row and column replaced by the identity with zero right-hand side.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# faces in the fixed order -x, +x, -y, +y, -z, +z: (axis, direction)
FACES = ((0, -1), (0, +1), (1, -1), (1, +1), (2, -1), (2, +1))


def grid3(a, dims):
    """View a flat x-fastest array as [z][y][x]."""
    nx, ny, nz = dims
    return np.asarray(a).reshape(nz, ny, nx)


def face_area(h, d):
    return h[0] * h[1] * h[2] / h[d]


def harmonic(a, b):
    """Harmonic mean of two positive permeabilities, eq. (2.10)."""
    return 2.0 * a * b / (a + b)


def interior_transmissibility(pb, d):
    """T between cell c and its +e_d neighbour, for all such pairs.

    Returns an array of shape [nz, ny, nx] shrunk by one along axis d:
    T = A_d * Ktilde / h_d with Ktilde the harmonic mean (2.10)."""
    dims, h = pb.dims, pb.h
    K = grid3((pb.kx, pb.ky, pb.kz)[d], dims)
    ax = 2 - d  # numpy axis of grid axis d in [z][y][x]
    lo = np.take(K, np.arange(0, K.shape[ax] - 1), axis=ax)
    hi = np.take(K, np.arange(1, K.shape[ax]), axis=ax)
    return face_area(h, d) * harmonic(lo, hi) / h[d]


def wall_cells(dims, f):
    """Flat indices of the cells touching wall f, ordered by the wall's value
    index (lower in-plane axis fastest)."""
    nx, ny, nz = dims
    d, s = FACES[f]
    a, b = [x for x in range(3) if x != d]
    n = (nx, ny, nz)
    ta, tb = np.meshgrid(np.arange(n[a]), np.arange(n[b]), indexing="xy")
    x = [None, None, None]
    x[a] = ta.reshape(-1)
    x[b] = tb.reshape(-1)
    x[d] = np.full(x[a].shape, 0 if s < 0 else n[d] - 1)
    return x[0] + nx * (x[1] + ny * x[2])


def wall_terms(pb):
    """Diagonal and right-hand-side contributions of the domain walls.

    Returns (diag_add[N], rhs_add[N]) for the cell rows sum Q = q."""
    N = pb.n
    diag = np.zeros(N)
    rhs = np.zeros(N)
    for f in range(6):
        wt = pb.wall_type[f]
        if wt == 0:
            continue
        d, _ = FACES[f]
        cells = wall_cells(pb.dims, f)
        g = pb.wall_value[f]
        g = np.zeros(len(cells)) if g is None else np.asarray(g, dtype=np.float64)
        A = face_area(pb.h, d)
        K = (pb.kx, pb.ky, pb.kz)[d][cells]
        if wt == 1:  # Dirichlet: Q = A 2K/h (p - g)
            t = A * 2.0 * K / pb.h[d]
            np.add.at(diag, cells, t)
            np.add.at(rhs, cells, t * g)
        elif wt == 2:  # Neumann: Q = A g (known outflow) moves to the right side
            np.add.at(rhs, cells, -A * g)
        else:
            raise ValueError("wall type must be 0, 1 or 2")
    return diag, rhs


def fine_system(pb):
    """Global TPFA matrix and right-hand side, eq. (2.11), with walls and pin."""
    dims = pb.dims
    nx, ny, nz = dims
    N = pb.n
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for d in range(3):
        T = interior_transmissibility(pb, d)
        ax = 2 - d
        c = np.take(idx, np.arange(0, idx.shape[ax] - 1), axis=ax).reshape(-1)
        n = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).reshape(-1)
        t = T.reshape(-1)
        np.add.at(diag, c, t)
        np.add.at(diag, n, t)
        rows += [c, n]
        cols += [n, c]
        vals += [-t, -t]
    wd, wr = wall_terms(pb)
    diag += wd
    rhs = np.asarray(pb.q, dtype=np.float64) + wr
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    if pb.pin >= 0:
        A, rhs = pin_system(A, rhs, pb.pin)
    return A, rhs


def pin_system(A, rhs, c):
    """Replace row and column c by the identity and set rhs[c] = 0 (keeps symmetry)."""
    A = A.tolil()
    A[c, :] = 0.0
    A[:, c] = 0.0
    A[c, c] = 1.0
    rhs = rhs.copy()
    rhs[c] = 0.0
    return A.tocsr(), rhs


def face_velocities_fine(pb, p):
    """Per-cell outward normal velocity on faces -x,+x,-y,+y,-z,+z, eq. (2.12):
    u = Q / A_d with Q = T (p_c - p_n) on interior faces and the wall rules."""
    dims = pb.dims
    nx, ny, nz = dims
    N = pb.n
    P = grid3(p, dims)
    U = np.zeros((6, nz, ny, nx))
    for d in range(3):
        T = interior_transmissibility(pb, d)
        ax = 2 - d
        A = face_area(pb.h, d)
        plo = np.take(P, np.arange(0, P.shape[ax] - 1), axis=ax)
        phi = np.take(P, np.arange(1, P.shape[ax]), axis=ax)
        u = T * (plo - phi) / A  # velocity along +e_d across the face
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, P.shape[ax] - 1)
        sl_hi[ax] = slice(1, P.shape[ax])
        U[2 * d + 1][tuple(sl_lo)] = u
        U[2 * d][tuple(sl_hi)] = -u
    U = U.reshape(6, N)
    for f in range(6):
        wt = pb.wall_type[f]
        if wt == 0:
            continue
        d, _ = FACES[f]
        cells = wall_cells(dims, f)
        g = pb.wall_value[f]
        g = np.zeros(len(cells)) if g is None else np.asarray(g, dtype=np.float64)
        K = (pb.kx, pb.ky, pb.kz)[d][cells]
        if wt == 1:
            U[f, cells] = 2.0 * K / pb.h[d] * (p[cells] - g)
        else:
            U[f, cells] = g
    return U


def fine_solve(pb):
    """Solve the fine-grid system (2.11) directly (the paper uses GMRES+AMG; a
    direct sparse solve is the exact reference).  Returns (p[N], U[6][N])."""
    A, rhs = fine_system(pb)
    p = spla.splu(A.tocsc()).solve(rhs)
    return p, face_velocities_fine(pb, p)
