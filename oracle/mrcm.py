"""The Multiscale Robin Coupled Method, step by step (oracle).

Follows Algorithm 2 of the paper ("Pseudocode for the DD Multiscale mixed
method"): loop 1 builds, for every subdomain, the local matrix A^H_l and the
right-hand sides of the particular problem (2.26) and of the MBF problems
(2.25), and solves them; the interface system (2.18)-(2.22) is assembled from
the MBF fluxes and solved; loop 2 reconstructs pressure and velocity by the
combination (2.23).

Discrete local problem (readings adopted where the paper defers to its
reference for the boundary terms):
* Inside a subdomain: the TPFA rows of (2.9)/(2.10), as total face rates.
* Robin face f on Gamma, seen from side s (cell c, axis d): the local problem
  (2.13)/(2.14) imposes  -beta u.n^l + p = G  with G = P_H - beta U_H n.n^l.
  With the half-cell velocity u = 2 K_d (p_c - p_f) / h_d this gives
      Q_f = T_f (p_c - G_f),   T_f = A_d / (h_d / (2 K_d(c)) + beta_f).
* beta per side, eq. (3.1):  beta_f = alpha H_d / K_d(c), H_d the extent of
  the own subdomain along the face normal (physical length), K_d(c) the own
  cell's permeability along the normal.
* sigma = n . n^l = +1 on the lower side of an interface, -1 on the upper.
* Right-hand-side columns, in this order: 0 the particular problem (sources,
  wall data, G = 0 on Gamma); 1..n the P-type MBFs (P_H, U_H) = (phi_j, 0),
  i.e. G = 1 on patch j; n+1..2n the U-type MBFs (P_H, U_H) = (0, phi_j),
  i.e. G = -sigma beta_f on patch j.  Patches j run over I^l in increasing
  global id.  Since beta varies along a patch, U-type columns are genuine
  extra solves (2 |I^l| + 1 right-hand sides per subdomain, Sec. 2.2.2).
* Interface rows, from (2.15) and (2.16) with the two garbled entries of
  (2.19)/(2.20) read consistently with (2.21)/(2.22):
      P-row i:  sum_s sum_{f in i} Q^s_f = 0
      U-row i:  sum_s sigma^s sum_{f in i} beta^s_f Q^s_f
                 - (sum_s sum_{f in i} A_f beta^s_f) pi^u_i = 0
  written per column as blocks F[i,col] = sum_{f in i} Q_f[col] and
  Fb[i,col] = sum_{f in i} beta_f Q_f[col]; b^P carries a minus sign like b^U.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fine import FACES, face_area, harmonic, wall_cells
from .geometry import Geometry, split_index


@dataclass
class GammaFaces:
    """The Robin faces of one subdomain (one row per fine face on Gamma)."""
    cell: np.ndarray     # local cell index (x fastest within the box)
    gcell: np.ndarray    # global cell index
    face: np.ndarray     # 0..5 (-x,+x,-y,+y,-z,+z)
    patch: np.ndarray    # global patch id
    lpatch: np.ndarray   # position of the patch in I^l
    sigma: np.ndarray    # +1 lower side, -1 upper side
    beta: np.ndarray     # Robin parameter beta_f
    T: np.ndarray        # Robin transmissibility T_f
    area: np.ndarray     # A_d


@dataclass
class LocalSystem:
    sub: int             # subdomain id l
    cells: np.ndarray    # global indices of the subdomain's cells, x fastest
    M: sp.csr_matrix     # local matrix A^H_l (pin applied)
    R: np.ndarray        # [N_l, m] right-hand sides, columns as documented above
    gamma: GammaFaces
    patches: np.ndarray  # I^l (global ids, increasing)
    pin_local: int       # local index of the pinned cell or -1


def robin_beta(alpha, H, K):
    """Robin parameter, eq. (3.1): beta = alpha H_l / K_l(x)."""
    return alpha * H / K


def harmonic_mean(a, b):
    return 2.0 * a * b / (a + b)


def robin_transmissibility(A, h, K, beta):
    """Q = T (p_c - G) for a Robin face: T = A / (h / (2K) + beta)."""
    return A / (h / (2.0 * K) + beta)


def gamma_faces(pb, geo, l, alpha, beta_mode=0):
    """Enumerate the Robin faces of subdomain l (faces of its box on Gamma).

    beta_mode 0: beta per side, eq. (3.1) with the own subdomain's extent H
    along the normal and the own cell's K.  beta_mode 1: one beta per fine
    face shared by both sides, eq. (3.1) with the harmonic means of the two
    sides' H and of the two cells' K (the two-point face value of K, as in
    (2.10))."""
    nx, ny, _ = pb.dims
    lo, hi = geo.sub_lo[l], geo.sub_hi[l]
    ext = hi - lo
    patches = geo.sub_patches[l]
    pos = {int(p): t for t, p in enumerate(patches)}
    out = {k: [] for k in ("cell", "gcell", "face", "patch", "lpatch", "sigma", "beta", "T", "area")}
    Ks = (pb.kx, pb.ky, pb.kz)
    for f in range(6):
        t = geo.sub_face_iface[l, f]
        if t < 0:
            continue
        I = geo.ifaces[t]
        d, side = FACES[f]
        a, b = I["a"], I["b"]
        sigma = +1 if side > 0 else -1  # +d face: this subdomain is the lower side
        ia = split_index(I["la"], I["na"])
        ib = split_index(I["lb"], I["nb"])
        H = ext[d] * pb.h[d]
        other = I["hi_sub"] if sigma > 0 else I["lo_sub"]
        H_other = (geo.sub_hi[other][d] - geo.sub_lo[other][d]) * pb.h[d]
        stride = (1, nx, nx * pb.dims[1])[d]
        A = face_area(pb.h, d)
        for tb in range(I["lb"]):
            for ta in range(I["la"]):
                x = [0, 0, 0]
                x[a] = ta
                x[b] = tb
                x[d] = 0 if side < 0 else ext[d] - 1
                lc = x[0] + ext[0] * (x[1] + ext[1] * x[2])
                gc = (lo[0] + x[0]) + nx * ((lo[1] + x[1]) + ny * (lo[2] + x[2]))
                K = Ks[d][gc]
                if beta_mode == 0:
                    beta = robin_beta(alpha, H, K)
                else:
                    Kn = Ks[d][gc + (stride if sigma > 0 else -stride)]
                    beta = robin_beta(alpha, harmonic_mean(H, H_other), harmonic_mean(K, Kn))
                p = I["p0"] + ia[ta] + I["na"] * ib[tb]
                out["cell"].append(lc)
                out["gcell"].append(gc)
                out["face"].append(f)
                out["patch"].append(p)
                out["lpatch"].append(pos[p])
                out["sigma"].append(sigma)
                out["beta"].append(beta)
                out["T"].append(robin_transmissibility(A, pb.h[d], K, beta))
                out["area"].append(A)
    ints = ("cell", "gcell", "face", "patch", "lpatch", "sigma")
    return GammaFaces(**{k: np.asarray(v, dtype=np.int64 if k in ints else np.float64)
                         for k, v in out.items()})


def local_system(pb, geo, l, alpha, beta_mode=0):
    """A^H_l and the right-hand sides of (2.25)/(2.26) for subdomain l."""
    lo, hi = geo.sub_lo[l], geo.sub_hi[l]
    ext = hi - lo
    lx, ly, lz = (int(e) for e in ext)
    Nl = lx * ly * lz
    cells = geo.sub_cells(l)
    idx = np.arange(Nl).reshape(lz, ly, lx)
    Ks = (pb.kx, pb.ky, pb.kz)
    rows, cols, vals = [], [], []
    diag = np.zeros(Nl)
    # interior TPFA faces, eq. (2.10)
    for d in range(3):
        K = Ks[d][cells].reshape(lz, ly, lx)
        ax = 2 - d
        if K.shape[ax] < 2:
            continue
        klo = np.take(K, np.arange(0, K.shape[ax] - 1), axis=ax)
        khi = np.take(K, np.arange(1, K.shape[ax]), axis=ax)
        t = (face_area(pb.h, d) * harmonic(klo, khi) / pb.h[d]).reshape(-1)
        c = np.take(idx, np.arange(0, idx.shape[ax] - 1), axis=ax).reshape(-1)
        n = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).reshape(-1)
        np.add.at(diag, c, t)
        np.add.at(diag, n, t)
        rows += [c, n]
        cols += [n, c]
        vals += [-t, -t]
    # Robin faces on Gamma
    g = gamma_faces(pb, geo, l, alpha, beta_mode)
    np.add.at(diag, g.cell, g.T)
    patches = geo.sub_patches[l]
    n = len(patches)
    m = 2 * n + 1
    R = np.zeros((Nl, m))
    R[:, 0] = np.asarray(pb.q)[cells]
    # P-type columns: G = 1 on patch j; U-type: G = -sigma beta on patch j
    np.add.at(R, (g.cell, 1 + g.lpatch), g.T)
    np.add.at(R, (g.cell, 1 + n + g.lpatch), g.T * (-g.sigma * g.beta))
    # domain walls on this subdomain's boundary (particular problem only)
    gmap = {int(c): t for t, c in enumerate(cells)}
    for f in range(6):
        if geo.sub_face_iface[l, f] >= 0:
            continue
        wt = pb.wall_type[f]
        if wt == 0:
            continue
        d, _ = FACES[f]
        wc = wall_cells(pb.dims, f)
        gv = pb.wall_value[f]
        gv = np.zeros(len(wc)) if gv is None else np.asarray(gv, dtype=np.float64)
        A = face_area(pb.h, d)
        for c, gval in zip(wc, gv):
            t = gmap.get(int(c))
            if t is None:
                continue
            if wt == 1:
                tt = A * 2.0 * Ks[d][c] / pb.h[d]
                diag[t] += tt
                R[t, 0] += tt * gval
            else:
                R[t, 0] -= A * gval
    rows.append(np.arange(Nl))
    cols.append(np.arange(Nl))
    vals.append(diag)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nl, Nl)).tocsr()
    pin_local = -1
    if pb.pin >= 0 and pb.pin in gmap:
        pin_local = gmap[int(pb.pin)]
        M = M.tolil()
        M[pin_local, :] = 0.0
        M[:, pin_local] = 0.0
        M[pin_local, pin_local] = 1.0
        M = M.tocsr()
        R[pin_local, :] = 0.0
    return LocalSystem(l, cells, M, R, g, patches, pin_local)


def robin_data(ls, col):
    """G_f for right-hand-side column col, at every Robin face of the subdomain."""
    g = ls.gamma
    n = len(ls.patches)
    G = np.zeros(len(g.cell))
    if col == 0:
        return G
    if col <= n:
        G[g.lpatch == col - 1] = 1.0
    else:
        sel = g.lpatch == col - 1 - n
        G[sel] = -g.sigma[sel] * g.beta[sel]
    return G


def refined_solve(M, R, extended=True, steps=2):
    """Solve M X = R (sparse, one right-hand side per column): sparse LU in
    FP64, then, when ``extended``, ``steps`` rounds of iterative refinement
    X += M^-1 (R - M X) whose residual is formed in extended precision
    (np.longdouble: a 64-bit significand on x86-64) and whose correction uses
    the same FP64 factor.  While the condition number times the FP64 unit
    roundoff stays below one, each round shrinks the error by that product,
    so two rounds leave X correctly rounded to FP64 up to a few units in the
    last place (classical mixed-precision refinement, Wilkinson; Moler 1967).

    Plain FP64 is not enough for an end-to-end reference at the 1e-8 level:
    the interface system amplifies the rounding errors of the local solves
    (on the 60x220x85 channelised workload a relative change of 1e-15 in the
    interface matrix moves the pressure by 1.7e-8)."""
    lu = spla.splu(M.tocsc())
    X = lu.solve(R)
    if not extended:
        return X
    Ml = M.astype(np.longdouble)
    Rl = np.asarray(R).astype(np.longdouble)
    Xl = X.astype(np.longdouble)
    for _ in range(steps):
        r = Rl - Ml @ Xl
        Xl = Xl + lu.solve(r.astype(np.float64)).astype(np.longdouble)
    return Xl.astype(np.float64)


def local_solve(ls, extended=True):
    """Loop 1 of Algorithm 2 for one subdomain: one factorisation, 2|I^l|+1 solves."""
    return refined_solve(ls.M, ls.R, extended)


def gamma_flux_blocks(ls, X):
    """F[i,col] = sum_{f in i} Q_f[col] and Fb[i,col] = sum_{f in i} beta_f Q_f[col],
    with Q_f = T_f (X[c_f, col] - G_f[col]); plus SAb[i] = sum_{f in i} A_f beta_f."""
    g = ls.gamma
    n = len(ls.patches)
    m = X.shape[1]
    F = np.zeros((n, m))
    Fb = np.zeros((n, m))
    for col in range(m):
        Q = g.T * (X[g.cell, col] - robin_data(ls, col))
        np.add.at(F[:, col], g.lpatch, Q)
        np.add.at(Fb[:, col], g.lpatch, g.beta * Q)
    SAb = np.zeros(n)
    np.add.at(SAb, g.lpatch, g.area * g.beta)
    return F, Fb, SAb


def patch_sigma(ls):
    """sigma of this subdomain on each of its patches."""
    g = ls.gamma
    s = np.zeros(len(ls.patches))
    s[g.lpatch] = g.sigma
    return s


def assemble_interface(n_patch, blocks):
    """Assemble A^int and b^int, eqs. (2.18)-(2.22), from per-subdomain blocks.

    ``blocks`` is a list of (patches, sigma, F, Fb, SAb).  Unknowns are
    X = (pi^p_1..pi^p_NV, pi^u_1..pi^u_NV)."""
    NV = n_patch
    rows, cols, vals = [], [], []
    b = np.zeros(2 * NV)
    for patches, sig, F, Fb, SAb in blocks:
        n = len(patches)
        I = np.repeat(patches, n)
        J = np.tile(patches, n)
        s = np.repeat(sig, n)
        FP = F[:, 1:1 + n].reshape(-1)
        FU = F[:, 1 + n:].reshape(-1)
        GP = Fb[:, 1:1 + n].reshape(-1)
        GU = Fb[:, 1 + n:].reshape(-1)
        rows += [I, I, NV + I, NV + I]
        cols += [J, NV + J, J, NV + J]
        vals += [FP, FU, s * GP, s * GU]
        rows.append(NV + patches)
        cols.append(NV + patches)
        vals.append(-SAb)
        np.add.at(b, patches, -F[:, 0])
        np.add.at(b, NV + patches, -sig * Fb[:, 0])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * NV, 2 * NV)).tocsr()
    return A, b


@dataclass
class MRCMResult:
    p: np.ndarray           # [N] pressure
    U: np.ndarray           # [6, N] outward normal velocity per cell face (own side)
    pi: np.ndarray          # [2 N_V] interface unknowns (pi^p then pi^u)
    A_int: sp.csr_matrix
    b_int: np.ndarray
    X: List[np.ndarray]     # per subdomain [N_l, m_l] MBFs (rows x fastest in the box)
    F: List[np.ndarray]
    Fb: List[np.ndarray]
    SAb: List[np.ndarray]
    systems: List[LocalSystem]
    geo: Geometry


def _one_subdomain(pb, geo, l, alpha, extended, beta_mode=0):
    ls = local_system(pb, geo, l, alpha, beta_mode)
    X = local_solve(ls, extended)
    F, Fb, SAb = gamma_flux_blocks(ls, X)
    return ls, X, F, Fb, SAb


_POOL_ARGS = None


def _pool_task(l):
    pb, geo, alpha, extended, beta_mode = _POOL_ARGS
    return _one_subdomain(pb, geo, l, alpha, extended, beta_mode)


def _pool_init():
    # one BLAS thread per worker process: the parallelism is over subdomains
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass


def build_mbfs(pb, geo, alpha, subdomains=None, extended=True, processes=1, beta_mode=0):
    """Loop 1 of Algorithm 2: local systems, MBFs and their Gamma-flux blocks.

    The subdomains are independent; ``processes`` > 1 spreads them over a
    pool of forked worker processes (same results, subdomain order kept)."""
    global _POOL_ARGS
    subs = list(range(geo.n_sub) if subdomains is None else subdomains)
    if processes > 1 and len(subs) > 1:
        import multiprocessing as mp
        _POOL_ARGS = (pb, geo, alpha, extended, beta_mode)
        try:
            with mp.get_context("fork").Pool(processes, initializer=_pool_init) as pool:
                out = pool.map(_pool_task, subs, chunksize=max(1, len(subs) // (8 * processes)))
        finally:
            _POOL_ARGS = None
    else:
        out = [_one_subdomain(pb, geo, l, alpha, extended, beta_mode) for l in subs]
    systems = [o[0] for o in out]
    Xs = [o[1] for o in out]
    Fs = [o[2] for o in out]
    Fbs = [o[3] for o in out]
    SAbs = [o[4] for o in out]
    return systems, Xs, Fs, Fbs, SAbs


def reconstruct(pb, geo, systems, Xs, pi):
    """Loop 2 of Algorithm 2 by the combination (2.23): p^l = X_l [1, pi^p, pi^u];
    velocities from the TPFA rule inside, the Robin rule on Gamma and the wall
    rules on the boundary.  Returns (p[N], U[6,N])."""
    NV = geo.n_patch
    N = pb.n
    p = np.zeros(N)
    U = np.zeros((6, N))
    for ls, X in zip(systems, Xs):
        c = np.concatenate([[1.0], pi[ls.patches], pi[NV + ls.patches]])
        pl = X @ c
        p[ls.cells] = pl
        _local_velocities(pb, geo, ls, pl, pi, U)
    return p, U


def _local_velocities(pb, geo, ls, pl, pi, U):
    NV = geo.n_patch
    cells = ls.cells
    ext = geo.sub_hi[ls.sub] - geo.sub_lo[ls.sub]
    lx, ly, lz = (int(e) for e in ext)
    P = pl.reshape(lz, ly, lx)
    Ks = (pb.kx, pb.ky, pb.kz)
    Uloc = np.zeros((6, lz, ly, lx))
    for d in range(3):
        K = Ks[d][cells].reshape(lz, ly, lx)
        ax = 2 - d
        if K.shape[ax] < 2:
            continue
        klo = np.take(K, np.arange(0, K.shape[ax] - 1), axis=ax)
        khi = np.take(K, np.arange(1, K.shape[ax]), axis=ax)
        A = face_area(pb.h, d)
        t = A * harmonic(klo, khi) / pb.h[d]
        plo = np.take(P, np.arange(0, P.shape[ax] - 1), axis=ax)
        phi = np.take(P, np.arange(1, P.shape[ax]), axis=ax)
        u = t * (plo - phi) / A
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, P.shape[ax] - 1)
        sl_hi[ax] = slice(1, P.shape[ax])
        Uloc[2 * d + 1][tuple(sl_lo)] = u
        Uloc[2 * d][tuple(sl_hi)] = -u
    Uloc = Uloc.reshape(6, -1)
    g = ls.gamma
    G = pi[g.patch] - g.sigma * g.beta * pi[NV + g.patch]
    Uloc[g.face, g.cell] = g.T * (pl[g.cell] - G) / g.area
    gmap = {int(c): t for t, c in enumerate(cells)}
    for f in range(6):
        wt = pb.wall_type[f]
        if wt == 0:
            continue
        d, _ = FACES[f]
        wc = wall_cells(pb.dims, f)
        gv = pb.wall_value[f]
        gv = np.zeros(len(wc)) if gv is None else np.asarray(gv, dtype=np.float64)
        for c, gval in zip(wc, gv):
            t = gmap.get(int(c))
            if t is None:
                continue
            if wt == 1:
                Uloc[f, t] = 2.0 * Ks[d][c] / pb.h[d] * (pl[t] - gval)
            else:
                Uloc[f, t] = gval
    U[:, cells] = Uloc


def reconstruct_resolve(pb, geo, systems, pi, extended=True):
    """The second option after (2.23): solve the local problems again with the
    Robin data G(pi) = P_H - sigma beta U_H and the particular data, instead of
    combining stored MBFs."""
    NV = geo.n_patch
    p = np.zeros(pb.n)
    for ls in systems:
        g = ls.gamma
        G = pi[g.patch] - g.sigma * g.beta * pi[NV + g.patch]
        rhs = ls.R[:, 0].copy()
        np.add.at(rhs, g.cell, g.T * G)
        if ls.pin_local >= 0:
            rhs[ls.pin_local] = 0.0
        p[ls.cells] = refined_solve(ls.M, rhs, extended)
    return p


def mrcm_solve(case_or_problem, partition=None, iface=None, alpha=None, extended=True, processes=1):
    """Full MRCM (Algorithm 2) on the CPU.  Accepts a Case or its parts.

    ``extended``: refine every local solve and the interface solve with an
    extended-precision residual (see ``refined_solve``); False gives the plain
    FP64 algorithm.  ``processes``: worker processes for loop 1."""
    beta_mode = 0
    if partition is None:
        case = case_or_problem
        pb, partition, iface, alpha = case.problem, case.partition, case.iface, case.alpha
        beta_mode = getattr(case, "beta_mode", 0)
    else:
        pb = case_or_problem
    geo = Geometry(pb.dims, partition, iface)
    systems, Xs, Fs, Fbs, SAbs = build_mbfs(pb, geo, alpha, extended=extended, processes=processes,
                                            beta_mode=beta_mode)
    blocks = [(ls.patches, patch_sigma(ls), F, Fb, SAb)
              for ls, F, Fb, SAb in zip(systems, Fs, Fbs, SAbs)]
    if geo.n_patch > 0:
        A, b = assemble_interface(geo.n_patch, blocks)
        # InterfaceSolver: a sparse LU (the paper uses MUMPS LU), refined
        pi = refined_solve(A, b, extended, steps=3)
    else:
        A, b = sp.csr_matrix((0, 0)), np.zeros(0)
        pi = np.zeros(0)
    p, U = reconstruct(pb, geo, systems, Xs, pi)
    return MRCMResult(p, U, pi, A, b, Xs, Fs, Fbs, SAbs, systems, geo)
