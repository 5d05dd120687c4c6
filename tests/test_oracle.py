"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage or property it checks.  None of them re-types the
oracle's own formulas: they compare it with the fine-grid solve, with closed
forms, with limits the paper states, with library routines and with the
counts the paper prints.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from mrcm_inputs import IfaceSpace, Partition, Problem, Case, small_case, uniform_cuts
from oracle.banded import band_cholesky, band_solve, bandwidth, to_band
from oracle.fine import fine_solve, fine_system
from oracle.geometry import Geometry, count_interface_unknowns, split_index, split_sizes
from oracle.monolithic import dirichlet_local, mrcm_monolithic, neumann_local
from oracle.mrcm import local_system, mrcm_solve, reconstruct_resolve
from oracle.norms import rel_kinv_velocity, rel_l2, rel_l2_pressure

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- T1 ------
@pytest.mark.parametrize("seed", [0, 1])
def test_single_subdomain_equals_fine(seed):
    """With one subdomain there is no skeleton (N_V = 0), so the MRCM local
    problem is the fine problem (Sec. 2.2: the methods differ only on Gamma)."""
    c = small_case((7, 5, 4), (1, 1, 1), seed=seed)
    pf, Uf = fine_solve(c.problem)
    r = mrcm_solve(c)
    assert r.geo.n_patch == 0
    assert rel_l2(r.p, pf) < 1e-13
    assert rel_l2(r.U, Uf) < 1e-13


# ---------------------------------------------------------------- T2 ------
@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3])
@pytest.mark.parametrize("nd", [(2, 2, 2), (3, 2, 1)])
def test_fine_trace_reproduces_fine_solution(alpha, nd):
    """Sec. 2.2: taking P_H = P_h and U_H = U_h (one patch per fine face) makes
    the MRCM and fine-grid solutions coincide, for any Robin parameter."""
    c = small_case((9, 6, 4), nd, split=((0, 0), (0, 0), (0, 0)), seed=3, alpha=alpha)
    pf, Uf = fine_solve(c.problem)
    r = mrcm_solve(c)
    assert rel_l2(r.p, pf) < 1e-10
    assert rel_l2(r.U, Uf) < 1e-9


def test_fine_trace_with_dirichlet_and_neumann_walls():
    """Same statement with non-homogeneous wall data (eqs. (2.5), (2.6)) and no pin."""
    c = small_case((8, 6, 4), (2, 2, 2), split=((0, 0), (0, 0), (0, 0)), seed=4, pin=-1)
    pb = c.problem
    rng = np.random.default_rng(9)
    pb.wall_type = [1, 2, 0, 2, 1, 0]
    pb.wall_value = [rng.standard_normal(6 * 4), 0.1 * rng.standard_normal(6 * 4), None,
                     0.1 * rng.standard_normal(8 * 4), rng.standard_normal(8 * 6), None]
    pf, Uf = fine_solve(pb)
    r = mrcm_solve(c)
    assert rel_l2(r.p, pf) < 1e-10
    assert rel_l2(r.U, Uf) < 1e-9
    # Dirichlet data is met in the half-cell sense: Q = A 2K/h (p - g)
    assert np.allclose(Uf[0, ::8], 2.0 * pb.kx[::8] * (pf[::8] - pb.wall_value[0]), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- T3 ------
def _linear_case(nd, alpha, split=((1, 1), (1, 1), (1, 1)), s=0.7, K=2.5, dims=(12, 6, 4)):
    nx, ny, nz = dims
    N = nx * ny * nz
    h = (2.0, 1.0, 0.5)
    Ax = h[1] * h[2]
    q = np.zeros(N)
    for k in range(nz):
        for j in range(ny):
            q[0 + nx * (j + ny * k)] = s * Ax
            q[nx - 1 + nx * (j + ny * k)] = -s * Ax
    kk = np.full(N, K)
    pin = nx - 1
    pb = Problem(nx, ny, nz, *h, kk, kk.copy(), kk.copy(), q, pin=pin)
    cuts = [np.linspace(0, n, m + 1).round().astype(np.int32) for n, m in zip(dims, nd)]
    return Case("linear", pb, Partition(*cuts), IfaceSpace(split), alpha)


def test_linear_pressure_fine_exact():
    """Constant K and a uniform x-flux s: every x-face carries velocity s, so
    p = -(s h_x / K) i + const is the exact TPFA solution (eqs. (2.9), (2.12))."""
    c = _linear_case((1, 1, 1), 1.0)
    pb = c.problem
    p, U = fine_solve(pb)
    i = np.arange(pb.n) % pb.nx
    exact = -(0.7 * pb.hx / 2.5) * (i - (pb.nx - 1))
    assert np.max(np.abs(p - exact)) < 1e-12
    ux = U[1].reshape(pb.nz, pb.ny, pb.nx)[:, :, :-1]
    assert np.allclose(ux, 0.7, rtol=1e-12)


@pytest.mark.parametrize("alpha", [1e-2, 1.0, 1e2])
def test_linear_pressure_mrcm_exact_for_normal_cuts(alpha):
    """With cuts only normal to grad p the true trace and flux are constant on
    each interface, so they lie in the patch spaces and the MRCM is exact for
    every alpha (uniqueness of (2.13)-(2.16))."""
    c = _linear_case((3, 1, 1), alpha, split=((2, 2), (1, 1), (1, 1)))
    pf, Uf = fine_solve(c.problem)
    r = mrcm_solve(c)
    assert np.max(np.abs(r.p - pf)) < 1e-10
    assert rel_l2(r.U, Uf) < 1e-10


def test_linear_pressure_parallel_cuts_error_decays_as_one_over_alpha():
    """With interfaces parallel to the flow the true normal flux (zero) is a
    patch constant but the trace varies along x: the flux-continuity limit
    (alpha -> infinity) is exact and the MRCM error decays like 1/alpha."""
    errs = []
    alphas = [1e2, 1e3, 1e4]
    for a in alphas:
        c = _linear_case((1, 2, 1), a)
        pf, _ = fine_solve(c.problem)
        r = mrcm_solve(c)
        errs.append(rel_l2(r.p, pf))
    slopes = np.diff(np.log10(errs)) / np.diff(np.log10(alphas))
    assert np.all(np.abs(slopes + 1.0) < 0.1), (errs, slopes)


# ---------------------------------------------------------------- T4 ------
def test_mass_conservation_per_cell_and_per_patch():
    """Each cell balances its own face fluxes against its source (the local
    problems are solved exactly), and each patch carries zero net flux, which
    is (2.15) tested with the patch indicator (Sec. 3.2.5: the MRCM is
    conservative on the support of the interface basis functions)."""
    c = small_case((10, 8, 6), (2, 2, 3), split=((2, 1), (1, 2), (2, 2)), seed=5, std=2.0)
    pb = c.problem
    r = mrcm_solve(c)
    A = np.array([pb.hy * pb.hz, pb.hx * pb.hz, pb.hx * pb.hy])
    Q = r.U * np.repeat(A, 2)[:, None]
    net = Q.sum(axis=0) - pb.q
    scale = np.abs(Q).sum(axis=0) + np.abs(pb.q)
    assert np.max(np.abs(net)) < 1e-12 * np.max(scale)
    # per patch: sum over both sides of the outward fluxes
    geo = r.geo
    bal = np.zeros(geo.n_patch)
    mag = np.zeros(geo.n_patch)
    for t in range(len(geo.ifaces)):
        d = geo.ifaces[t]["d"]
        lo, hi, patch = geo.iface_faces(t)
        qlo = Q[2 * d + 1, lo]
        qhi = Q[2 * d, hi]
        np.add.at(bal, patch, qlo + qhi)
        np.add.at(mag, patch, np.abs(qlo) + np.abs(qhi))
    assert np.max(np.abs(bal) / mag) < 1e-11


# ---------------------------------------------------------------- T5 ------
def test_alpha_limits():
    """alpha -> 0 tends to pressure data on Gamma with weak flux continuity
    (error O(alpha)); alpha -> infinity tends to flux data with weak pressure
    continuity (error O(1/alpha)) -- the two limits named in the Introduction
    and in Sec. 3.2.4."""
    base = dict(dims=(8, 6, 4), nd=(2, 2, 2), split=((2, 1), (1, 2), (2, 2)), seed=2)
    c = small_case(**base)
    pd, _ = dirichlet_local(c)
    pn, _ = neumann_local(c)
    small = [1e-3, 1e-4, 1e-5]
    large = [1e2, 1e3, 1e4]
    ed = [rel_l2(mrcm_solve(small_case(alpha=a, **base)).p, pd) for a in small]
    en = [rel_l2(mrcm_solve(small_case(alpha=a, **base)).p, pn) for a in large]
    sd = np.diff(np.log10(ed)) / np.diff(np.log10(small))
    sn = np.diff(np.log10(en)) / np.diff(np.log10(large))
    assert np.all(np.abs(sd - 1.0) < 0.1), (ed, sd)
    assert np.all(np.abs(sn + 1.0) < 0.1), (en, sn)


# ---------------------------------------------------------------- T6 ------
def test_reconstruction_options_agree():
    """After (2.23) the paper gives two ways to recover the solution: combine
    stored MBFs, or solve the local problems again with the interface data."""
    c = small_case((8, 8, 4), (2, 2, 2), split=((1, 2), (2, 1), (2, 2)), seed=6)
    r = mrcm_solve(c)
    p2 = reconstruct_resolve(c.problem, r.geo, r.systems, r.pi)
    assert rel_l2(p2, r.p) < 1e-12


# ---------------------------------------------------------------- T7 ------
@pytest.mark.parametrize("split", [((1, 1), (1, 1), (1, 1)), ((2, 2), (1, 2), (2, 1))])
def test_monolithic_equals_mbf_path(split):
    """All local pressures and interface unknowns solved as one system, with
    no MBFs and no superposition, equal the MBF path of Algorithm 2."""
    c = small_case((8, 6, 6), (2, 2, 3), split=split, seed=7, std=1.5)
    r = mrcm_solve(c)
    pm, pim = mrcm_monolithic(c)
    assert rel_l2(r.p, pm) < 1e-11
    assert rel_l2(r.pi, pim) < 1e-10


def test_ragged_partition_monolithic():
    c = small_case((9, 7, 5), (3, 2, 2), split=((2, 1), (1, 1), (2, 2)), seed=8,
                   parts=([2, 4, 3], [3, 4], [2, 3]))
    r = mrcm_solve(c)
    pm, _ = mrcm_monolithic(c)
    assert rel_l2(r.p, pm) < 1e-11


# ---------------------------------------------------------------- T8 ------
def test_interface_matrix_structure():
    """A^UP = -(A^PU)^T, A^PP and A^UU symmetric, A^PP <= 0, A^UU < 0.
    (A^PP is minus a sum of Robin-to-flux maps, A^UU minus a sum of positive
    face terms; these follow from (2.19)-(2.21).)"""
    c = small_case((8, 6, 4), (2, 2, 2), split=((1, 2), (2, 1), (2, 2)), seed=1)
    r = mrcm_solve(c)
    A = r.A_int.toarray()
    NV = r.geo.n_patch
    APP, APU, AUP, AUU = A[:NV, :NV], A[:NV, NV:], A[NV:, :NV], A[NV:, NV:]
    assert np.max(np.abs(AUP + APU.T)) < 1e-12 * np.max(np.abs(APU))
    assert np.max(np.abs(APP - APP.T)) < 1e-12 * np.max(np.abs(APP))
    assert np.max(np.abs(AUU - AUU.T)) < 1e-12 * np.max(np.abs(AUU))
    assert np.max(np.linalg.eigvalsh(APP)) < 0
    assert np.max(np.linalg.eigvalsh(AUU)) < 0


def test_interface_null_vector_without_pin():
    """Without a pin and without Dirichlet walls the P-rows annihilate
    (pi^p, pi^u) = (1, 0): a constant pressure drives no flux."""
    c = small_case((8, 6, 4), (2, 2, 2), seed=1, pin=-1, wells=False)
    from oracle.geometry import Geometry as G
    from oracle.mrcm import build_mbfs, patch_sigma, assemble_interface
    geo = G(c.problem.dims, c.partition, c.iface)
    # unpinned local problems are nonsingular thanks to the Robin terms
    systems, Xs, Fs, Fbs, SAbs = build_mbfs(c.problem, geo, 1.0)
    blocks = [(ls.patches, patch_sigma(ls), F, Fb, SAb) for ls, F, Fb, SAb in zip(systems, Fs, Fbs, SAbs)]
    A, b = assemble_interface(geo.n_patch, blocks)
    x = np.concatenate([np.ones(geo.n_patch), np.zeros(geo.n_patch)])
    y = A @ x
    assert np.max(np.abs(y)) < 1e-12 * np.max(np.abs(A.toarray()))


# ---------------------------------------------------------------- T9 ------
def test_band_cholesky_matches_lapack_and_dense():
    """The textbook band factor equals LAPACK's dpbtrf (via SciPy) and the
    dense Cholesky factor, and the band solve equals a sparse LU solve."""
    c = small_case((6, 5, 4), (1, 2, 2), seed=9, std=2.0)
    geo = Geometry(c.problem.dims, c.partition, c.iface)
    ls = local_system(c.problem, geo, 3, 1.0)
    M = ls.M
    b = bandwidth(M)
    assert b == 6 * 3  # lx * ly for x-fastest ordering of a 6x3x2 box
    Lb = band_cholesky(to_band(M, b))
    lap = sla.cholesky_banded(to_band(M, b).T, lower=True)
    assert np.max(np.abs(Lb.T - lap)) < 1e-13 * np.max(np.abs(lap))
    Ld = np.linalg.cholesky(M.toarray())
    assert np.max(np.abs(Lb - to_band(Ld, b))) < 1e-13 * np.max(np.abs(Ld))
    X = band_solve(Lb, ls.R)
    Xs = spla.splu(M.tocsc()).solve(ls.R)
    assert np.max(np.abs(X - Xs)) < 1e-12 * np.max(np.abs(Xs))


def test_band_cholesky_rejects_indefinite():
    A = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(np.linalg.LinAlgError):
        band_cholesky(to_band(A, 1))


# ---------------------------------------------------------------- T10 -----
def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "paper_interface_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((t[0], [int(x) for x in t[2:5]], [int(x) for x in t[5:8]],
                         [int(x) for x in t[8:11]], float(t[11])))
    return rows


@pytest.mark.parametrize("row", _golden_counts(), ids=lambda r: r[0])
def test_interface_unknown_counts_match_paper(row):
    """eq. (2.24) with H-bar = H reproduces the N_Gamma column the paper prints
    (to its rounding; a few printed values are off by up to 0.4K)."""
    name, proc, core, grid, printed_k = row
    nd = [p * c for p, c in zip(proc, core)]
    assert all(g % n == 0 for g, n in zip(grid, nd))
    n_gamma = count_interface_unknowns(nd)
    assert abs(n_gamma / 1000.0 - printed_k) <= 0.4 + 1e-9, (n_gamma, printed_k)


def test_subdomain_sizes_match_paper():
    """Local problem sizes of the weak-scaling runs: 22K cells (Table of the
    weak-scaling decomposition: 80x1760x160 over 8x8x16 subdomains)."""
    assert (80 // 8) * (1760 // 8) * (160 // 16) == 22000
    # strong scaling: 2.4K, 19.0K and 32.0K cells for the 60x10x50 decomposition
    assert (360 // 60) * (660 // 10) * (300 // 50) == 2376
    assert (720 // 60) * (1320 // 10) * (600 // 50) == 19008
    assert (660 // 60) * (2420 // 10) * (600 // 50) == 31944


def test_rhs_count_per_interior_subdomain():
    """Sec. 2.2.3: one patch per face gives 12 MBF solves + 1 particular = 13
    right-hand sides for an interior subdomain; splitting every face in two
    gives 25."""
    c = small_case((9, 9, 9), (3, 3, 3), seed=0)
    geo = Geometry(c.problem.dims, c.partition, c.iface)
    centre = geo.sub_id((1, 1, 1))
    assert 2 * len(geo.sub_patches[centre]) + 1 == 13
    c2 = small_case((9, 9, 9), (3, 3, 3), split=((2, 1), (2, 1), (2, 1)), seed=0)
    geo2 = Geometry(c2.problem.dims, c2.partition, c2.iface)
    assert 2 * len(geo2.sub_patches[centre]) + 1 == 25


def test_patch_split_is_balanced_and_contiguous():
    for n in range(1, 25):
        for k in range(1, n + 1):
            sizes = split_sizes(n, k)
            assert sum(sizes) == n and max(sizes) - min(sizes) <= 1
            idx = split_index(n, k)
            assert np.all(np.diff(idx) >= 0) and idx[0] == 0 and idx[-1] == k - 1
            assert np.all(np.bincount(idx) == sizes)


# ------------------------------------------------------------- norms ------
def test_norms_reduce_to_plain_l2_for_unit_data():
    c = small_case((4, 3, 2), (1, 1, 1), seed=0)
    pb = c.problem
    pb.kx[:] = pb.ky[:] = pb.kz[:] = 1.0
    U = np.random.default_rng(0).standard_normal((6, pb.n))
    Z = np.zeros_like(U)
    # unit K, unit cells: ||u||^2 = sum (1/2) u^2 over all 6 faces
    assert np.isclose(rel_kinv_velocity(Z, U, pb), 1.0)
    assert np.isclose(rel_l2_pressure(2 * U[0], U[0]), 1.0)


# ------------------------------------------------------ T3 with walls -----
def _wall_case(d, kind, dims=(8, 6, 5), nd=(2, 2, 1), split=((1, 1), (1, 1), (1, 1)), alpha=1.0):
    """Constant K, no sources, flow along axis d driven by the two walls
    normal to d; every other wall is no-flow and nothing is pinned.
    kind 'dd': Dirichlet g0 on the - wall and g1 on the + wall.
    kind 'nd': Neumann inflow s on the - wall (outward velocity -s),
               Dirichlet g1 on the + wall.
    kind 'dn': Dirichlet g0 on the - wall, Neumann outflow s on the + wall."""
    nx, ny, nz = dims
    N = nx * ny * nz
    h = (2.0, 1.0, 0.5)
    K = (2.5, 0.7, 0.3)   # anisotropic but constant: only K_d drives the flow
    pb = Problem(nx, ny, nz, *h, np.full(N, K[0]), np.full(N, K[1]), np.full(N, K[2]), np.zeros(N), pin=-1)
    n_wall = N // dims[d]
    g0, g1, s = 1.3, -0.4, 0.25
    wt = [0] * 6
    wv = [None] * 6
    if kind == "dd":
        wt[2 * d], wv[2 * d] = 1, np.full(n_wall, g0)
        wt[2 * d + 1], wv[2 * d + 1] = 1, np.full(n_wall, g1)
    elif kind == "nd":
        wt[2 * d], wv[2 * d] = 2, np.full(n_wall, -s)
        wt[2 * d + 1], wv[2 * d + 1] = 1, np.full(n_wall, g1)
    else:
        wt[2 * d], wv[2 * d] = 1, np.full(n_wall, g0)
        wt[2 * d + 1], wv[2 * d + 1] = 2, np.full(n_wall, s)
    pb.wall_type, pb.wall_value = wt, wv
    cuts = [np.linspace(0, n, k + 1).round().astype(np.int32) for n, k in zip(dims, nd)]
    case = Case("walls", pb, Partition(*cuts), IfaceSpace(split), alpha)
    # closed forms along axis d (i = cell coordinate, n cells of size hd)
    n, hd, Kd = dims[d], h[d], K[d]
    i = (np.arange(N) // (1, nx, nx * ny)[d]) % n
    if kind == "dd":
        # half-cell rule at both walls: the pressure drop g0 - g1 splits into
        # n - 1 full cell spacings and two half cells, all of resistance h/K
        exact = g0 + (g1 - g0) * (i + 0.5) / n
        vel = -Kd * (g1 - g0) / (n * hd)       # velocity along +e_d
    elif kind == "nd":
        exact = g1 + s * hd * (n - i - 0.5) / Kd
        vel = s
    else:
        exact = g0 - s * hd * (i + 0.5) / Kd
        vel = s
    return case, exact, vel


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("kind", ["dd", "nd", "dn"])
def test_wall_closed_forms_fine(d, kind):
    """Eqs. (2.5), (2.6) with constant K: between a Dirichlet and a Dirichlet
    or Neumann wall the TPFA pressure is linear in the cell coordinate, with a
    half cell of resistance h/(2K) between the last cell centre and a
    Dirichlet wall, and a Neumann wall passing exactly its data.  A full-cell
    wall term, or the opposite sign of the Neumann datum, changes the answer."""
    case, exact, vel = _wall_case(d, kind)
    pb = case.problem
    p, U = fine_solve(pb)
    assert np.max(np.abs(p - exact)) < 1e-12 * max(1.0, np.max(np.abs(exact)))
    # every face normal to d carries the same velocity along +e_d, walls included
    assert np.allclose(U[2 * d + 1], vel, rtol=1e-12, atol=1e-13)
    assert np.allclose(U[2 * d], -vel, rtol=1e-12, atol=1e-13)
    for e in range(3):
        if e != d:
            assert np.max(np.abs(U[2 * e])) < 1e-12 and np.max(np.abs(U[2 * e + 1])) < 1e-12


@pytest.mark.parametrize("kind", ["dd", "nd", "dn"])
@pytest.mark.parametrize("alpha", [1e-2, 1.0, 1e2])
def test_wall_closed_forms_mrcm(kind, alpha):
    """The same closed forms through the MRCM's local problems (walls enter
    only the particular problem (2.26)).  Cuts normal to the flow carry a
    constant trace and flux, which the one-patch spaces contain, so the MRCM
    is exact for every alpha; cuts parallel to the flow are exact with the
    fine trace (Sec. 2.2)."""
    for d, nd, split in ((0, (3, 1, 1), ((1, 1), (1, 1), (1, 1))),
                         (1, (1, 2, 1), ((1, 1), (1, 1), (1, 1))),
                         (2, (2, 2, 2), ((0, 0), (0, 0), (0, 0)))):
        case, exact, vel = _wall_case(d, kind, nd=nd, split=split, alpha=alpha)
        r = mrcm_solve(case)
        assert np.max(np.abs(r.p - exact)) < 1e-10 * max(1.0, np.max(np.abs(exact))), (d, kind)
        assert np.allclose(r.U[2 * d + 1], vel, rtol=1e-9, atol=1e-11)
        assert np.allclose(r.U[2 * d], -vel, rtol=1e-9, atol=1e-11)
        # the monolithic formulation, which assembles its walls separately
        pm, _ = mrcm_monolithic(case)
        assert np.max(np.abs(pm - exact)) < 1e-10 * max(1.0, np.max(np.abs(exact))), (d, kind)


# ------------------------------------------------ shared (face) beta -----
def test_face_beta_equals_per_side_beta_where_both_sides_agree():
    """With K constant across every interface and equal subdomain extents,
    the per-side and the face-shared Robin parameters coincide face by face,
    so the two readings give the same MRCM solution (up to rounding)."""
    c = small_case((8, 6, 4), (2, 2, 2), split=((2, 1), (1, 2), (2, 2)), seed=3)
    pb = c.problem
    pb.kx[:] = 2.0
    pb.ky[:] = 0.5
    pb.kz[:] = 0.3
    r0 = mrcm_solve(c)
    c.beta_mode = 1
    r1 = mrcm_solve(c)
    assert rel_l2(r1.p, r0.p) < 1e-12 and rel_l2(r1.pi, r0.pi) < 1e-12


@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3])
def test_face_beta_keeps_the_fine_trace_exact_and_the_monolithic_form(alpha):
    """Sec. 2.2: the fine-trace spaces reproduce the fine solution for any
    positive Robin parameter on each side, the shared face value included;
    and the MBF path equals the monolithic solve under it."""
    c = small_case((9, 6, 4), (3, 2, 1), split=((0, 0), (0, 0), (0, 0)), seed=3, alpha=alpha, std=2.0)
    c.beta_mode = 1
    pf, Uf = fine_solve(c.problem)
    r = mrcm_solve(c)
    assert rel_l2(r.p, pf) < 1e-10 and rel_l2(r.U, Uf) < 1e-9
    c2 = small_case((8, 6, 6), (2, 2, 3), split=((2, 2), (1, 2), (2, 1)), seed=7, std=1.5, alpha=alpha)
    c2.beta_mode = 1
    r2 = mrcm_solve(c2)
    pm, _ = mrcm_monolithic(c2)
    assert rel_l2(r2.p, pm) < 1e-11


def test_face_beta_is_symmetric_across_each_interface():
    """The shared value is the same seen from both sides: the two sides'
    Robin faces of every fine face carry one beta."""
    from oracle.mrcm import gamma_faces
    c = small_case((9, 7, 5), (3, 2, 2), split=((2, 1), (1, 1), (2, 2)), seed=8, std=2.0,
                   parts=([2, 4, 3], [3, 4], [2, 3]))
    pb = c.problem
    geo = Geometry(pb.dims, c.partition, c.iface)
    seen = {}
    for l in range(geo.n_sub):
        g = gamma_faces(pb, geo, l, 0.7, beta_mode=1)
        d = g.face // 2
        stride = np.array([1, pb.nx, pb.nx * pb.ny])[d]
        other = np.where(g.sigma > 0, g.gcell + stride, g.gcell - stride)
        for a, b, beta in zip(g.gcell, other, g.beta):
            key = (min(a, b), max(a, b))
            if key in seen:
                assert abs(seen[key] - beta) <= 1e-15 * beta
            else:
                seen[key] = beta
    assert len(seen) > 0
