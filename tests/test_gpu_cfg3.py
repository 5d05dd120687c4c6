"""The ragged 200x440x170 workload (about 15M cells, 9,108 subdomains of eight
shapes from 15x15x3 to 20x20x5, 2-8 patches per interface, 120,176 patches) on
one GPU, end to end in FP64.  The oracle cannot solve it whole, so:
  * the MBFs and flux blocks of one subdomain of every shape (and a few more)
    are compared with the oracle's, column by column (1e-9 relative);
  * the interface solve's relative residual on the assembled system is small,
    and one FP64 refinement step keeps it small;
  * the reconstructed velocity conserves mass in every cell: the net outflow
    equals the source to 1e-8 of the largest face flux in the domain (a
    property that holds at any size).  The balance is the local solves'
    rounding times the interface coefficients; with log-k of standard
    deviation 3 (permeabilities spread over about eight orders of magnitude)
    it measures 3e-10 (test_gpu_parity.py holds a small case with log-k
    standard deviation 2 to 1e-12 of each cell's face fluxes).
The FP32 form with FP64 refinement is held to the same three checks on the
same inputs: its ragged batches, two-stream pipeline and per-column
refinement at the full 9,108-subdomain size.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config3  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from oracle.mrcm import build_mbfs as oracle_build  # noqa: E402


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _maxrel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


@pytest.fixture(scope="module")
def case3():
    t0 = time.perf_counter()
    case = config3()
    print(f"cfg3 inputs: {time.perf_counter() - t0:.1f} s", flush=True)
    return case


def _sampled_mbfs_match_oracle(m, case, tol):
    """One subdomain of every shape, and two more, against the oracle."""
    pb = case.problem
    geo = Geometry(pb.dims, case.partition, case.iface)
    first = {}
    for l in range(geo.n_sub):
        first.setdefault(tuple(int(x) for x in geo.sub_hi[l] - geo.sub_lo[l]), l)
    sample = sorted(set(first.values()) | {4553, 9107})
    _, Xs, Fs, _, _ = oracle_build(pb, geo, case.alpha, subdomains=sample)
    for l, Xo, Fo in zip(sample, Xs, Fs):
        Xg = m.copy_mbfs(l)[np.argsort(m.local_order(l))]
        for c in range(Xo.shape[1]):
            assert _maxrel(Xg[:, c], Xo[:, c]) < tol, (l, c)
        Fg, _, _ = m.copy_flux(l)
        assert _maxrel(Fg, Fo) < tol, l


def _mass_imbalance(pb, U):
    """Largest per-cell |net outflow - source| over the largest face flux."""
    Uh = U.cpu().numpy()
    A = np.array([pb.hy * pb.hz, pb.hx * pb.hz, pb.hx * pb.hy])
    Q = Uh * np.repeat(A, 2)[:, None]
    net = np.abs(Q.sum(axis=0) - pb.q)
    return float(np.max(net) / np.max(np.abs(Q))), float(np.max(net / (np.max(np.abs(Q), axis=0) + 1e-300)))


def test_cfg3_ragged_workload_end_to_end(case3):
    import paper_2103_08513_amd as lib
    case = case3
    pb = case.problem
    m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha)
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    m.build_mbfs(*args)  # creates the handle
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.build_mbfs(*args)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = m.info()
    assert info.n_sub == 9108 and info.n_patch == 120176
    t0 = time.perf_counter()
    m.assemble_interface()
    X = m.solve_interface(residual=True)
    p, U = m.reconstruct(X)
    torch.cuda.synchronize()
    t_rest = time.perf_counter() - t0
    n_if, w = m.interface_dims()
    print(f"cfg3: build {1e3 * t_build:.1f} ms ({info.n_mbfs} MBFs), interface n = {n_if}, bandwidth {w}, "
          f"assembly + solve + reconstruction {1e3 * t_rest:.0f} ms, interface residual "
          f"{m.interface_residual:.2e}", flush=True)
    assert m.interface_residual < 1e-9
    # one FP64 refinement step of the interface solve: residual of the
    # unfactored system, lower and upper sweeps with the stored factors (the
    # ring-buffer lower sweep of systems beyond the LDS-resident size)
    res0 = m.interface_residual
    X1 = m.solve_interface(refine=1, residual=True)
    torch.cuda.synchronize()
    print(f"cfg3: interface residual after one refinement step {m.interface_residual:.2e} "
          f"(before {res0:.2e})", flush=True)
    assert m.interface_residual < max(1e-12, 2.0 * res0)
    assert float(torch.linalg.norm(X1 - X) / torch.linalg.norm(X)) < 1e-6
    # sampled MBFs against the oracle: one subdomain of every shape, and more
    _sampled_mbfs_match_oracle(m, case, 1e-9)
    # mass conservation per cell from the reconstructed velocities
    worst, local = _mass_imbalance(pb, U)
    print(f"cfg3: largest per-cell mass imbalance {worst:.2e} of the largest face flux "
          f"({local:.2e} of the cell's own largest face flux)", flush=True)
    assert worst < 1e-8
    m.close()


def test_cfg3_fp32_form(case3):
    import paper_2103_08513_amd as lib
    case = case3
    pb = case.problem
    m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=lib.FP32_IR)
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    m.build_mbfs(*args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.build_mbfs(*args)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = m.info()
    print(f"cfg3 FP32 form: build {1e3 * t_build:.1f} ms, {info.ir_iters} refinement sweeps to "
          f"{info.ir_residual:.2e}", flush=True)
    # log-k of standard deviation 3: columns whose FP64 residual stalls at
    # the rounding bound of its own evaluation stop there, just above 1e-13
    assert info.ir_residual <= 1e-11
    m.assemble_interface()
    X = m.solve_interface(residual=True)
    p, U = m.reconstruct(X)
    torch.cuda.synchronize()
    assert m.interface_residual < 1e-9
    _sampled_mbfs_match_oracle(m, case, 1e-9)
    worst, local = _mass_imbalance(pb, U)
    print(f"cfg3 FP32 form: interface residual {m.interface_residual:.2e}, largest per-cell mass imbalance "
          f"{worst:.2e} of the largest face flux", flush=True)
    assert worst < 1e-8
    m.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_cfg3_shaped_block_against_the_whole_oracle(precision):
    """A 70x70x19 block with the ragged workload's structure (eight subdomain
    shapes in one launch, 2-8 patches per interface, log-k std 3), small enough
    for the whole oracle: every subdomain's MBFs and flux blocks, the
    interface system, pi, p and U, in FP64 and in FP32 with refinement."""
    import paper_2103_08513_amd as lib
    from mrcm_inputs import config3_block
    from oracle.mrcm import mrcm_solve
    from oracle.norms import rel_l2
    case = config3_block()
    pb = case.problem
    ref = mrcm_solve(case, processes=8)
    m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=precision)
    p, U, X = m.solve(_dev(pb.kx), _dev(pb.ky), _dev(pb.kz), _dev(pb.q), refine=1)
    torch.cuda.synchronize()
    worst = 0.0
    for l in range(len(ref.systems)):
        Xg = m.copy_mbfs(l)
        Xo = ref.X[l][m.local_order(l)]
        for c in range(Xo.shape[1]):
            worst = max(worst, _maxrel(Xg[:, c], Xo[:, c]))
        F, Fb, _ = m.copy_flux(l)
        worst = max(worst, _maxrel(F, ref.F[l]), _maxrel(Fb, ref.Fb[l]))
    A, b = m.copy_interface()
    e_a, e_b = _maxrel(A, ref.A_int.toarray()), _maxrel(b, ref.b_int)
    ep, eu, epi = rel_l2(p.cpu().numpy(), ref.p), rel_l2(U.cpu().numpy(), ref.U), rel_l2(X.cpu().numpy(), ref.pi)
    print(f"70x70x19 ragged block, precision {precision}: MBF/flux blocks {worst:.2e}, A_int {e_a:.2e}, "
          f"b_int {e_b:.2e}, pi {epi:.2e}, p {ep:.2e}, U {eu:.2e}", flush=True)
    assert worst < 1e-9
    assert e_a < 1e-10 and e_b < 1e-10
    assert epi < 1e-8 and ep < 1e-8 and eu < 1e-8
    m.close()


def test_cfg3_autotune_cache_and_recorded_step(case3, tmp_path):
    """Orchestration at the cfg3 size: the autotuner (build tunables and the
    interface panel width) with its per-shape cache -- a second call is a
    hit with the same values -- and the tuned step recorded as a HIP graph,
    whose replays equal the eager step bitwise."""
    import paper_2103_08513_amd as lib
    pb = case3.problem
    stream = torch.cuda.Stream()
    cache = tmp_path / "tune.txt"
    with torch.cuda.stream(stream):
        kx, ky, kz, q = (_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q))
        m = lib.MRCM(pb, case3.partition, case3.iface, alpha=case3.alpha, precision=lib.FP64)
        t0 = time.perf_counter()
        first = m.autotune(kx, ky, kz, q, stream=stream, cache=str(cache))
        t1 = time.perf_counter()
        again = m.autotune(kx, ky, kz, q, stream=stream, cache=str(cache))
        t2 = time.perf_counter()
        print(f"cfg3 autotune {first} in {t1 - t0:.1f} s; cached {again['from_cache']} in {t2 - t1:.3f} s",
              flush=True)
        assert not first["from_cache"] and again["from_cache"]
        for key in ("solve_tiles", "solve_group", "iface_panel"):
            assert again[key] == first[key]
        assert 1 <= first["iface_panel"] <= 4
        assert len(cache.read_text().splitlines()) == 1
        m.solve(kx, ky, kz, q, refine=1)  # handles with the tuned values
        nv = m.info().n_patch
        X = torch.empty(2 * nv, dtype=torch.float64, device="cuda")
        p = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        U = torch.empty(6 * pb.n, dtype=torch.float64, device="cuda")
        g = m.capture(kx, ky, kz, q, X, p, U, refine=1, stream=stream)
        for k in range(3):
            g.launch(stream=stream)
            g.check(stream=stream)
            p_g, U_g, X_g = p.clone(), U.clone(), X.clone()
            p_e, U_e, X_e = m.solve(kx, ky, kz, q, refine=1)
            stream.synchronize()
            assert torch.equal(p_g, p_e), k
            assert torch.equal(U_g, U_e.reshape(-1)), k
            assert torch.equal(X_g, X_e), k
        g.close()
        m.close()
