"""The 600x2200x85 workload (112.2M cells, 56,100 subdomains of 20x20x5,
430,840 patches, an interface system of 861,680 unknowns; channelised field
raised to a permeability contrast of 1e8) on one GPU with every factor
resident.  The oracle cannot solve it whole, so:
  * the 60x220x85 block at its origin corner (the exact permeability, laid
    out as the 60x220x85 workload) runs end to end on the GPU and in the whole
    oracle: pi, p and U at 1e-8, flux blocks at 1e-9;
  * at full size, the MBFs and flux blocks of sampled subdomains are compared
    with the oracle's, the interface solve's relative residual is small, and
    the reconstructed velocities balance every cell's source to 1e-8 of the
    largest face flux.
FP64 and FP32 with FP64 refinement alike.
"""
import os
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config5, config5_block  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from oracle.mrcm import build_mbfs as oracle_build, mrcm_solve  # noqa: E402
from oracle.norms import rel_l2  # noqa: E402


def _maxrel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def _procs():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def case5():
    t0 = time.perf_counter()
    c = config5()
    print(f"600x2200x85 inputs: {time.perf_counter() - t0:.1f} s, contrast exponent {c.theta:.4f}", flush=True)
    return c


@pytest.mark.parametrize("precision", [0, 1])
def test_cfg5_block_against_the_whole_oracle(case5, precision):
    import paper_2103_08513_amd as lib
    block = config5_block(case5)
    pb = block.problem
    ref = mrcm_solve(block, processes=_procs())
    m = lib.MRCM(pb, block.partition, block.iface, alpha=block.alpha, precision=precision)
    args = [torch.as_tensor(a, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    p, U, X = m.solve(*args, refine=2)
    torch.cuda.synchronize()
    worst = 0.0
    for l in range(len(ref.systems)):
        F, Fb, _ = m.copy_flux(l)
        worst = max(worst, _maxrel(F, ref.F[l]), _maxrel(Fb, ref.Fb[l]))
    ep, eu, epi = rel_l2(p.cpu().numpy(), ref.p), rel_l2(U.cpu().numpy(), ref.U), rel_l2(X.cpu().numpy(), ref.pi)
    print(f"60x220x85 block of the 600x2200x85 field, precision {precision}: flux blocks {worst:.2e}, "
          f"pi {epi:.2e}, p {ep:.2e}, U {eu:.2e}", flush=True)
    assert worst < 1e-9
    assert epi < 1e-8 and ep < 1e-8 and eu < 1e-8
    m.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_cfg5_full_size(case5, precision):
    import paper_2103_08513_amd as lib
    c = case5
    pb = c.problem
    args = [torch.as_tensor(a, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    m = lib.MRCM(pb, c.partition, c.iface, alpha=c.alpha, precision=precision)
    t0 = time.perf_counter()
    p, U, X = m.solve(*args, refine=2)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    info = m.info()
    assert info.n_sub == 56100 and info.n_patch == 430840 and info.n_mbfs == 4 * 430840
    if precision == 1:
        assert info.ir_residual <= 1e-11
    m.solve_interface(X, refine=2, residual=True)
    ii = m.interface_info()
    print(f"600x2200x85, precision {precision}: first solve {t:.2f} s (allocations included), device "
          f"{(info.device_bytes + ii.device_bytes) / 1e9:.1f} GB, interface n {ii.n}, {ii.nodes} separators, "
          f"largest front {ii.max_front}, residual {m.interface_residual:.2e}", flush=True)
    assert m.interface_residual < 1e-10
    # per-cell mass balance of the reconstructed velocities
    Uh = U.cpu().numpy()
    A = np.array([pb.hy * pb.hz, pb.hx * pb.hz, pb.hx * pb.hy])
    Q = Uh * np.repeat(A, 2)[:, None]
    worst = float(np.max(np.abs(Q.sum(axis=0) - pb.q)) / np.max(np.abs(Q)))
    del Uh, Q
    # sampled subdomains: corners, the two well columns' subdomains, interior
    geo = Geometry(pb.dims, c.partition, c.iface)
    sample = sorted({0, 29, 3270, 3299, 56099, 56070, 28050, 28079, 12345, 40000})
    _, Xs, Fs, Fbs, _ = oracle_build(pb, geo, c.alpha, subdomains=sample, processes=_procs())
    emb = 0.0
    for l, Xo, Fo, Fbo in zip(sample, Xs, Fs, Fbs):
        Xg = m.copy_mbfs(l)[np.argsort(m.local_order(l))]
        for col in range(Xo.shape[1]):
            emb = max(emb, _maxrel(Xg[:, col], Xo[:, col]))
        F, Fb, _ = m.copy_flux(l)
        emb = max(emb, _maxrel(F, Fo), _maxrel(Fb, Fbo))
    print(f"600x2200x85, precision {precision}: mass imbalance {worst:.2e} of the largest face flux; "
          f"sampled MBFs and flux blocks {emb:.2e}", flush=True)
    assert worst < 1e-8
    assert emb < 1e-9
    if precision == 1:
        _mean_at_full_size(m, pb, c.partition, U)
    m.close()


def _mean_at_full_size(m, pb, part, U):
    """The Mean post-processing of the reconstructed velocity at full size (the
    factor scratch in chunks), checked by properties that hold at any size:
    one value per face, Gamma faces the two sides' mean, walls unchanged,
    pinned cells at zero, and every other cell's balance."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pt, Ut = m.postprocess_mean(U.reshape(-1))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    pt, Ut = m.postprocess_mean(U.reshape(-1), pt=pt, Ut=Ut.reshape(-1))
    torch.cuda.synchronize()
    t2 = time.perf_counter() - t0 - t
    nx, ny, nz = pb.dims
    G = Ut.reshape(6, nz, ny, nx)
    U6 = U.reshape(6, nz, ny, nx)
    for d in range(3):
        ax = 3 - d  # tensor axis of grid axis d in [6][nz][ny][nx]
        n = pb.dims[d]
        lo = G[2 * d + 1].narrow(ax - 1, 0, n - 1)
        hi = G[2 * d].narrow(ax - 1, 1, n - 1)
        assert torch.equal(lo, -hi), d
        cuts = torch.as_tensor(np.asarray(part.cuts[d][1:-1], dtype=np.int64) - 1, device="cuda")
        mean = 0.5 * (U6[2 * d + 1].index_select(ax - 1, cuts) - U6[2 * d].index_select(ax - 1, cuts + 1))
        assert torch.equal(G[2 * d + 1].index_select(ax - 1, cuts), mean), d
        for f, pos in ((2 * d, 0), (2 * d + 1, n - 1)):
            assert torch.equal(G[f].select(ax - 1, pos), U6[f].select(ax - 1, pos)), f
    A = torch.tensor([pb.hy * pb.hz, pb.hy * pb.hz, pb.hx * pb.hz, pb.hx * pb.hz, pb.hx * pb.hy, pb.hx * pb.hy],
                     dtype=torch.float64, device="cuda")
    Q = Ut.reshape(6, -1) * A[:, None]
    bal = (Q.sum(dim=0) - torch.as_tensor(pb.q, device="cuda")).abs()
    qmax = float(Q.abs().max())
    del Q
    pinned = torch.zeros(pb.n, dtype=torch.bool, device="cuda")
    lo = [torch.as_tensor(np.asarray(cut[:-1], dtype=np.int64), device="cuda") for cut in part.cuts]
    corner = (lo[0][None, None, :] + nx * (lo[1][None, :, None] + ny * lo[2][:, None, None])).reshape(-1)
    pinned[corner] = True
    assert torch.all(pt[pinned] == 0.0)
    free = float(bal[~pinned].max()) / qmax
    defect = float(bal[pinned].max()) / qmax
    print(f"600x2200x85 Mean: {t:.2f} s first call (set-up included), {t2 * 1e3:.1f} ms second; balance of the "
          f"free cells {free:.2e}, of the pinned cells {defect:.2e} of the largest face flux", flush=True)
    assert free < 1e-10
    assert defect < 1e-6
