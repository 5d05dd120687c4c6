"""GPU parity of the learned warm start (include/mrcm_nn.h) with the oracle
(oracle/surrogate.py), through the C ABI:
  * convolution forward, its gradients (input with the ReLU mask, weights,
    bias), the network's loss and parameter gradients, and Adam steps, at
    FP32 tolerances (relative 1e-5 for one layer, 1e-4 through the network);
  * inputs and targets gathered from a built handle against the oracle's
    features of its own local systems and solutions;
  * the scatter of network outputs into the MBF layout;
  * training on the 40x40x20 workload's fields lowers the loss, and on an
    unseen field the trained network's Galerkin-scaled starting guess is
    closer to the exact MBFs in the energy norm than a zero start.  The
    conjugate-gradient iterations to the 1e-10 residual are reported both
    ways: the guess is too coarse (tens of percent) to shorten a solve that
    has to gain ten orders of magnitude.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config1, small_case  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from oracle.mrcm import local_solve, local_system  # noqa: E402
from oracle import surrogate as onn  # noqa: E402


def _f32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _lib():
    from paper_2103_08513_amd import _lib
    return _lib.load()


def _s():
    from ctypes import c_void_p
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    from ctypes import c_void_p
    return None if t is None else c_void_p(t.data_ptr())


SHAPES = [(3, 2, 8, (4, 5, 3), 1), (2, 8, 8, (20, 20, 5), 1), (2, 8, 1, (5, 4, 6), 1),
          (1, 16, 16, (3, 3, 3), 1), (2, 12, 12, (20, 20, 5), 2), (2, 12, 12, (10, 10, 5), 4)]


@pytest.mark.parametrize("B,ci,co,dims,dil", SHAPES)
def test_conv3d_forward_and_backward(B, ci, co, dims, dil):
    rng = np.random.default_rng(B * 100 + ci * 10 + co)
    d, h, w = dims
    x = rng.standard_normal((B, ci) + dims)
    wt = rng.standard_normal((co, ci, 3, 3, 3)) * 0.2
    b = rng.standard_normal(co)
    dy = rng.standard_normal((B, co) + dims)
    mask = np.maximum(rng.standard_normal((B, ci) + dims), 0.0)
    lib = _lib()
    xg, wg, bg = _f32(x), _f32(wt), _f32(b)
    y = torch.empty((B, co) + dims, dtype=torch.float32, device="cuda")
    assert lib.mrcm_conv3d_forward(_p(xg), _p(wg), _p(bg), _p(y), None, B, ci, co, d, h, w, dil, 0, _s()) == 0
    yo = onn.conv3d(x, wt, b, dil).numpy()
    assert _rel(y.cpu().numpy(), yo) < 1e-5
    # relu variant
    assert lib.mrcm_conv3d_forward(_p(xg), _p(wg), _p(bg), _p(y), None, B, ci, co, d, h, w, dil, 1, _s()) == 0
    assert _rel(y.cpu().numpy(), np.maximum(yo, 0.0)) < 1e-5
    dx = torch.empty_like(xg)
    dw = torch.empty_like(wg)
    db = torch.empty_like(bg)
    ws = torch.empty(co * ci * 27, dtype=torch.float32, device="cuda")
    assert lib.mrcm_conv3d_backward(_p(xg), _p(wg), _p(_f32(dy)), _p(dx), _p(dw), _p(db), _p(ws),
                                    _p(_f32(mask)), B, ci, co, d, h, w, dil, _s()) == 0
    gx, gw, gb = onn.layer_grads(x, wt, b, dy, dil)
    assert _rel(dx.cpu().numpy(), gx * (mask > 0)) < 1e-5
    assert _rel(dw.cpu().numpy(), gw) < 1e-5
    assert _rel(db.cpu().numpy(), gb) < 1e-5


def test_network_loss_and_gradients_match_oracle():
    from paper_2103_08513_amd.surrogate import WarmStartNet
    net = WarmStartNet(seed=3)
    rng = np.random.default_rng(4)
    dims = (6, 5, 4)
    x = rng.standard_normal((5, 2) + dims)
    t = rng.standard_normal((5, 1) + dims)
    loss, grads = net.loss_and_grads(_f32(x), _f32(t), dims)
    params = [p.cpu().numpy().astype(np.float64) for p in net.params]
    lo, go, _ = onn.loss_and_grads(params, x, t, list(net.dilations))
    assert abs(float(loss.item()) - lo) < 1e-5 * lo
    for g, gref in zip(grads, go):
        assert _rel(g.cpu().numpy(), gref) < 1e-4


def test_adam_steps_match_oracle():
    rng = np.random.default_rng(5)
    n = 1000
    p = rng.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    pg, mg, vg = _f32(p), _f32(m), _f32(v)
    lib = _lib()
    from ctypes import c_float
    for t in (1, 2, 3):
        g = rng.standard_normal(n)
        assert lib.mrcm_adam_step(_p(pg), _p(_f32(g)), _p(mg), _p(vg), n, t, c_float(1e-2), c_float(0.9),
                                  c_float(0.999), c_float(1e-8), _s()) == 0
        p, m, v = onn.adam_step(p, g, m, v, t, 1e-2)
    assert _rel(pg.cpu().numpy(), p) < 1e-5


def _fp64_model(case):
    import paper_2103_08513_amd as lib
    pb = case.problem
    mdl = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=lib.FP64, fp64_refine=1)
    mdl.build_mbfs(_dev(pb.kx), _dev(pb.ky), _dev(pb.kz), _dev(pb.q))
    torch.cuda.synchronize()
    return mdl


def test_features_targets_and_scatter_match_oracle():
    from paper_2103_08513_amd.surrogate import features, net_subdomains
    case = small_case((40, 20, 5), (2, 1, 1), split=((2, 2), (1, 1), (1, 1)), seed=22)
    pb = case.problem
    mdl = _fp64_model(case)
    subs, dims = net_subdomains(mdl)
    assert dims == (20, 20, 5) and subs == [0, 1]
    inp, tgt = features(mdl, subs, dims)
    torch.cuda.synchronize()
    geo = Geometry(pb.dims, case.partition, case.iface)
    s0 = 0
    for l in subs:
        ls = local_system(pb, geo, l, case.alpha)
        X = local_solve(ls)
        si = mdl.subdomain(l)
        fi, ft = onn.features_and_targets(pb, ls, tuple(si.lo), tuple(si.ext), X)
        m = fi.shape[0]
        assert _rel(inp[s0:s0 + m].cpu().numpy(), fi) < 1e-6
        assert _rel(tgt[s0:s0 + m].cpu().numpy(), ft) < 1e-6
        s0 += m
    assert s0 == inp.shape[0]
    # scatter: sample s of subdomain l, column c lands at row r, column c
    from paper_2103_08513_amd import _lib as L
    from ctypes import c_int32
    out = torch.arange(inp.shape[0] * 2000, dtype=torch.float32, device="cuda").reshape(-1, 2000)
    x0 = torch.zeros(mdl.mbf_layout()[-1], dtype=torch.float64, device="cuda")
    arr = (c_int32 * 2)(*subs)
    assert L.load().mrcm_nn_scatter(mdl._mbfs, arr, 2, _p(out), _p(x0), _s()) == 0
    offs = mdl.mbf_layout()
    x0h = x0.cpu().numpy()
    s0 = 0
    for l in subs:
        si = mdl.subdomain(l)
        blk = x0h[offs[l]:offs[l + 1]].reshape(si.n_cells, si.n_rhs)
        for c in (0, si.n_rhs - 1):
            assert np.array_equal(blk[:, c], (s0 + c) * 2000 + np.arange(2000, dtype=np.float64))
        s0 += si.n_rhs
    mdl.close()


def test_training_lowers_loss_and_the_scaled_guess_has_less_energy_error_than_zero():
    import paper_2103_08513_amd as lib
    from paper_2103_08513_amd.surrogate import WarmStartNet, features, net_subdomains, warm_start
    net = WarmStartNet(seed=0)
    inps, tgts = [], []
    for seed in (0, 1, 2):
        mdl = _fp64_model(config1(seed=seed))
        subs, dims = net_subdomains(mdl)
        i, t = features(mdl, subs, dims)
        inps.append(i)
        tgts.append(t)
        mdl.close()
    inp, tgt = torch.cat(inps), torch.cat(tgts)
    hist = net.train(inp, tgt, dims, epochs=8, batch=64, lr=3e-3, seed=0)
    print(f"training loss by epoch: {[round(h, 4) for h in hist]}", flush=True)
    assert hist[-1] < 0.7 * hist[0]
    case = config1(seed=1000)
    pb = case.problem
    args = (_dev(pb.kx), _dev(pb.ky), _dev(pb.kz), _dev(pb.q))
    m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=lib.PCG, pcg_max_iter=2000)
    m.build_mbfs(*args)
    cold = m.info().pcg_iters
    subs, dims = net_subdomains(m)
    x0 = warm_start(m, net, subs, dims)
    # energy-norm error of the Galerkin-scaled network guess on sampled
    # subdomains, against the oracle's exact local solutions (a zero start
    # has error 1)
    geo = Geometry(pb.dims, case.partition, case.iface)
    offs = m.mbf_layout()
    x0h = x0.cpu().numpy()
    errs = []
    for l in (0, 21, 42, 63):
        ls = local_system(pb, geo, l, case.alpha)
        X = local_solve(ls)
        si = m.subdomain(l)
        v = x0h[offs[l]:offs[l + 1]].reshape(si.n_cells, si.n_rhs)[np.argsort(m.local_order(l))]
        for c in range(X.shape[1]):
            x, b = X[:, c], ls.R[:, c]
            xAx = x @ (ls.M @ x)
            if xAx == 0.0:
                continue
            vAv = v[:, c] @ (ls.M @ v[:, c])
            cs = (v[:, c] @ b) / vAv if vAv > 0 else 0.0
            e = x - cs * v[:, c]
            errs.append(np.sqrt((e @ (ls.M @ e)) / xAx))
    m.build_mbfs(*args, x0=x0, x0_scale=True)
    torch.cuda.synchronize()
    warm = m.info().pcg_iters
    assert m.info().pcg_fallback == 0
    print(f"unseen field: energy-norm error of the scaled guess {np.mean(errs):.3f} (mean over "
          f"{len(errs)} columns; 1 for a zero start); CG iterations to 1e-10: {cold} from zero, {warm} "
          f"from the network ({100.0 * (cold - warm) / cold:+.1f}% fewer)", flush=True)
    assert np.mean(errs) < 1.0
    m.close()
