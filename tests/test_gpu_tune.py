"""The autotuner (mrcm_autotune) and the tunables it sets.

On the 60x220x85 workload: the autotuner returns a valid pair, and builds with
every solve_tiles / solve_group setting it may choose give the same MBFs as
the default up to rounding order (1e-12 relative per column) and the same
end-to-end pressure up to the interface system's amplification of rounding
(1e-7 relative L2; each of them is 1.6e-8 from the oracle).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config2  # noqa: E402


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _rel_l2(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_autotune_and_tunables_keep_the_solution():
    import paper_2103_08513_amd as lib
    case = config2()
    pb = case.problem
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    ref = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha)
    p_ref, _, _ = ref.solve(*args)
    X_ref = [ref.copy_mbfs(l) for l in (0, 280, 560)]
    tuned = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha)
    choice = tuned.autotune(*args)
    print(f"autotune: {choice}", flush=True)
    assert 0 <= choice["solve_tiles"] <= 3 and choice["solve_group"] >= -1
    assert choice["build_ms"] <= choice["build_ms_default"]
    for tiles, group in ((choice["solve_tiles"], choice["solve_group"]), (1, 0), (2, -1), (0, 344)):
        m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, solve_tiles=tiles, solve_group=group)
        p, _, _ = m.solve(*args)
        torch.cuda.synchronize()
        for l, Xr in zip((0, 280, 560), X_ref):
            Xg = m.copy_mbfs(l)
            err = np.max(np.abs(Xg - Xr), axis=0) / np.maximum(np.max(np.abs(Xr), axis=0), 1e-300)
            assert err.max() < 1e-12, (tiles, group, l, float(err.max()))
        e = _rel_l2(p, p_ref)
        print(f"solve_tiles {tiles}, solve_group {group}: pressure differs from the default by {e:.2g}", flush=True)
        assert e < 1e-7
        m.close()
    tuned.close()
    ref.close()


def test_autotune_cache_keys_on_shapes(tmp_path):
    """The per-shape cache: a second call on the same shapes is a hit with the
    same values, whatever the coefficients (alpha, the field); another
    partition is a miss that adds its own line."""
    import paper_2103_08513_amd as lib
    from mrcm_inputs import config1, small_case
    cache = str(tmp_path / "tune.txt")
    c = config1()
    pb = c.problem
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    m = lib.MRCM(pb, c.partition, c.iface, alpha=c.alpha)
    a = m.autotune(*args, cache=cache)
    c2 = config1(seed=1)
    m2 = lib.MRCM(c2.problem, c2.partition, c2.iface, alpha=2.0)
    b = m2.autotune(*[_dev(x) for x in (c2.problem.kx, c2.problem.ky, c2.problem.kz, c2.problem.q)], cache=cache)
    assert not a["from_cache"] and b["from_cache"]
    assert (a["solve_tiles"], a["solve_group"], a["iface_panel"]) == (b["solve_tiles"], b["solve_group"],
                                                                       b["iface_panel"])
    s = small_case((20, 10, 8), (2, 1, 1), split=((2, 2), (1, 1), (1, 1)), seed=3)
    m3 = lib.MRCM(s.problem, s.partition, s.iface, alpha=s.alpha)
    c3 = m3.autotune(*[_dev(x) for x in (s.problem.kx, s.problem.ky, s.problem.kz, s.problem.q)], cache=cache)
    assert not c3["from_cache"]
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and all(ln.startswith("mrcm-tune-2 ") for ln in lines)
    for x in (m, m2, m3):
        x.close()


def test_interface_panel_widths_agree():
    """The interface factorisation in panels of 1, 2 and 4 blocks (one
    rank-16 step per block, or one rank-32/64 trailing update per panel)
    gives bitwise the same interface solution: every entry receives the same
    FP64 MFMA accumulations in the same block and k order, whether it passes
    through memory between blocks or stays in the accumulators."""
    import paper_2103_08513_amd as lib
    case = config2()
    pb = case.problem
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    ref = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha)
    p_ref, _, X_ref = ref.solve(*args, refine=1)
    for panel in (1, 2, 4):
        m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, iface_panel=panel)
        p, _, X = m.solve(*args, refine=1)
        torch.cuda.synchronize()
        ex, ep = _rel_l2(X, X_ref), _rel_l2(p, p_ref)
        print(f"iface_panel {panel}: pi differs by {ex:.2g}, p by {ep:.2g}", flush=True)
        assert torch.equal(X, X_ref) and torch.equal(p, p_ref), (ex, ep)
        m.close()
    ref.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_work_queue_launches_give_bitwise_the_grid_result(precision):
    """launch_mode MRCM_LAUNCH_QUEUE (persistent workgroups over per-XCD work
    queues) against the plain grid launches, on the 60x220x85 workload (the
    FP64 form's two-stream pipeline, and the FP32 form) and on a ragged
    small case: every item is computed the same way whichever workgroup takes
    it, so the MBFs and the pressure are bitwise equal."""
    import paper_2103_08513_amd as lib
    from mrcm_inputs import small_case
    for case in (config2(), small_case((37, 23, 11), (3, 2, 2), split=((2, 1), (1, 2), (2, 2)), seed=5)):
        pb = case.problem
        args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
        out = []
        for lm in (lib.LAUNCH_GRID, lib.LAUNCH_QUEUE):
            m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=precision, launch_mode=lm)
            p, U, X = m.solve(*args, refine=1)
            torch.cuda.synchronize()
            n_sub = m.info().n_sub
            out.append((p.clone(), U.clone(), [m.copy_mbfs(l) for l in range(0, n_sub, max(1, n_sub // 7))]))
            m.close()
        (p0, U0, X0), (p1, U1, X1) = out
        assert torch.equal(p0, p1) and torch.equal(U0, U1)
        assert all(np.array_equal(a, b) for a, b in zip(X0, X1))
