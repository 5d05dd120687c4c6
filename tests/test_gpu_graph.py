"""The recorded MRCM step (mrcm_graph_capture / mrcm_graph_launch): every
replay gives bitwise the result of the eager calls on the same inputs.

Replays alternate with eager work on the same handles and with new fields
copied into the captured input buffers, and every replay is checked, so a
node that only works on the first replay would show.  The 60x220x85 case
runs the FP64 build's two-stream pipeline inside the graph.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config1, config2  # noqa: E402


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("cfg", ["40x40x20", "60x220x85"])
def test_graph_replays_match_eager(cfg):
    import paper_2103_08513_amd as lib
    make = config1 if cfg == "40x40x20" else config2
    cases = [make(seed=0), make(seed=1)]
    pb = cases[0].problem
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = lib.MRCM(pb, cases[0].partition, cases[0].iface, alpha=cases[0].alpha, precision=lib.FP64)
        kx, ky, kz, q = (_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q))
        m.solve(kx, ky, kz, q)  # creates the handles
        nv = m.info().n_patch
        X = torch.empty(2 * nv, dtype=torch.float64, device="cuda")
        p = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        U = torch.empty(6 * pb.n, dtype=torch.float64, device="cuda")
        g = m.capture(kx, ky, kz, q, X, p, U, stream=stream)
        for k, idx in enumerate((0, 1, 0)):
            c = cases[idx].problem
            for buf, a in zip((kx, ky, kz, q), (c.kx, c.ky, c.kz, c.q)):
                buf.copy_(_dev(a))
            g.launch(stream=stream)
            g.check(stream=stream)
            p_g, U_g, X_g = p.clone(), U.clone(), X.clone()
            # eager calls on fresh copies of the same field
            ek = [_dev(a) for a in (c.kx, c.ky, c.kz, c.q)]
            p_e, U_e, X_e = m.solve(*ek)
            stream.synchronize()
            print(f"{cfg} replay {k} (field {idx}): max |p_graph - p_eager| = "
                  f"{float((p_g - p_e).abs().max()):.3g}", flush=True)
            assert torch.equal(p_g, p_e), k
            assert torch.equal(U_g, U_e.reshape(-1)), k
            assert torch.equal(X_g, X_e), k
        g.close()
        m.close()


def test_graph_rejects_the_iterative_forms():
    import paper_2103_08513_amd as lib
    case = config1()
    pb = case.problem
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=lib.PCG)
        kx, ky, kz, q = (_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q))
        m.solve(kx, ky, kz, q)
        nv = m.info().n_patch
        X = torch.empty(2 * nv, dtype=torch.float64, device="cuda")
        p = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        U = torch.empty(6 * pb.n, dtype=torch.float64, device="cuda")
        with pytest.raises(lib.MRCMError) as ei:
            m.capture(kx, ky, kz, q, X, p, U, stream=stream)
        assert ei.value.code == -7
        m.close()
