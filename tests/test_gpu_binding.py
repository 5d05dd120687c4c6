"""The Python binding refuses tensors of the wrong size before any library
call: the library reads and writes exactly the sizes the configuration
implies, so a short tensor would be an out-of-bounds device access."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import small_case  # noqa: E402


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def test_short_tensors_are_refused():
    import paper_2103_08513_amd as lib
    case = small_case((8, 6, 4), (2, 2, 2), seed=1)
    pb = case.problem
    m = lib.MRCM(pb, case.partition, case.iface)
    args = [_dev(a) for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    for i in range(4):
        bad = list(args)
        bad[i] = bad[i][:-1].contiguous()
        with pytest.raises(ValueError):
            m.build_mbfs(*bad)
    # nothing has been built: the later steps refuse to run
    with pytest.raises(ValueError):
        m.reconstruct(torch.zeros(4, dtype=torch.float64, device="cuda"))
    m.build_mbfs(*args)
    m.assemble_interface()
    n = 2 * m.info().n_patch
    with pytest.raises(ValueError):
        m.solve_interface(torch.empty(n - 1, dtype=torch.float64, device="cuda"))
    X = m.solve_interface()
    N = pb.n
    with pytest.raises(ValueError):
        m.reconstruct(X[:-1].contiguous())
    with pytest.raises(ValueError):
        m.reconstruct(X, p=torch.empty(N - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        m.reconstruct(X, U=torch.empty(6 * N - 6, dtype=torch.float64, device="cuda"))
    p, U = m.reconstruct(X)
    torch.cuda.synchronize()
    assert torch.isfinite(p).all() and torch.isfinite(U).all()
    m.close()
