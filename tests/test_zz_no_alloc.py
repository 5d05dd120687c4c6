"""mrcm_mse_noalloc, the entry point that allocates nothing, against mrcm_mse
(the same kernels with a caller's workspace): two calls in a row, the second
on a smaller input, each compared bitwise in the loss and the gradient."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_mse_noalloc_matches_the_workspace_form():
    from paper_2103_08513_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(0)
    # the first size needs the whole 1024-entry array of partial sums, the
    # second only part of it (whose other entries keep the first call's values)
    for n in (3_000_000, 777):
        y = torch.as_tensor(rng.standard_normal(n).astype(np.float32), device=dev)
        t = torch.as_tensor(rng.standard_normal(n).astype(np.float32), device=dev)
        dy0, dy1 = torch.empty_like(y), torch.full_like(y, np.nan)
        loss0 = torch.zeros(1, dtype=torch.float64, device=dev)
        loss1 = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
        work = torch.zeros(1024, dtype=torch.float64, device=dev)
        assert lib.mrcm_mse(_p(y), _p(t), _p(dy0), _p(loss0), _p(work), n, s) == 0
        assert lib.mrcm_mse_noalloc(_p(y), _p(t), _p(dy1), _p(loss1), n, s) == 0
        torch.cuda.synchronize()
        assert torch.equal(dy0, dy1)
        assert torch.equal(loss0, loss1)
        ref = float(np.mean((y.cpu().numpy().astype(np.float64) - t.cpu().numpy()) ** 2))
        assert abs(loss1.item() - ref) <= 1e-6 * ref
    # argument errors are caught before any launch
    assert lib.mrcm_mse_noalloc(_p(y), _p(t), _p(dy1), _p(loss1), 0, s) == -1
    assert lib.mrcm_mse_noalloc(_p(y), _p(t), _p(dy1), _p(loss1), (1 << 40) + 1, s) == -1
    assert lib.mrcm_mse_noalloc(None, _p(t), _p(dy1), _p(loss1), 5, s) == -1
