"""The 60x220x85 channelised workload end to end against the oracle.

3x11x17 = 561 subdomains of 20x20x5 cells (b = 100, up to 33 right-hand
sides), 3,880 patches, for each Robin parameter the workload names
(alpha = 0.01, 1, 100).  Compared: every subdomain's flux blocks F and Fb,
the assembled interface matrix and right-hand side, the interface unknowns,
and the reconstructed pressure and velocities.  The reference is the oracle
with extended-precision refinement of every solve: the plain FP64 algorithm
is itself 1.7e-8 away on the pressure (tests/test_oracle_floor.py).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from mrcm_inputs import config2  # noqa: E402
from oracle.mrcm import mrcm_solve  # noqa: E402
from oracle.norms import rel_l2  # noqa: E402


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _maxrel(a, b):
    scale = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (scale if scale > 0 else 1.0))


def _procs():
    return max(1, min(16, len(os.sched_getaffinity(0))))


_REF = {}


def _oracle(alpha):
    if alpha not in _REF:
        _REF.clear()
        _REF[alpha] = mrcm_solve(config2(alpha=alpha), processes=_procs())
    return _REF[alpha]


def _gpu(case, precision, refine=1):
    import paper_2103_08513_amd as lib
    pb = case.problem
    m = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=precision)
    p, U, X = m.solve(_dev(pb.kx), _dev(pb.ky), _dev(pb.kz), _dev(pb.q), refine=refine)
    torch.cuda.synchronize()
    return m, p.cpu().numpy(), U.cpu().numpy(), X.cpu().numpy()


@pytest.mark.parametrize("alpha", [1.0, 0.01, 100.0])
def test_config2_end_to_end_fp64(alpha):
    case = config2(alpha=alpha)
    print(f"cfg2 alpha {alpha:g}: oracle on {_procs()} processes ...", flush=True)
    ref = _oracle(alpha)
    m, p, U, X = _gpu(case, 0)
    worst_f = worst_fb = 0.0
    for l in range(len(ref.systems)):
        F, Fb, SAb = m.copy_flux(l)
        worst_f = max(worst_f, _maxrel(F, ref.F[l]))
        worst_fb = max(worst_fb, _maxrel(Fb, ref.Fb[l]))
        assert _maxrel(SAb, ref.SAb[l]) < 1e-13
    A, b = m.copy_interface()
    Ao = ref.A_int.toarray()
    e_a = _maxrel(A, Ao)
    e_b = _maxrel(b, ref.b_int)
    del A, Ao
    e_p, e_u, e_pi = rel_l2(p, ref.p), rel_l2(U, ref.U), rel_l2(X, ref.pi)
    print(f"cfg2 alpha {alpha:g} FP64: F {worst_f:.2e}, Fb {worst_fb:.2e}, A_int {e_a:.2e}, b_int {e_b:.2e}, "
          f"pi {e_pi:.2e}, p {e_p:.2e}, U {e_u:.2e}", flush=True)
    assert worst_f < 1e-9 and worst_fb < 1e-9
    assert e_a < 1e-12 and e_b < 1e-12
    assert e_pi < 1e-8 and e_p < 1e-8 and e_u < 1e-8
    m.close()


def test_config2_end_to_end_fp32_refined():
    case = config2()
    ref = _oracle(1.0)
    m, p, U, X = _gpu(case, 1)
    info = m.info()
    e_p, e_u, e_pi = rel_l2(p, ref.p), rel_l2(U, ref.U), rel_l2(X, ref.pi)
    print(f"cfg2 FP32+IR: {info.ir_iters} sweeps, residual {info.ir_residual:.2e}; pi {e_pi:.2e}, "
          f"p {e_p:.2e}, U {e_u:.2e}", flush=True)
    assert e_pi < 1e-8 and e_p < 1e-8 and e_u < 1e-8
    m.close()
