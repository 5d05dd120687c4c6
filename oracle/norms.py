"""Error norms of Sec. 3.1 (oracle).

Pressure: the L2 norm over the domain, sum_c V p_c^2.
Velocity: the K^-1-weighted L2 norm, evaluated with the trapezoidal rule of
the lowest-order Raviart-Thomas space on each cell:
    ||u||^2 = sum_c sum_d (V / 2) (u_{c,d-}^2 + u_{c,d+}^2) / K_d(c)
using each cell's own outward face velocities (their signs do not matter).
"""
from __future__ import annotations

import numpy as np


def rel_l2_pressure(p, p_ref, V=1.0):
    return float(np.sqrt(np.sum(V * (p - p_ref) ** 2) / np.sum(V * p_ref ** 2)))


def kinv_norm2(U, pb):
    V = pb.hx * pb.hy * pb.hz
    Ks = (pb.kx, pb.ky, pb.kz)
    s = 0.0
    for d in range(3):
        s += np.sum(0.5 * V * (U[2 * d] ** 2 + U[2 * d + 1] ** 2) / Ks[d])
    return s


def rel_kinv_velocity(U, U_ref, pb):
    return float(np.sqrt(kinv_norm2(U - U_ref, pb) / kinv_norm2(U_ref, pb)))


def rel_l2(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
