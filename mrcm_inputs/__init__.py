"""Seeded synthetic workloads for the Multiscale Robin Coupled Method (MRCM).

This module produces *data only*: grids, permeability fields, source terms,
subdomain partitions and interface-space splits.  It holds none of the
method's arithmetic (no transmissibilities, no Robin terms, no solves), so the
CPU oracle and the HIP library can both consume what it generates without
sharing any computation.

Conventions (the paper's problem statement, Sec. 2, eqs. (2.3)-(2.6)):

* Cartesian grid ``nx x ny x nz`` with cell sizes ``hx, hy, hz``; a cell
  ``(i, j, k)`` has flat index ``c = i + nx*(j + ny*k)`` (x fastest).
* ``kx, ky, kz``: the diagonal of the (mobility-scaled) permeability tensor,
  one value per cell, float64, positive.
* ``q``: total volumetric source rate per cell (``f * V``); positive injects.
* Walls, in the order -x,+x,-y,+y,-z,+z: type 0 no-flow, 1 Dirichlet
  (pressure ``g_p``), 2 Neumann (outward normal velocity ``g_u``).  A wall's
  values are indexed by the two in-plane cell coordinates, the lower axis
  fastest (-x/+x: ``j + ny*k``; -y/+y: ``i + nx*k``; -z/+z: ``i + nx*j``).
* ``pin``: flat index of a cell whose pressure is fixed to zero, or -1.
* Partition: strictly increasing cut arrays per axis, from 0 to n.
* Interface space: per normal axis, the number of constant patches along
  each of the two tangential axes (ascending axis order); ``(0, 0)`` asks for
  one patch per fine face (the fine trace).  An optional per-interface
  override has one ``(na, nb)`` pair per interface, interfaces listed
  x-normal first, then y-normal, then z-normal, each in increasing order of
  the lower subdomain's lexicographic id.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem", "Partition", "IfaceSpace", "Case",
    "grf", "channelised", "uniform_cuts", "ragged_cuts",
    "config1", "config2", "config3", "config3_block", "config4_field", "config5", "config5_block", "contrast_power",
    "small_case",
]


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray
    q: np.ndarray
    wall_type: List[int] = field(default_factory=lambda: [0] * 6)
    wall_value: List[Optional[np.ndarray]] = field(default_factory=lambda: [None] * 6)
    pin: int = -1

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)

    @property
    def h(self):
        return (self.hx, self.hy, self.hz)


@dataclass
class Partition:
    cut_x: np.ndarray
    cut_y: np.ndarray
    cut_z: np.ndarray

    @property
    def cuts(self):
        return (self.cut_x, self.cut_y, self.cut_z)

    @property
    def nd(self):
        return (len(self.cut_x) - 1, len(self.cut_y) - 1, len(self.cut_z) - 1)


@dataclass
class IfaceSpace:
    # uniform_split[d] = (na, nb) for interfaces normal to axis d.
    uniform_split: Sequence[Sequence[int]] = ((1, 1), (1, 1), (1, 1))
    split: Optional[np.ndarray] = None  # [n_interfaces, 2] int32 override


@dataclass
class Case:
    name: str
    problem: Problem
    partition: Partition
    iface: IfaceSpace
    alpha: float = 1.0
    # Robin parameter on Gamma: 0 per side (own subdomain extent and own cell's
    # permeability), 1 one value per face shared by both sides
    beta_mode: int = 0


# ----------------------------------------------------------------------------
# Random fields
# ----------------------------------------------------------------------------

def grf(shape, std, corr_len, seed, mean=0.0):
    """Gaussian random field with exponential covariance, by circulant embedding.

    ``shape = (nx, ny, nz)``; ``corr_len`` is a scalar or per-axis correlation
    length in cells; covariance ``C(r) = std^2 exp(-r)`` with
    ``r = |(dx/lx, dy/ly, dz/lz)|``.  The field is periodic on a torus of at
    least twice the grid in every axis and cropped.  Returns a flat float64
    array in x-fastest order.
    """
    rng = np.random.default_rng(seed)
    cl = np.broadcast_to(np.asarray(corr_len, dtype=np.float64), (3,))
    ext = [int(2 ** np.ceil(np.log2(2 * s))) if s > 1 else 1 for s in shape]
    ax = []
    for e, c in zip(ext, cl):
        d = np.arange(e, dtype=np.float64)
        d = np.minimum(d, e - d)
        ax.append(d / c)
    r = np.sqrt(ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[2][None, None, :] ** 2)
    cov = std ** 2 * np.exp(-r)
    lam = np.real(np.fft.fftn(cov))
    lam = np.maximum(lam, 0.0)
    w = rng.standard_normal(ext)
    y = np.real(np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(w)))
    y = y[: shape[0], : shape[1], : shape[2]] + mean
    return np.ascontiguousarray(y.transpose(2, 1, 0)).reshape(-1)  # [z][y][x] -> x fastest


def channelised(shape, seed, frac=0.3, mean_ch=7.0, mean_bg=0.0, std=1.0):
    """Two-facies channelised log-permeability (channels run along y).

    Each channel has a sinusoidal centre line ``x(y) = x0 + A sin(2 pi y / L + phi)``,
    a width of 6-12 cells and a vertical band of 2-6 cells.  Channels are added
    until the channel fraction reaches ``frac``.  Log-permeability is i.i.d.
    normal per cell, mean ``mean_ch`` in channels and ``mean_bg`` outside.
    """
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    facies = np.zeros((nz, ny, nx), dtype=bool)
    yy = np.arange(ny)
    xx = np.arange(nx)
    guard = 0
    total = nx * ny * nz
    count = 0  # channel cells so far (kept incrementally instead of re-counting the grid)
    while count / total < frac and guard < 10000:
        guard += 1
        x0 = rng.uniform(0, nx)
        amp = rng.uniform(2, 12)
        lam = rng.uniform(0.3, 1.0) * ny
        phi = rng.uniform(0, 2 * np.pi)
        width = rng.integers(6, 13)
        thick = rng.integers(2, 7)
        z0 = rng.integers(0, max(1, nz - thick + 1))
        xc = x0 + amp * np.sin(2 * np.pi * yy / lam + phi)
        band = np.abs(xx[None, :] - xc[:, None]) <= width / 2.0  # [ny, nx]
        slab = facies[z0:z0 + thick]
        count += int(np.count_nonzero(~slab[:, band]))
        slab[:, band] = True
    noise = rng.standard_normal((nz, ny, nx))
    y = np.where(facies, mean_ch, mean_bg) + std * noise
    return y.reshape(-1)


# ----------------------------------------------------------------------------
# Partitions
# ----------------------------------------------------------------------------

def uniform_cuts(n, size):
    assert n % size == 0
    return np.arange(0, n + 1, size, dtype=np.int32)


def ragged_cuts(n, parts):
    """Cuts from an explicit list of part sizes (must sum to n)."""
    parts = np.asarray(parts, dtype=np.int64)
    assert parts.sum() == n and (parts > 0).all()
    return np.concatenate([[0], np.cumsum(parts)]).astype(np.int32)


def _cell(i, j, k, nx, ny):
    return i + nx * (j + ny * k)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def config1(seed=0):
    """40x40x20 unit cells, 4x4x4 subdomains of 10x10x5, Gaussian log-k (std 2,
    exponential covariance, correlation length 4 cells), kz = 0.1 kx, unit
    injector at (0,0,0), unit producer at (39,39,19) which is also the pinned
    cell, one patch per interface, alpha = 1."""
    nx, ny, nz = 40, 40, 20
    y = grf((nx, ny, nz), 2.0, 4.0, seed)
    kx = np.exp(y)
    q = np.zeros(nx * ny * nz)
    q[_cell(0, 0, 0, nx, ny)] = 1.0
    prod = _cell(39, 39, 19, nx, ny)
    q[prod] = -1.0
    pb = Problem(nx, ny, nz, 1.0, 1.0, 1.0, kx, kx.copy(), 0.1 * kx, q, pin=prod)
    part = Partition(uniform_cuts(nx, 10), uniform_cuts(ny, 10), uniform_cuts(nz, 5))
    return Case("cfg1-40x40x20", pb, part, IfaceSpace(((1, 1), (1, 1), (1, 1))), 1.0)


def config2(seed=0, alpha=1.0):
    """60x220x85 cells of 20x10x2 ft, 3x11x17 subdomains of 20x20x5,
    channelised two-facies field (lognormal, mean 7 / 0, std 1), kz = 0.1 kx,
    quarter-five-spot well columns at (0,0,.) and (59,219,.), patches 2x1 on
    x/y-normal faces and 2x2 on z-normal faces."""
    nx, ny, nz = 60, 220, 85
    y = channelised((nx, ny, nz), seed)
    kx = np.exp(y)
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(0, 0, k, nx, ny)] += 1.0 / nz
        q[_cell(nx - 1, ny - 1, k, nx, ny)] -= 1.0 / nz
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, 20.0, 10.0, 2.0, kx, kx.copy(), 0.1 * kx, q, pin=pin)
    part = Partition(uniform_cuts(nx, 20), uniform_cuts(ny, 20), uniform_cuts(nz, 5))
    return Case(f"cfg2-60x220x85-a{alpha:g}", pb, part, IfaceSpace(((2, 1), (2, 1), (2, 2))), alpha)


def contrast_power(k, contrast=1e8):
    """K -> K^theta with theta = ln(contrast) / ln(K_max / K_min) of the given
    field, so that the result spans exactly `contrast` (the paper raises its
    permeability to a power to vary the contrast)."""
    lk = np.log(k)
    theta = np.log(contrast) / (lk.max() - lk.min())
    return np.exp(theta * lk), float(theta)


def config5(seed=0, alpha=1.0):
    """600x2200x85 cells of 20x10x2 ft (112.2M), 30x110x17 = 56,100 subdomains
    of 20x20x5, the channelised field of the 60x220x85 workload raised to the
    power that makes its contrast 1e8, kz = 0.1 kx, patches 2x1 on x/y-normal
    and 2x2 on z-normal faces (430,840 patches), quarter-five-spot well columns
    at (0,0,.) and (599,2199,.), pin at (599,2199,84)."""
    nx, ny, nz = 600, 2200, 85
    kx, theta = contrast_power(np.exp(channelised((nx, ny, nz), seed)), 1e8)
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(0, 0, k, nx, ny)] += 1.0 / nz
        q[_cell(nx - 1, ny - 1, k, nx, ny)] -= 1.0 / nz
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, 20.0, 10.0, 2.0, kx, kx.copy(), 0.1 * kx, q, pin=pin)
    part = Partition(uniform_cuts(nx, 20), uniform_cuts(ny, 20), uniform_cuts(nz, 5))
    case = Case(f"cfg5-600x2200x85-a{alpha:g}", pb, part, IfaceSpace(((2, 1), (2, 1), (2, 2))), alpha)
    case.theta = theta
    return case


def config5_block(big):
    """The 60x220x85 block at the origin corner of a 600x2200x85 case (its
    permeability exactly), laid out as the 60x220x85 workload: 3x11x17
    subdomains of 20x20x5, the same patches, quarter-five-spot columns at the
    block's corners (0,0,.) and (59,219,.), pin at (59,219,84)."""
    nx, ny, nz = 60, 220, 85
    B = big.problem
    def win(a):
        return np.ascontiguousarray(np.asarray(a).reshape(B.nz, B.ny, B.nx)[:nz, :ny, :nx]).reshape(-1)
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(0, 0, k, nx, ny)] += 1.0 / nz
        q[_cell(nx - 1, ny - 1, k, nx, ny)] -= 1.0 / nz
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, B.hx, B.hy, B.hz, win(B.kx), win(B.ky), win(B.kz), q, pin=pin)
    part = Partition(uniform_cuts(nx, 20), uniform_cuts(ny, 20), uniform_cuts(nz, 5))
    return Case("cfg5-block-60x220x85", pb, part, IfaceSpace(((2, 1), (2, 1), (2, 2))), big.alpha)


def config4_field(seed):
    """A field of the learned warm start's data: the 60x220x85 workload's
    channelised generator on a 60x60x15 grid of 20x10x2 ft cells (3x3x3
    subdomains of 20x20x5, so one interior, face, edge and corner subdomains),
    the same patches, kz = 0.1 kx, quarter-five-spot columns and the pin in
    the far corner."""
    nx, ny, nz = 60, 60, 15
    kx = np.exp(channelised((nx, ny, nz), seed))
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(0, 0, k, nx, ny)] += 1.0 / nz
        q[_cell(nx - 1, ny - 1, k, nx, ny)] -= 1.0 / nz
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, 20.0, 10.0, 2.0, kx, kx.copy(), 0.1 * kx, q, pin=pin)
    part = Partition(uniform_cuts(nx, 20), uniform_cuts(ny, 20), uniform_cuts(nz, 5))
    return Case(f"cfg4-field-{seed}", pb, part, IfaceSpace(((2, 1), (2, 1), (2, 2))), 1.0)


def config3(seed=0, patch_seed=3):
    """~15M-cell ragged batch: 200x440x170 cells of 20x10x2 ft, Gaussian log-k
    (std 3, correlation lengths 20x20x3 cells), kz = 0.1 kx; cuts with 15-cell
    x/y blocks at both ends and 3-cell z blocks, 2, 4 or 8 patches per
    interface drawn with ``default_rng(patch_seed)``; five-spot wells."""
    nx, ny, nz = 200, 440, 170
    y = grf((nx, ny, nz), 3.0, (20.0, 20.0, 3.0), seed)
    kx = np.exp(y)
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(nx // 2, ny // 2, k, nx, ny)] += 1.0 / nz
        for (i, j) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
            q[_cell(i, j, k, nx, ny)] -= 1.0 / (4 * nz)
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, 20.0, 10.0, 2.0, kx, kx.copy(), 0.1 * kx, q, pin=pin)
    part = Partition(ragged_cuts(nx, [15, 15] + [20] * 7 + [15, 15]),
                     ragged_cuts(ny, [15, 15] + [20] * 19 + [15, 15]),
                     ragged_cuts(nz, [3, 3, 3] + [5] * 31 + [3, 3]))
    split = _random_splits(part, np.random.default_rng(patch_seed))
    return Case("cfg3-200x440x170", pb, part, IfaceSpace(((1, 1), (1, 1), (1, 1)), split), 1.0)


def _random_splits(part, rng):
    """2, 4 or 8 patches per interface, split (2x1), (2x2) or (4x2) with the
    larger count along the longer tangential side; interfaces in the order of
    the interface-space override (x-normal, y-normal, z-normal, each in
    increasing lower-subdomain id)."""
    ndx, ndy, ndz = part.nd
    nif = (ndx - 1) * ndy * ndz + ndx * (ndy - 1) * ndz + ndx * ndy * (ndz - 1)
    choice = rng.choice([2, 4, 8], size=nif)
    split = np.zeros((nif, 2), dtype=np.int32)
    t = 0
    ext = [np.diff(c) for c in part.cuts]
    for d in range(3):
        a, b = [x for x in range(3) if x != d]
        counts = list(part.nd)
        counts[d] -= 1
        for sz in range(counts[2]):
            for sy in range(counts[1]):
                for sx in range(counts[0]):
                    sxyz = (sx, sy, sz)
                    la, lb = ext[a][sxyz[a]], ext[b][sxyz[b]]
                    big, small = {2: (2, 1), 4: (2, 2), 8: (4, 2)}[int(choice[t])]
                    split[t] = (big, small) if la >= lb else (small, big)
                    t += 1
    return split


def config3_block(seed=0, patch_seed=3):
    """A 70x70x19 block with the ragged 200x440x170 workload's structure, small
    enough for the whole oracle: cuts 15/20/20/15 along x and y and 3/5/5/3/3
    along z (4x4x5 = 80 subdomains of eight shapes, 15x15x3 to 20x20x5),
    2, 4 or 8 patches per interface drawn with default_rng(patch_seed), the
    same Gaussian log-k (std 3, correlation lengths 20x20x3 cells), cells of
    20x10x2 ft, a five-spot of well columns and the pin in the far corner."""
    nx, ny, nz = 70, 70, 19
    y = grf((nx, ny, nz), 3.0, (20.0, 20.0, 3.0), seed)
    kx = np.exp(y)
    q = np.zeros(nx * ny * nz)
    for k in range(nz):
        q[_cell(nx // 2, ny // 2, k, nx, ny)] += 1.0 / nz
        for (i, j) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
            q[_cell(i, j, k, nx, ny)] -= 1.0 / (4 * nz)
    pin = _cell(nx - 1, ny - 1, nz - 1, nx, ny)
    pb = Problem(nx, ny, nz, 20.0, 10.0, 2.0, kx, kx.copy(), 0.1 * kx, q, pin=pin)
    part = Partition(ragged_cuts(nx, [15, 20, 20, 15]), ragged_cuts(ny, [15, 20, 20, 15]),
                     ragged_cuts(nz, [3, 5, 5, 3, 3]))
    split = _random_splits(part, np.random.default_rng(patch_seed))
    return Case("cfg3-block-70x70x19", pb, part, IfaceSpace(((1, 1), (1, 1), (1, 1)), split), 1.0)


def small_case(dims=(8, 6, 4), nd=(2, 2, 2), split=((1, 1), (1, 1), (1, 1)), seed=0, std=1.0,
               h=(1.0, 1.0, 1.0), alpha=1.0, parts=None, pin="corner", wells=True):
    """Small seeded case for parity and pin tests.  ``parts`` optionally gives
    explicit part sizes per axis (ragged partitions)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    ly = rng.standard_normal(nx * ny * nz) * std
    kx = np.exp(ly)
    ky = np.exp(ly + 0.3 * rng.standard_normal(nx * ny * nz))
    kz = 0.1 * np.exp(ly + 0.3 * rng.standard_normal(nx * ny * nz))
    q = np.zeros(nx * ny * nz)
    if wells:
        q[_cell(0, 0, 0, nx, ny)] = 1.0
        q[_cell(nx - 1, ny - 1, nz - 1, nx, ny)] = -1.0
    p = _cell(nx - 1, ny - 1, nz - 1, nx, ny) if pin == "corner" else int(pin)
    pb = Problem(nx, ny, nz, *h, kx, ky, kz, q, pin=p)
    if parts is None:
        cuts = []
        for n, k in zip(dims, nd):
            base = np.linspace(0, n, k + 1).round().astype(np.int32)
            cuts.append(base)
    else:
        cuts = [ragged_cuts(n, ps) for n, ps in zip(dims, parts)]
    part = Partition(*cuts)
    return Case(f"small-{nx}x{ny}x{nz}", pb, part, IfaceSpace(split), alpha)
