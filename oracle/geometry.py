"""Domain decomposition, skeleton and interface space (oracle).

Follows Sec. 2.2 (non-overlapping subdomains, skeleton Gamma, normal
n = n^{min(l,l')}) and the construction of V_H by condensing fine faces into
constant patches (Sec. 2.2.2, the paragraph defining H-bar and eq. (2.24)).

Readings adopted where the paper is silent:
* Subdomains are numbered lexicographically, l = sx + ndx*(sy + ndy*sz).  For
  neighbours along axis d the lower-coordinate one has the smaller id, so
  n = +e_d and sigma = n . n^l is +1 on the lower side, -1 on the upper.
* Interfaces are listed x-normal, then y-normal, then z-normal, each in
  increasing order of the lower subdomain id; patches of one interface are
  consecutive, numbered pa + na*pb over the two tangential axes (a < b).
* n cells split into k patches: the first n mod k patches get ceil(n/k) cells,
  the rest floor(n/k).
"""
from __future__ import annotations

import numpy as np

AXES = (0, 1, 2)


def split_sizes(n, k):
    """Balanced split of n cells into k consecutive groups, larger groups first."""
    base, extra = divmod(n, k)
    return [base + (1 if t < extra else 0) for t in range(k)]


def split_index(n, k):
    """Group index of each of the n cells under split_sizes(n, k)."""
    out = []
    for g, s in enumerate(split_sizes(n, k)):
        out += [g] * s
    return np.asarray(out, dtype=np.int64)


class Geometry:
    """Subdomain boxes, interfaces and patch maps for one partition.

    Attributes
    ----------
    sub_lo, sub_hi : [n_sub, 3] box corners (hi exclusive)
    ifaces : list of dicts with keys d, lo_sub, hi_sub, a, b, la, lb, na, nb, p0
    n_patch : number of patches N_V (the interface system has 2 N_V unknowns)
    sub_patches : per subdomain, sorted global ids of the patches on its
                  boundary (the index set I^l)
    sub_face_iface : [n_sub, 6] interface index on faces -x,+x,-y,+y,-z,+z, or -1
    """

    def __init__(self, dims, partition, iface_space):
        self.dims = tuple(int(x) for x in dims)
        self.cuts = [np.asarray(c, dtype=np.int64) for c in partition.cuts]
        for n, c in zip(self.dims, self.cuts):
            assert c[0] == 0 and c[-1] == n and np.all(np.diff(c) > 0)
        self.nd = tuple(len(c) - 1 for c in self.cuts)
        ndx, ndy, ndz = self.nd
        self.n_sub = ndx * ndy * ndz
        self.sub_lo = np.zeros((self.n_sub, 3), dtype=np.int64)
        self.sub_hi = np.zeros((self.n_sub, 3), dtype=np.int64)
        self.sub_s = np.zeros((self.n_sub, 3), dtype=np.int64)
        for sz in range(ndz):
            for sy in range(ndy):
                for sx in range(ndx):
                    l = self.sub_id((sx, sy, sz))
                    s = (sx, sy, sz)
                    self.sub_s[l] = s
                    for d in AXES:
                        self.sub_lo[l, d] = self.cuts[d][s[d]]
                        self.sub_hi[l, d] = self.cuts[d][s[d] + 1]
        self.sub_face_iface = -np.ones((self.n_sub, 6), dtype=np.int64)
        self.ifaces = []
        override = None if iface_space.split is None else np.asarray(iface_space.split)
        p0 = 0
        for d in AXES:
            a, b = [x for x in AXES if x != d]
            for l in range(self.n_sub):
                s = self.sub_s[l]
                if s[d] + 1 >= self.nd[d]:
                    continue
                s2 = s.copy()
                s2[d] += 1
                l2 = self.sub_id(s2)
                la = int(self.sub_hi[l, a] - self.sub_lo[l, a])
                lb = int(self.sub_hi[l, b] - self.sub_lo[l, b])
                t = len(self.ifaces)
                if override is not None:
                    na, nb = (int(x) for x in override[t])
                else:
                    na, nb = (int(x) for x in iface_space.uniform_split[d])
                if na == 0 and nb == 0:
                    na, nb = la, lb
                assert 1 <= na <= la and 1 <= nb <= lb, "patch split must fit the face"
                self.ifaces.append(dict(d=d, lo_sub=l, hi_sub=l2, a=a, b=b, la=la, lb=lb,
                                        na=na, nb=nb, p0=p0))
                self.sub_face_iface[l, 2 * d + 1] = t
                self.sub_face_iface[l2, 2 * d] = t
                p0 += na * nb
        self.n_patch = p0
        self.sub_patches = []
        for l in range(self.n_sub):
            ps = []
            for f in range(6):
                t = self.sub_face_iface[l, f]
                if t >= 0:
                    I = self.ifaces[t]
                    ps += list(range(I["p0"], I["p0"] + I["na"] * I["nb"]))
            self.sub_patches.append(np.asarray(sorted(ps), dtype=np.int64))

    def sub_id(self, s):
        ndx, ndy, _ = self.nd
        return int(s[0] + ndx * (s[1] + ndy * s[2]))

    def sub_cells(self, l):
        """Global flat indices of the cells of subdomain l, x fastest within the box."""
        nx, ny, _ = self.dims
        lo, hi = self.sub_lo[l], self.sub_hi[l]
        i = np.arange(lo[0], hi[0])
        j = np.arange(lo[1], hi[1])
        k = np.arange(lo[2], hi[2])
        return (i[None, None, :] + nx * (j[None, :, None] + ny * k[:, None, None])).reshape(-1)

    def iface_faces(self, t):
        """Fine faces of interface t: (lower-side cell, upper-side cell, patch id),
        each an array over the la*lb faces."""
        I = self.ifaces[t]
        nx, ny, _ = self.dims
        d, a, b = I["d"], I["a"], I["b"]
        lo = self.sub_lo[I["lo_sub"]]
        hi = self.sub_hi[I["lo_sub"]]
        ia = split_index(I["la"], I["na"])
        ib = split_index(I["lb"], I["nb"])
        lower, upper, patch = [], [], []
        for tb in range(I["lb"]):
            for ta in range(I["la"]):
                x = [0, 0, 0]
                x[a] = lo[a] + ta
                x[b] = lo[b] + tb
                x[d] = hi[d] - 1
                c_lo = x[0] + nx * (x[1] + ny * x[2])
                x[d] = hi[d]
                c_hi = x[0] + nx * (x[1] + ny * x[2])
                lower.append(c_lo)
                upper.append(c_hi)
                patch.append(I["p0"] + ia[ta] + I["na"] * ib[tb])
        return np.asarray(lower), np.asarray(upper), np.asarray(patch)


def count_interface_unknowns(n_sub_axes, patches_per_iface_axes=((1, 1), (1, 1), (1, 1))):
    """N_Gamma = 2 * (number of patches) for a tensor-product decomposition with
    nd = (nd1, nd2, nd3) subdomains per axis and a uniform patch count per
    interface orientation; eq. (2.24) with H/H-bar patches per tangential axis.
    Pure integer arithmetic, so it runs for billion-cell decompositions."""
    nd = n_sub_axes
    total = 0
    for d in AXES:
        n_if = 1
        for e in AXES:
            n_if *= (nd[e] - 1) if e == d else nd[e]
        na, nb = patches_per_iface_axes[d]
        total += n_if * na * nb
    return 2 * total
