"""MI355X (gfx950) implementation of the Multiscale Robin Coupled Method.

Python binding of the C ABI in ``include/mrcm.h``: it marshals torch device
tensors (FP64, contiguous) and the current HIP stream into the library calls
``mrcm_build_mbfs``, ``mrcm_assemble_interface``, ``mrcm_solve_interface``,
``mrcm_reconstruct`` and ``mrcm_postprocess_mean``, and the two-phase saturation
step ``mrcm_transport_dt``, ``mrcm_transport_step``, ``mrcm_transport_advance``,
``mrcm_mobility_scale``, and the IMPES loop ``mrcm_impes_run``.  Every step of the method runs in the library's
kernels; importing this package does not need a GPU, but every call does.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import byref, c_double, c_int32, c_void_p

import numpy as np

from . import _lib
from ._lib import (CIfaceInfo, CImpesOptions, CImpesStats, CInfo, CIfaceSpace, COptions, CPartition, CProblem,
                   CSubInfo, CTwoPhase, MRCMError)

FP64 = 0
FP32_IR = 1
PCG = 2

# Robin parameter on Gamma and what a handle keeps (mrcm_options)
BETA_PER_SIDE = 0
BETA_FACE = 1
KEEP_FACTORS = 1
KEEP_MBFS = 2

# interface solvers (mrcm_solve_interface)
LAUNCH_GRID = 0
LAUNCH_QUEUE = 1
IFACE_AUTO = 0
IFACE_BAND = 1
IFACE_MULTIFRONTAL = 2

__all__ = ["MRCM", "MRCMError", "FP64", "FP32_IR", "PCG", "IFACE_AUTO", "IFACE_BAND", "IFACE_MULTIFRONTAL",
           "BETA_PER_SIDE", "BETA_FACE", "KEEP_FACTORS", "KEEP_MBFS",
           "build_mbfs", "assemble_interface",
           "solve_interface", "reconstruct", "postprocess_mean", "TwoPhase", "transport_dt", "transport_step", "transport_advance",
           "mobility_scale", "library"]


def library():
    return _lib.load()


def _dev_ptr(t, name, numel=None, device=None):
    """Device address of a contiguous float64 tensor, after checking its
    device and, when given, its number of entries: the library reads and
    writes exactly that many, so a shorter tensor must never reach it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the HIP device")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor on the HIP device")
    if device is not None:
        want = device.index if device.index is not None else torch.cuda.current_device()
        if t.device.index != want:
            raise ValueError(f"{name} is on cuda:{t.device.index}; the model runs on cuda:{want}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries; {numel} are required")
    return c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


class Graph:
    """A recorded MRCM step (mrcm_graph_capture): launch() replays it on a
    stream, check() synchronises and raises on a status the kernels set."""

    def __init__(self, model, handle, keep):
        self.model = model
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None):
        _lib.check(self.model.lib.mrcm_graph_launch(self.handle, _stream_ptr(stream)), "mrcm_graph_launch")

    def check(self, stream=None):
        _lib.check(self.model.lib.mrcm_graph_check(self.handle, _stream_ptr(stream)), "mrcm_graph_check")

    def close(self):
        if self.handle:
            self.model.lib.mrcm_graph_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MRCM:
    """One MRCM configuration (grid, walls, pin, partition, interface space,
    Robin parameter, precision) and its device handles.

    ``problem`` / ``partition`` / ``iface`` are the data classes of
    ``mrcm_inputs`` (or any objects with the same attributes)."""

    def __init__(self, problem, partition, iface, alpha=1.0, precision=FP64, ir_tol=1e-13,
                 ir_max_iter=30, fp64_refine=1, pcg_max_iter=50, solve_tiles=0, solve_group=0, device="cuda",
                 beta_mode=BETA_PER_SIDE, keep=KEEP_FACTORS | KEEP_MBFS, iface_panel=0, launch_mode=0):
        import torch
        self.lib = library()
        self.device = torch.device(device)
        self.pb = problem
        self.nv = None
        self._mbfs = c_void_p()
        self._iface = c_void_p()
        self._graphs = []
        self._keep = []
        nx, ny, nz = problem.nx, problem.ny, problem.nz
        cp = CProblem()
        cp.nx, cp.ny, cp.nz = nx, ny, nz
        cp.hx, cp.hy, cp.hz = problem.hx, problem.hy, problem.hz
        for f in range(6):
            cp.wall_type[f] = int(problem.wall_type[f])
            cp.wall_value[f] = None
        cp.pin_cell = int(problem.pin)
        self._cp = cp
        self._wall_tensors = [None] * 6
        for f in range(6):
            v = problem.wall_value[f]
            if v is not None:
                d = f // 2
                n_wall = (nx * ny * nz) // (nx, ny, nz)[d]
                v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
                if v.size != n_wall:
                    raise ValueError(f"wall {f} has {v.size} values; its face has {n_wall} cells")
                t = torch.as_tensor(v, device=self.device)
                self._wall_tensors[f] = t
                cp.wall_value[f] = t.data_ptr()
        cuts = [np.ascontiguousarray(c, dtype=np.int32) for c in partition.cuts]
        self._keep += cuts
        part = CPartition()
        part.ndx, part.ndy, part.ndz = (len(c) - 1 for c in cuts)
        part.cut_x, part.cut_y, part.cut_z = (c.ctypes.data_as(ctypes.POINTER(c_int32)) for c in cuts)
        self._part = part
        ifs = CIfaceSpace()
        for d in range(3):
            ifs.uniform_split[d][0] = int(iface.uniform_split[d][0])
            ifs.uniform_split[d][1] = int(iface.uniform_split[d][1])
        if iface.split is not None:
            sp = np.ascontiguousarray(iface.split, dtype=np.int32).reshape(-1)
            self._keep.append(sp)
            ifs.split = sp.ctypes.data_as(ctypes.POINTER(c_int32))
        else:
            ifs.split = None
        self._ifs = ifs
        opt = COptions()
        opt.alpha = float(alpha)
        opt.precision = int(precision)
        opt.ir_tol = float(ir_tol)
        opt.ir_max_iter = int(ir_max_iter)
        opt.fp64_refine = int(fp64_refine)
        opt.pcg_max_iter = int(pcg_max_iter)
        opt.solve_tiles = int(solve_tiles)
        opt.solve_group = int(solve_group)
        opt.beta_mode = int(beta_mode)
        opt.keep = int(keep)
        opt.iface_panel = int(iface_panel)
        opt.launch_mode = int(launch_mode)
        opt.pcg_x0 = None
        self._opt = opt

    @property
    def n_cells(self):
        return self.pb.nx * self.pb.ny * self.pb.nz

    def _set_fields(self, kx, ky, kz, q):
        N = self.n_cells
        cp = self._cp
        cp.kx = _dev_ptr(kx, "kx", N, self.device).value
        cp.ky = _dev_ptr(ky, "ky", N, self.device).value
        cp.kz = _dev_ptr(kz, "kz", N, self.device).value
        cp.q = _dev_ptr(q, "q", N, self.device).value

    def _n_unknowns(self):
        if not self._mbfs.value:
            raise ValueError("build_mbfs has not run on this model")
        return 2 * self.info().n_patch

    # -- the four steps of Algorithm 2 ------------------------------------
    def build_mbfs(self, kx, ky, kz, q, stream=None, x0=None, x0_scale=False):
        """x0 (PCG only): starting guess, a float64 device tensor in the layout
        of the MBFs (all subdomains' local blocks concatenated, see
        ``mbf_layout``), or None.  A warm start needs the handle of an earlier
        build, whose layout fixes the tensor's length.  x0_scale: replace each
        column's guess v by its Galerkin multiple (v, b) / (v, A v) v."""
        cp = self._cp
        if x0 is not None:
            if not self._mbfs.value:
                raise ValueError("a starting guess needs a handle from an earlier build_mbfs")
            total = self.mbf_layout()[-1]
            if x0.numel() != total:
                raise ValueError(f"x0 has {x0.numel()} entries; the MBF layout has {total}")
        self._opt.pcg_x0 = None if x0 is None else _dev_ptr(x0, "x0", device=self.device).value
        self._opt.pcg_x0_scale = 1 if x0_scale else 0
        self._set_fields(kx, ky, kz, q)
        self._inputs = (kx, ky, kz, q)
        code = self.lib.mrcm_build_mbfs(byref(cp), byref(self._part), byref(self._ifs),
                                        byref(self._opt), _stream_ptr(stream), byref(self._mbfs))
        _lib.check(code, "mrcm_build_mbfs")
        return self

    def assemble_interface(self, stream=None):
        code = self.lib.mrcm_assemble_interface(self._mbfs, _stream_ptr(stream), byref(self._iface))
        _lib.check(code, "mrcm_assemble_interface")
        return self

    def solve_interface(self, X=None, refine=0, stream=None, residual=False, method=IFACE_AUTO, rtol=0.0):
        """Interface solve (mrcm_solve_interface): ``method`` one of IFACE_*;
        ``refine`` refinement steps at most (exactly that many when rtol is
        0); ``rtol`` > 0 stops refining once the relative residual is below
        it.  With residual=True the relative residual of the returned X is
        also computed (one more residual and a stream synchronisation) and
        kept in ``interface_residual``; ``interface_iters`` holds the
        refinement steps taken."""
        import torch
        n = self._n_unknowns()
        if not self._iface.value:
            raise ValueError("assemble_interface has not run on this model")
        if X is None:
            X = torch.empty(n, dtype=torch.float64, device=self.device)
        res = c_double(0.0)
        its = c_int32(0)
        code = self.lib.mrcm_solve_interface(self._iface, int(method), float(rtol), int(refine), _stream_ptr(stream),
                                             _dev_ptr(X, "X", n, self.device) if n > 0 else None, byref(its),
                                             byref(res) if residual else None)
        _lib.check(code, "mrcm_solve_interface")
        self.interface_residual = res.value if residual else None
        self.interface_iters = its.value
        return X

    def interface_info(self):
        inf = CIfaceInfo()
        _lib.check(self.lib.mrcm_interface_query(self._iface, byref(inf)), "mrcm_interface_query")
        return inf

    def reconstruct(self, X, p=None, U=None, stream=None):
        import torch
        N = self.n_cells
        n = self._n_unknowns()
        if p is None:
            p = torch.empty(N, dtype=torch.float64, device=self.device)
        if U is None:
            U = torch.empty(6 * N, dtype=torch.float64, device=self.device)
        if n > 0 and X is None:
            raise ValueError("X is required: the model has interface unknowns")
        xp = _dev_ptr(X, "X", n, self.device) if n > 0 else None
        code = self.lib.mrcm_reconstruct(self._mbfs, xp, _stream_ptr(stream), _dev_ptr(p, "p", N, self.device),
                                         _dev_ptr(U, "U", 6 * N, self.device))
        _lib.check(code, "mrcm_reconstruct")
        return p, U.view(6, N)

    def postprocess_mean(self, U, pt=None, Ut=None, stream=None):
        """The Mean post-processing of a velocity U[6][N] (mrcm_postprocess_mean):
        returns (pt[N], Ut[6][N])."""
        import torch
        N = self.n_cells
        if pt is None:
            pt = torch.empty(N, dtype=torch.float64, device=self.device)
        if Ut is None:
            Ut = torch.empty(6 * N, dtype=torch.float64, device=self.device)
        code = self.lib.mrcm_postprocess_mean(self._mbfs, _dev_ptr(U, "U", 6 * N, self.device), _stream_ptr(stream),
                                              _dev_ptr(pt, "pt", N, self.device), _dev_ptr(Ut, "Ut", 6 * N, self.device))
        _lib.check(code, "mrcm_postprocess_mean")
        return pt, Ut.view(6, N)

    def impes_run(self, kx, ky, kz, q, S, mu_w, mu_o, skip, t_end=float("inf"), max_steps=0, cfl=1.0 / 6.0,
                  dt_max=float("inf"), refine=1, stream=None):
        """The IMPES loop (mrcm_impes_run) on this configuration: a Darcy
        solve under K lambda(S) with the Mean post-processing every `skip`
        saturation steps, while t <= t_end and fewer than max_steps (if > 0)
        steps are taken.  S (float64 device tensor, N) holds the initial
        saturation and receives the final one.  The run builds and frees its
        own MBF handle.  Returns a dict of the loop's counts, time and device
        milliseconds."""
        N = self.n_cells
        cp = CProblem.from_buffer_copy(self._cp)
        for name, t in (("kx", kx), ("ky", ky), ("kz", kz), ("q", q)):
            setattr(cp, name, _dev_ptr(t, name, N, self.device).value)
        tp = CTwoPhase(self.pb.nx, self.pb.ny, self.pb.nz, self.pb.hx, self.pb.hy, self.pb.hz, float(mu_w),
                       float(mu_o))
        io = CImpesOptions(int(skip), int(max_steps), float(t_end), float(cfl), float(dt_max), int(refine))
        st = CImpesStats()
        code = self.lib.mrcm_impes_run(byref(cp), byref(self._part), byref(self._ifs), byref(self._opt), byref(tp),
                                       byref(io), _stream_ptr(stream), _dev_ptr(S, "S", N, self.device), byref(st))
        _lib.check(code, "mrcm_impes_run")
        return {k: getattr(st, k) for k, _ in CImpesStats._fields_}

    def solve(self, kx, ky, kz, q, refine=0, stream=None, method=IFACE_AUTO):
        """Whole MRCM: MBFs, interface assembly and solve, reconstruction."""
        self.build_mbfs(kx, ky, kz, q, stream)
        self.assemble_interface(stream)
        X = self.solve_interface(refine=refine, stream=stream, method=method)
        return self.reconstruct(X, stream=stream) + (X,)

    def autotune(self, kx, ky, kz, q, stream=None, cache=None):
        """Time the build for candidate solve_tiles / solve_group values and
        the interface solve for candidate iface_panel values on these inputs
        (mrcm_autotune) and keep the fastest for the following builds; with
        ``cache`` (a file path) the per-shape cache of mrcm_autotune_cached is
        consulted first and the result recorded.  Existing handles are
        released (their geometry includes the tunables).  Returns the chosen
        values, the build times and whether they came from the cache."""
        cp = self._cp
        self._set_fields(kx, ky, kz, q)
        self._opt.pcg_x0 = None
        best = COptions()
        t_best, t_rule = c_double(0.0), c_double(0.0)
        hit = c_int32(0)
        if cache is None:
            code = self.lib.mrcm_autotune(byref(cp), byref(self._part), byref(self._ifs), byref(self._opt),
                                          _stream_ptr(stream), byref(best), byref(t_best), byref(t_rule))
        else:
            code = self.lib.mrcm_autotune_cached(byref(cp), byref(self._part), byref(self._ifs), byref(self._opt),
                                                 _stream_ptr(stream), os.fsencode(cache), byref(best), byref(t_best),
                                                 byref(t_rule), byref(hit))
        _lib.check(code, "mrcm_autotune")
        self.close()
        self._opt.solve_tiles = best.solve_tiles
        self._opt.solve_group = best.solve_group
        self._opt.iface_panel = best.iface_panel
        self._opt.launch_mode = best.launch_mode
        return {"solve_tiles": best.solve_tiles, "solve_group": best.solve_group, "iface_panel": best.iface_panel,
                "launch_mode": best.launch_mode,
                "build_ms": t_best.value, "build_ms_default": t_rule.value, "from_cache": bool(hit.value)}

    def capture(self, kx, ky, kz, q, X, p, U, refine=0, stream=None):
        """Record one whole MRCM step (build, assembly, interface solve,
        reconstruction) as a HIP graph (FP64 form, handles already built).
        The graph keeps the addresses of kx, ky, kz, q, X, p and U: a replay
        reads their current contents.  Returns a Graph."""
        cp = self._cp
        self._set_fields(kx, ky, kz, q)
        self._opt.pcg_x0 = None
        self._opt.pcg_x0_scale = 0
        g = c_void_p()
        n = self._n_unknowns()
        N = self.n_cells
        code = self.lib.mrcm_graph_capture(byref(cp), byref(self._part), byref(self._ifs), byref(self._opt),
                                           self._mbfs, self._iface, int(refine),
                                           _dev_ptr(X, "X", n, self.device) if n > 0 else None,
                                           _dev_ptr(p, "p", N, self.device), _dev_ptr(U, "U", 6 * N, self.device),
                                           _stream_ptr(stream), byref(g))
        _lib.check(code, "mrcm_graph_capture")
        graph = Graph(self, g, (kx, ky, kz, q, X, p, U))
        self._graphs.append(graph)
        return graph

    # -- introspection ------------------------------------------------------
    def info(self):
        inf = CInfo()
        _lib.check(self.lib.mrcm_query(self._mbfs, byref(inf)), "mrcm_query")
        return inf

    def mbf_layout(self):
        """Offsets of each subdomain's block (n_cells x n_rhs, row-major) in the
        concatenated MBF layout, with the total length last."""
        offs = [0]
        for l in range(self.info().n_sub):
            si = self.subdomain(l)
            offs.append(offs[-1] + si.n_cells * si.n_rhs)
        return offs

    def subdomain(self, l):
        si = CSubInfo()
        _lib.check(self.lib.mrcm_get_subdomain(self._mbfs, int(l), byref(si)), "mrcm_get_subdomain")
        return si

    def local_order(self, l):
        """Box-local x-fastest index of each library row of subdomain l."""
        si = self.subdomain(l)
        ext = list(si.ext)
        ax = list(si.ax)
        n = [ext[a] for a in ax]
        r = np.arange(si.n_cells)
        t = [r % n[0], (r // n[0]) % n[1], r // (n[0] * n[1])]
        x = [None, None, None]
        for k in range(3):
            x[ax[k]] = t[k]
        return x[0] + ext[0] * (x[1] + ext[1] * x[2])

    def copy_mbfs(self, l):
        si = self.subdomain(l)
        out = np.empty((si.n_cells, si.n_rhs))
        _lib.check(self.lib.mrcm_copy_mbfs(self._mbfs, int(l), out.ctypes.data_as(c_void_p)), "mrcm_copy_mbfs")
        return out

    def copy_flux(self, l):
        si = self.subdomain(l)
        F = np.empty((si.n_patch, si.n_rhs))
        Fb = np.empty((si.n_patch, si.n_rhs))
        SAb = np.empty(si.n_patch)
        _lib.check(self.lib.mrcm_copy_flux(self._mbfs, int(l), F.ctypes.data_as(c_void_p),
                                           Fb.ctypes.data_as(c_void_p), SAb.ctypes.data_as(c_void_p)),
                   "mrcm_copy_flux")
        return F, Fb, SAb

    def copy_factor(self, l):
        si = self.subdomain(l)
        out = np.empty((si.n_cells, si.band + 1))
        _lib.check(self.lib.mrcm_copy_factor(self._mbfs, int(l), out.ctypes.data_as(c_void_p)),
                   "mrcm_copy_factor")
        return out

    def interface_dims(self):
        n = c_int32()
        w = c_int32()
        _lib.check(self.lib.mrcm_interface_dims(self._iface, byref(n), byref(w)), "mrcm_interface_dims")
        return n.value, w.value

    def copy_interface(self):
        n, _ = self.interface_dims()
        A = np.empty((n, n))
        b = np.empty(n)
        _lib.check(self.lib.mrcm_copy_interface(self._iface, A.ctypes.data_as(c_void_p),
                                                b.ctypes.data_as(c_void_p)), "mrcm_copy_interface")
        return A, b

    def close(self):
        # graphs hold the handles' device addresses: release them first
        for graph in getattr(self, "_graphs", []):
            graph.close()
        self._graphs = []
        if self._iface:
            self.lib.mrcm_interface_destroy(self._iface)
            self._iface = c_void_p()
        if self._mbfs:
            self.lib.mrcm_mbfs_destroy(self._mbfs)
            self._mbfs = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Function-style aliases with the C names.
def build_mbfs(model: MRCM, kx, ky, kz, q, stream=None):
    return model.build_mbfs(kx, ky, kz, q, stream)


def assemble_interface(model: MRCM, stream=None):
    return model.assemble_interface(stream)


def solve_interface(model: MRCM, refine=0, stream=None, method=IFACE_AUTO, rtol=0.0):
    return model.solve_interface(refine=refine, stream=stream, method=method, rtol=rtol)


def reconstruct(model: MRCM, X, stream=None):
    return model.reconstruct(X, stream=stream)


def postprocess_mean(model: MRCM, U, stream=None):
    return model.postprocess_mean(U, stream=stream)


class TwoPhase:
    """The IMPES saturation step of a two-phase run on an nx x ny x nz grid of
    hx x hy x hz cells (mrcm_transport_dt, mrcm_transport_step,
    mrcm_mobility_scale).  Saturations, sources and velocities are float64
    device tensors: S and q with N entries, U with 6 N (face-major)."""

    def __init__(self, dims, h, mu_w, mu_o):
        self.dims = tuple(int(d) for d in dims)
        self.h = tuple(float(x) for x in h)
        self.mu_w, self.mu_o = float(mu_w), float(mu_o)
        self.n = self.dims[0] * self.dims[1] * self.dims[2]
        self._c = CTwoPhase(self.dims[0], self.dims[1], self.dims[2], *self.h, self.mu_w, self.mu_o)
        self.lib = _lib.load()

    def dt(self, U, S, cfl=1.0, dt_max=float("inf"), out=None, stream=None):
        """min(dt_max, the CFL bound of eq. CFL) into a one-entry device
        tensor, which stays on the device; dt_max when nothing moves."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=S.device)
        code = self.lib.mrcm_transport_dt(byref(self._c), _dev_ptr(U, "U", 6 * self.n), _dev_ptr(S, "S", self.n),
                                          c_double(cfl), c_double(dt_max), _stream_ptr(stream),
                                          _dev_ptr(out, "dt", 1))
        _lib.check(code, "mrcm_transport_dt")
        return out

    def step(self, U, q, S, dt, out=None, stream=None):
        """One saturation step; dt a one-entry device tensor (dt()) or a number."""
        import torch
        if not isinstance(dt, torch.Tensor):
            dt = torch.full((1,), float(dt), dtype=torch.float64, device=S.device)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=S.device)
        qp = _dev_ptr(q, "q", self.n) if q is not None else None
        code = self.lib.mrcm_transport_step(byref(self._c), _dev_ptr(U, "U", 6 * self.n), qp,
                                            _dev_ptr(S, "S", self.n), _dev_ptr(dt, "dt", 1), _stream_ptr(stream),
                                            _dev_ptr(out, "S_out", self.n))
        _lib.check(code, "mrcm_transport_step")
        return out

    def mark_sources(self, q, stream=None):
        """The marks of q's sources (mrcm_transport_mark_sources): a uint8
        device tensor for advance(marks=...), valid while q holds."""
        import torch
        nb = self.lib.mrcm_transport_marks_bytes(byref(self._c))
        marks = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=q.device)
        code = self.lib.mrcm_transport_mark_sources(byref(self._c), _dev_ptr(q, "q", self.n), _stream_ptr(stream),
                                                    c_void_p(marks.data_ptr()))
        _lib.check(code, "mrcm_transport_mark_sources")
        return marks

    def advance(self, U, q, S, dt, cfl=1.0, dt_max=float("inf"), out=None, dt_next=None, stream=None, marks=None):
        """One step with dt (a one-entry device tensor) and the next step's
        dt under the same U: returns (S_out, dt_next).  marks: from
        mark_sources(q), or None (q read everywhere)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=S.device)
        if dt_next is None:
            dt_next = torch.empty(1, dtype=torch.float64, device=S.device)
        qp = _dev_ptr(q, "q", self.n) if q is not None else None
        mp = None
        if marks is not None:
            nb = self.lib.mrcm_transport_marks_bytes(byref(self._c))
            if marks.dtype != torch.uint8 or marks.device.type != "cuda" or marks.numel() < nb:
                raise ValueError(f"marks must be a uint8 device tensor of {nb} entries from mark_sources")
            mp = c_void_p(marks.data_ptr())
        code = self.lib.mrcm_transport_advance(byref(self._c), _dev_ptr(U, "U", 6 * self.n), qp, mp,
                                               _dev_ptr(S, "S", self.n), _dev_ptr(dt, "dt", 1), c_double(cfl),
                                               c_double(dt_max), _stream_ptr(stream), _dev_ptr(out, "S_out", self.n),
                                               _dev_ptr(dt_next, "dt_next", 1))
        _lib.check(code, "mrcm_transport_advance")
        return out, dt_next

    def mobility_scale(self, S, kx, ky, kz, out=None, stream=None):
        """K lambda(S) per cell: returns (kx', ky', kz')."""
        import torch
        if out is None:
            out = tuple(torch.empty(self.n, dtype=torch.float64, device=S.device) for _ in range(3))
        ins = [_dev_ptr(t, n, self.n) for t, n in ((kx, "kx"), (ky, "ky"), (kz, "kz"))]
        outs = [_dev_ptr(t, n, self.n) for t, n in zip(out, ("kx_out", "ky_out", "kz_out"))]
        code = self.lib.mrcm_mobility_scale(byref(self._c), _dev_ptr(S, "S", self.n), *ins, _stream_ptr(stream),
                                            *outs)
        _lib.check(code, "mrcm_mobility_scale")
        return tuple(out)


def transport_dt(tp: TwoPhase, U, S, cfl=1.0, dt_max=float("inf"), stream=None):
    return tp.dt(U, S, cfl, dt_max, stream=stream)


def transport_step(tp: TwoPhase, U, q, S, dt, stream=None):
    return tp.step(U, q, S, dt, stream=stream)


def transport_advance(tp: TwoPhase, U, q, S, dt, cfl=1.0, dt_max=float("inf"), stream=None, marks=None):
    return tp.advance(U, q, S, dt, cfl, dt_max, stream=stream, marks=marks)


def mobility_scale(tp: TwoPhase, S, kx, ky, kz, stream=None):
    return tp.mobility_scale(S, kx, ky, kz, stream=stream)
