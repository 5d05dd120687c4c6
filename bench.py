#!/usr/bin/env python3
"""MRCM benchmark: one step = one whole MRCM solve (Algorithm 2) on the GPU.

Workload: the 600x2200x85 channelised reservoir block (112.2M cells of
20x10x2 ft, permeability contrast 1e8), 30x110x17 = 56,100 subdomains of
20x20x5 cells, patches 2x1 on x/y-normal and 2x2 on z-normal interfaces
(430,840 patches, 1,723,360 MBFs, 861,680 interface unknowns), alpha = 1,
quarter-five-spot well columns, synthetic seeded field.  Every factor stays
resident in HBM.  Inputs are resident in HBM before the timed region.

Reported: MBFs per second of whole MRCM solve (value), cells per second, the
build-only rate, stage times from HIP events, the FP32-with-refinement and
network-started forms of the same step, the roofline position of the
dominant kernel, the error against the CPU oracle on the workload's exact
60x220x85 corner block, full-size residual and mass balance, and the
oracle's own rate on this host (cpu_baseline, a bounded sample).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
WORKLOAD = "600x2200x85"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _stages(L, _lib, steps):
    prof = _lib.CProfile()
    L.mrcm_profile_get(ctypes.byref(prof))
    out = {}
    for i, name in enumerate(_lib.STAGES):
        if prof.count[i]:
            out[name] = {"ms_total": prof.ms[i], "count": int(prof.count[i]), "ms_avg": prof.ms[i] / prof.count[i],
                         "ms_per_step": prof.ms[i] / steps}
    return out


def run_gpu(case, precision, steps, warmup, refine, graph=False, tune=False, net=None, pcg_max_iter=1000,
            profile=True, mean=False, transport=False, cpu=True):
    """K timed whole solves of `case` in the given form (0 FP64, 1 FP32 with
    FP64 refinement, 2 conjugate gradients started from the network `net`),
    then the same K steps with stage profiling, then (FP64) the step replayed
    from a recorded HIP graph, then (mean) K timed Mean post-processings of
    the last step's velocity, then (transport) the two-phase saturation step
    under the Mean velocity."""
    import torch
    import paper_2103_08513_amd as lib
    from paper_2103_08513_amd import _lib
    pb = case.problem
    dev = torch.device("cuda:0")
    kx, ky, kz, q = (torch.as_tensor(a, dtype=torch.float64, device=dev) for a in (pb.kx, pb.ky, pb.kz, pb.q))
    model = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=precision,
                     pcg_max_iter=pcg_max_iter)
    tuned = model.autotune(kx, ky, kz, q) if tune else None
    N = pb.n
    p = torch.empty(N, dtype=torch.float64, device=dev)
    U = torch.empty(6 * N, dtype=torch.float64, device=dev)
    X = None
    nn_subs = x0 = None
    if net is not None:
        from paper_2103_08513_amd.surrogate import net_subdomains
        model.build_mbfs(kx, ky, kz, q)
        torch.cuda.synchronize()
        nn_subs, nn_dims = net_subdomains(model)
        x0 = torch.zeros(model.mbf_layout()[-1], dtype=torch.float64, device=dev)

    def step():
        nonlocal X
        if nn_subs is not None:
            from paper_2103_08513_amd.surrogate import warm_start_unet
            warm_start_unet(model, net, nn_subs, nn_dims, x0)
        model.build_mbfs(kx, ky, kz, q, x0=x0, x0_scale=nn_subs is not None)
        model.assemble_interface()
        X = model.solve_interface(X, refine=refine)
        model.reconstruct(X, p, U)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    L = _lib.load()
    L.mrcm_profile_reset()
    L.mrcm_profile_enable(0)
    # timed region: K whole solves, synchronised on both sides
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    # stage times from HIP events over the same number of steps
    stages = {}
    if profile:
        L.mrcm_profile_reset()
        L.mrcm_profile_enable(1)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        stages = _stages(L, _lib, steps)
        L.mrcm_profile_enable(0)
    graph_ms = None
    if graph and precision == 0:
        Xg = torch.empty_like(X)
        torch.cuda.synchronize()
        gs = torch.cuda.Stream()  # capture needs a stream other than the null stream
        g = model.capture(kx, ky, kz, q, Xg, p, U, refine=refine, stream=gs)
        for _ in range(warmup):
            g.launch(stream=gs)
        g.check(stream=gs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch(stream=gs)
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / steps
        g.check(stream=gs)
        g.close()
    mean_out = transport_out = None
    if mean:
        mean_out = time_mean(model, pb, case.partition, U, steps)
    if transport:
        transport_out = time_transport(model, pb, U, max(50, 10 * steps), cpu)
    # residual and mass balance once, outside the timed and profiled loops
    model.solve_interface(X, refine=refine, residual=True)
    torch.cuda.synchronize()
    info = model.info()
    iinfo = model.interface_info()
    Uh = U.view(6, N).cpu().numpy()
    A = np.array([pb.hy * pb.hz, pb.hx * pb.hz, pb.hx * pb.hy])
    Q = Uh * np.repeat(A, 2)[:, None]
    imbalance = float(np.max(np.abs(Q.sum(axis=0) - pb.q)) / np.max(np.abs(Q)))
    del Uh, Q
    shapes = []
    for l in range(info.n_sub):
        si = model.subdomain(l)
        shapes.append((si.n_cells, si.band, si.n_rhs, si.solve_group))
    out = dict(ms_step=ms_step, graph_ms=graph_ms, tuned=tuned, stages=stages, info=info, iinfo=iinfo,
               interface_residual=model.interface_residual, refine_iters=model.interface_iters,
               mass_imbalance=imbalance, sub_shapes=shapes, mean=mean_out, transport=transport_out)
    model.close()
    del p, U, X, kx, ky, kz, q
    torch.cuda.empty_cache()
    return out


def time_mean(model, pb, part, U, steps):
    """The Mean post-processing (mrcm_postprocess_mean) of the step's velocity:
    one untimed call (it sets up its buffers), then K calls timed with HIP
    events on the stream they run on, and the balance of the result."""
    import torch
    N = pb.n
    pt = torch.empty(N, dtype=torch.float64, device=U.device)
    Ut = torch.empty(6 * N, dtype=torch.float64, device=U.device)
    model.postprocess_mean(U, pt=pt, Ut=Ut)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        model.postprocess_mean(U, pt=pt, Ut=Ut)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    A = torch.tensor([pb.hy * pb.hz] * 2 + [pb.hx * pb.hz] * 2 + [pb.hx * pb.hy] * 2, dtype=torch.float64,
                     device=U.device)
    Q = Ut.view(6, N) * A[:, None]
    bal = (Q.sum(dim=0) - torch.as_tensor(pb.q, device=U.device)).abs()
    qmax = float(Q.abs().max())
    del Q
    nx, ny, _ = pb.dims
    lo = [torch.as_tensor(np.asarray(c[:-1], dtype=np.int64), device=U.device) for c in part.cuts]
    pinned = torch.zeros(N, dtype=torch.bool, device=U.device)
    pinned[(lo[0][None, None, :] + nx * (lo[1][None, :, None] + ny * lo[2][:, None, None])).reshape(-1)] = True
    out = {"ms": ms, "mcells_per_s": N / (ms * 1e-3) / 1e6,
           "balance_free_cells": float(bal[~pinned].max()) / qmax,
           "balance_pinned_cells": float(bal[pinned].max()) / qmax,
           "what": "Mean post-processing of the step's velocity (unique Gamma flux, one Neumann problem per "
                   "subdomain by FP64 band Cholesky and one refinement sweep, factors chunked through an 8 GiB "
                   "scratch); balances relative to the largest face flux"}
    del pt, Ut, bal, pinned
    return out


# HBM bytes per cell of one saturation step fused with the next step's CFL
# speed (mrcm_transport_advance with the marks of q's sources): U 48, S 8
# read, S' 8 written (q is read in the marked tiles only, a few of them); the
# neighbours' saturations are re-reads of S served by the caches.
TRANSPORT_BYTES_PER_CELL = 64
# the CFL reduction alone (mrcm_transport_dt): U 48, S 8
SPEED_BYTES_PER_CELL = 56
# K lambda(S) (mrcm_mobility_scale): S 8, K 24 read, K' 24 written
MOBILITY_BYTES_PER_CELL = 56


def time_transport(model, pb, U, steps, cpu=True):
    """The IMPES saturation step under the Mean velocity of the step's U: a
    seeded saturation field (uniform in [0, 1]), mu_o / mu_w = 5, the
    quarter-five-spot wells of the workload.  K timed mrcm_transport_advance
    calls (ping-pong S and dt) with the marks of q's sources, and K with the
    dense q, the CFL reduction and the mobility, each with HIP events on the
    stream they run on; and the oracle's step on a slab of five z-planes, on
    the host."""
    import torch
    import paper_2103_08513_amd as lib
    N = pb.n
    dev = U.device
    _, Ut = model.postprocess_mean(U)
    tp = lib.TwoPhase(pb.dims, (pb.hx, pb.hy, pb.hz), 1.0, 5.0)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    S = [torch.rand(N, dtype=torch.float64, device=dev, generator=g), torch.empty(N, dtype=torch.float64, device=dev)]
    q = torch.as_tensor(pb.q, dtype=torch.float64, device=dev)
    dts = [torch.empty(1, dtype=torch.float64, device=dev) for _ in range(2)]
    V = pb.hx * pb.hy * pb.hz
    dt_max = 0.2 * V / float(np.max(pb.q))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_dt = timed(lambda: tp.dt(Ut, S[0], cfl=1.0 / 6.0, dt_max=dt_max, out=dts[0]), 10)
    kx, ky, kz = (torch.as_tensor(a, dtype=torch.float64, device=dev) for a in (pb.kx, pb.ky, pb.kz))
    kout = tuple(torch.empty(N, dtype=torch.float64, device=dev) for _ in range(3))
    ms_mob = timed(lambda: tp.mobility_scale(S[0], kx, ky, kz, out=kout), 10)
    del kx, ky, kz, kout
    state = [0]
    marks = tp.mark_sources(q)
    use_marks = [None]

    def adv():
        i = state[0]
        tp.advance(Ut, q, S[i], dts[i], cfl=1.0 / 6.0, dt_max=dt_max, out=S[1 - i], dt_next=dts[1 - i],
                   marks=use_marks[0])
        state[0] = 1 - i

    tp.dt(Ut, S[0], cfl=1.0 / 6.0, dt_max=dt_max, out=dts[0])
    ms_dense = timed(adv, steps)
    use_marks[0] = marks
    ms_adv = timed(adv, steps)
    # the step kernel alone: HIP events around its launch (the library's stage
    # profiling) over the same number of steps again
    from paper_2103_08513_amd import _lib
    L = lib.library()
    L.mrcm_profile_reset()
    L.mrcm_profile_enable(1)
    for _ in range(steps):
        adv()
    torch.cuda.synchronize()
    kst = _stages(L, _lib, steps).get("transport")
    L.mrcm_profile_enable(0)
    ms_kernel = kst["ms_avg"] if kst else ms_adv
    Sf = S[state[0]]
    lo, hi = float(Sf.min()), float(Sf.max())
    prof = _summary("k_transport", WORKLOAD, "transport_kernels.hip")
    traffic = None
    if prof:
        try:
            traffic = float(prof["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            traffic = None
    out = {"ms_per_step": ms_adv, "ms_kernel": ms_kernel, "ms_per_step_dense_q": ms_dense,
           "gcells_per_s": N / (ms_adv * 1e-3) / 1e9, "steps": steps,
           "s_range": [lo, hi], "ms_cfl_reduction": ms_dt, "ms_mobility": ms_mob,
           "roofline": {"kernel": "k_transport<true> (mrcm_transport_advance)", "bound": "hbm",
                        "achieved": TRANSPORT_BYTES_PER_CELL * N / (ms_kernel * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": TRANSPORT_BYTES_PER_CELL * N / (ms_kernel * 1e-3) / 1e9 / PEAK_HBM_GBS,
                        "traffic": traffic, "bytes_per_cell": TRANSPORT_BYTES_PER_CELL, "ms_avg": ms_kernel,
                        "note": "HIP events around the step kernel's launches, q read in the marked tiles only "
                                "(ms_per_step: the whole call, with the accumulator clear and the finalising kernel; "
                                "ms_per_step_dense_q: the same calls without the marks)"},
           "roofline_cfl": {"achieved": SPEED_BYTES_PER_CELL * N / (ms_dt * 1e-3) / 1e9, "unit": "GB/s",
                            "frac": SPEED_BYTES_PER_CELL * N / (ms_dt * 1e-3) / 8e12},
           "roofline_mobility": {"achieved": MOBILITY_BYTES_PER_CELL * N / (ms_mob * 1e-3) / 1e9, "unit": "GB/s",
                                 "frac": MOBILITY_BYTES_PER_CELL * N / (ms_mob * 1e-3) / 8e12},
           "what": "IMPES saturation step fused with the next step's CFL speed, velocity held (the inner loop "
                   "between Darcy solves), q read in the tiles its marks name; seeded S uniform in [0, 1], "
                   "mu_o / mu_w = 5, cfl 1/6"}
    if cpu:
        from oracle.transport import transport_step
        nx, ny, nz = pb.dims
        kz5 = 5
        sd = (nx, ny, kz5)
        Us = Ut.view(6, nz, ny * nx)[:, :kz5].cpu().numpy().reshape(6, -1)
        Ss = S[0].view(nz, ny * nx)[:kz5].cpu().numpy().reshape(-1)
        qs = np.asarray(pb.q).reshape(nz, -1)[:kz5].reshape(-1)
        t = time.perf_counter()
        transport_step(sd, (pb.hx, pb.hy, pb.hz), Us, qs, Ss, dt_max * 1e-3, 1.0, 5.0)
        sec = time.perf_counter() - t
        n5 = nx * ny * kz5
        out["cpu_oracle"] = {"kind": "oracle", "cells": n5, "s": sec, "gcells_per_s": n5 / sec / 1e9, "cores": 1,
                             "sample": f"oracle transport_step on the {nx}x{ny}x{kz5} slab of z-planes 0-4"}
        del Us, Ss
    del S, Ut, q
    torch.cuda.empty_cache()
    return out


def time_impes(case, skip, n_darcy):
    """The IMPES loop in the library (mrcm_impes_run) on the workload: from an
    all-oil start, mu_o / mu_w = 5, cfl 1/6, the loop's own step
    dt_max = 0.2 V / max q, `skip` saturation steps per Darcy solve (the
    paper's skipping constant C), n_darcy Darcy solves.  Its own MBF handle
    (created by the first Darcy solve, whose device time includes that)."""
    import torch
    import paper_2103_08513_amd as lib
    pb = case.problem
    dev = torch.device("cuda:0")
    kx, ky, kz, q = (torch.as_tensor(a, dtype=torch.float64, device=dev) for a in (pb.kx, pb.ky, pb.kz, pb.q))
    model = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha)
    S = torch.zeros(pb.n, dtype=torch.float64, device=dev)
    dt_max = 0.2 * pb.hx * pb.hy * pb.hz / float(np.max(pb.q))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = model.impes_run(kx, ky, kz, q, S, 1.0, 5.0, skip=skip, max_steps=skip * n_darcy, dt_max=dt_max, refine=1)
    wall = time.perf_counter() - t0
    water = float(S.sum()) * pb.hx * pb.hy * pb.hz
    injected = st["t"] * float(np.sum(pb.q[pb.q > 0]))
    model.close()
    del kx, ky, kz, q, S
    torch.cuda.empty_cache()
    return {"skip": skip, "darcy_solves": st["darcy_solves"], "steps": st["steps"], "t": st["t"], "wall_s": wall,
            "wall_s_per_darcy_period": wall / max(1, st["darcy_solves"]),
            "ms_darcy_first": st["ms_darcy_first"],
            "ms_darcy_per_later_solve": ((st["ms_darcy"] - st["ms_darcy_first"]) / (st["darcy_solves"] - 1)
                                         if st["darcy_solves"] > 1 else None),
            "ms_mean_per_solve": st["ms_mean"] / max(1, st["darcy_solves"]),
            "ms_per_saturation_step": st["ms_transport"] / max(1, st["steps"]),
            "water_in_place_over_injected": water / injected if injected > 0 else None,
            "what": "mrcm_impes_run from an all-oil start: a Darcy solve (K lambda(S), MBFs rebuilt in place, "
                    "interface, reconstruction) and the Mean post-processing every C saturation steps; device times "
                    "from HIP events (the first Darcy solve creates the MBF and interface handles), wall time "
                    "around the call (one synchronisation per saturation step)"}


def block_errors(case5, precisions, procs, refine):
    """The workload's exact 60x220x85 corner block, laid out as the 60x220x85
    workload, solved on the GPU in each form and by the whole oracle."""
    import torch
    import paper_2103_08513_amd as lib
    from mrcm_inputs import config5_block
    from oracle.mrcm import mrcm_solve
    from oracle.norms import rel_l2
    block = config5_block(case5)
    pb = block.problem
    t = time.perf_counter()
    ref = mrcm_solve(block, processes=procs)
    t_ref = time.perf_counter() - t
    args = [torch.as_tensor(a, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)]
    errs = {}
    for prec in precisions:
        m = lib.MRCM(pb, block.partition, block.iface, alpha=block.alpha, precision=prec)
        p, U, X = m.solve(*args, refine=refine)
        torch.cuda.synchronize()
        errs[{0: "fp64", 1: "fp32ir"}[prec]] = {"p": rel_l2(p.cpu().numpy(), ref.p),
                                               "U": rel_l2(U.cpu().numpy(), ref.U),
                                               "pi": rel_l2(X.cpu().numpy(), ref.pi)}
        m.close()
    return errs, t_ref


def cpu_baseline(case5, n_sample, procs):
    """The oracle as it stands: loop 1 of Algorithm 2 (local systems, MBFs by
    sparse LU with extended-precision refinement, flux blocks) on a bounded,
    evenly strided sample of the workload's subdomains, on a pool of worker
    processes over the host's cores."""
    from oracle.geometry import Geometry
    from oracle.mrcm import build_mbfs
    pb = case5.problem
    geo = Geometry(pb.dims, case5.partition, case5.iface)
    stride = max(1, geo.n_sub // n_sample)
    sample = list(range(0, geo.n_sub, stride))[:n_sample]
    t = time.perf_counter()
    systems, *_ = build_mbfs(pb, geo, case5.alpha, subdomains=sample, processes=procs)
    t = time.perf_counter() - t
    mbfs = sum(2 * len(ls.patches) for ls in systems)
    cells = sum(len(ls.cells) for ls in systems)
    return {"value": mbfs / t, "unit": "MBFs/s", "cores": procs, "kind": "oracle",
            "sample": f"loop 1 (local systems, MBFs, flux blocks) of {len(sample)} of the {geo.n_sub} subdomains "
                      f"(every {stride}th), {mbfs} MBFs, on a pool of {procs} processes",
            "seconds": t, "mcells_per_s": cells / t / 1e6}


def solve_algorithmic_bytes(shapes, es, group):
    """Bytes one band-solve launch must move by the method's own count: the
    band factor read once forward and once backward, and the MBFs (n_cells x
    n_rhs, FP64) once, over the subdomains of the given solve group."""
    nbytes = 0.0
    for l_n, l_b, l_m, l_g in shapes:
        if group is not None and l_g != group:
            continue
        nbytes += 2.0 * es * l_n * (l_b + 1) + 8.0 * l_n * l_m
    return nbytes


def _summary(kernel, workload, source):
    """Fields of a committed rocprofv3 summary, if it was taken on the
    current source of the kernel (sha256 recorded in the summary)."""
    path = os.path.join(HERE, "profiles", f"{kernel}.{workload}.txt")
    src = os.path.join(HERE, "paper_2103_08513_amd", "csrc", source)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return fields if fields.get("kernel_source_sha256") == sha else None


def roofline_solve(res, precision):
    """k_solve, group 1's first solve (the 'solve_rest' stage: one launch)."""
    st = res["stages"].get("solve_rest")
    if st is None:
        return None
    es = 4 if precision == 1 else 8
    nbytes = solve_algorithmic_bytes(res["sub_shapes"], es, 1)
    sec = st["ms_avg"] * 1e-3
    ach = nbytes / sec / 1e9
    traffic = None
    if precision == 0:
        f = _summary("k_solve", WORKLOAD + ".pmc", "local_kernels.hip")
        if f:
            try:
                traffic = float(f["hbm_bytes_per_launch"])
            except (KeyError, ValueError):
                traffic = None
    return {"kernel": "k_solve (group 1's first solve, one launch)", "bound": "hbm", "achieved": ach,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": traffic,
            "ms_avg": st["ms_avg"], "algorithmic_bytes": nbytes}


def roofline_factor(res, precision):
    st = res["stages"].get("factor")
    if st is None:
        return None
    info = res["info"]
    sec = st["ms_per_step"] * 1e-3
    peak = PEAK_FP32_TFLOPS if precision == 1 else PEAK_FP64_TFLOPS
    ach = info.factor_flops / sec / 1e12
    out = {"kernel": "k_factor64" if precision == 0 else "k_factor32", "bound": "mfma", "achieved": ach,
           "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "ms_per_step": st["ms_per_step"],
           "algorithmic_flops": info.factor_flops}
    if precision == 0:
        f = _summary("k_factor64", WORKLOAD + ".sq", "local_kernels.hip")
        if f and "mfma_busy_frac" in f:
            out["mfma_busy_frac"] = float(f["mfma_busy_frac"])
    return out


def roofline_interface(res):
    st = res["stages"].get("lu")
    if st is None:
        return None
    ii = res["iinfo"]
    sec = st["ms_per_step"] * 1e-3
    ach = ii.factor_flops / sec / 1e12
    return {"kernel": "k_mf_step (multifrontal LDL^T, all launches)", "bound": "mfma", "achieved": ach,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
            "ms_per_step": st["ms_per_step"], "algorithmic_flops": ii.factor_flops}


def train_surrogate(train_seeds=range(1000), test_seeds=range(1000, 1100), per_field=50, epochs=4):
    """The encoder-decoder warm start trained (outside any timed region) on
    MBFs the FP64 path builds for channelised fields (seeds 0-999, 50 MBFs per
    field), then its gain measured on unseen fields (seeds 1000-1099): the
    conjugate-gradient form's inner iterations from zero and from the
    network's Galerkin-scaled guess."""
    import torch
    import paper_2103_08513_amd as lib
    from mrcm_inputs import config4_field
    from paper_2103_08513_amd.surrogate import EncoderDecoder, UNET_LAYERS, mbf_dataset, net_subdomains, warm_start_unet
    t0 = time.perf_counter()
    inp, tgt, dims = mbf_dataset(train_seeds, per_field)
    t_data = time.perf_counter() - t0
    net = EncoderDecoder(UNET_LAYERS, seed=0)
    t0 = time.perf_counter()
    hist = net.train(inp, tgt, epochs=epochs, batch=128, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples = int(inp.shape[0])
    del inp, tgt
    it0 = itn = 0
    for seed in test_seeds:
        c = config4_field(seed)
        pb = c.problem
        args = [torch.as_tensor(a, dtype=torch.float64, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)]
        m = lib.MRCM(pb, c.partition, c.iface, alpha=c.alpha, precision=lib.PCG, pcg_max_iter=1000)
        m.build_mbfs(*args)
        it0 += m.info().pcg_iters
        subs, d = net_subdomains(m)
        x0 = warm_start_unet(m, net, subs, d)
        m.build_mbfs(*args, x0=x0, x0_scale=True)
        itn += m.info().pcg_iters
        m.close()
    info = {"params": net.n_params(), "layers": [list(L) for L in UNET_LAYERS],
            "train": f"channelised 60x60x15 fields, seeds {train_seeds[0]}-{train_seeds[-1]}, {per_field} MBFs each",
            "samples": n_samples, "epochs": epochs, "loss_by_epoch": hist, "data_seconds": t_data,
            "train_seconds": t_train,
            "test": f"seeds {test_seeds[0]}-{test_seeds[-1]}: CG inner iterations to 1e-10 from zero {it0}, "
                    f"from the network {itn}",
            "test_iterations_saved_frac": (it0 - itn) / it0}
    log(f"network trained: {info['params']} parameters, loss {[round(h, 3) for h in hist]}; unseen fields: "
        f"{100 * info['test_iterations_saved_frac']:.1f} % fewer CG iterations")
    return net, info


def copy_calibration(mbytes):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = int(mbytes * 1024 * 1024 // 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": {"read": 8 * n, "write": 8 * n}, "launches": 3}),
          flush=True)


def _form_line(res, n_mbfs, n_cells, precision, err=None):
    return {"precision": {0: "fp64", 1: "fp32ir", 2: "surrogate+pcg"}[precision], "ms_per_step": res["ms_step"],
            "value": n_mbfs / (res["ms_step"] * 1e-3), "mcells_per_s": n_cells / (res["ms_step"] * 1e-3) / 1e6,
            "stages_ms": {k: round(v["ms_per_step"], 3) for k, v in res["stages"].items()},
            "ir": {"sweeps": int(res["info"].ir_iters), "residual": res["info"].ir_residual},
            "pcg": {"inner_iterations": int(res["info"].pcg_iters), "fallback_subdomains": int(res["info"].pcg_fallback)},
            "interface_residual": res["interface_residual"], "mass_imbalance": res["mass_imbalance"],
            "rel_err_vs_oracle_block": err}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--refine", type=int, default=1,
                    help="refinement steps of the interface solve (one reaches the FP64 residual floor at 600x2200x85)")
    ap.add_argument("--precision", choices=["fp64", "fp32ir"], default="fp64", help="form of the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other precision")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the network-started form")
    ap.add_argument("--no-block", action="store_true", help="skip the oracle comparison on the corner block")
    ap.add_argument("--no-graph", action="store_true", help="skip the replay of the recorded step")
    ap.add_argument("--tune", action="store_true", help="run the autotuner first (a handle per candidate)")
    ap.add_argument("--no-mean", action="store_true", help="skip the Mean post-processing measurement")
    ap.add_argument("--no-transport", action="store_true", help="skip the saturation-step measurement")
    ap.add_argument("--impes-skip", type=int, default=600, help="skipping constant C of the IMPES leg")
    ap.add_argument("--impes-darcy", type=int, default=3, help="Darcy solves of the IMPES leg (0: skip it)")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="subdomains in the oracle's timed sample")
    ap.add_argument("--copy-calibration", type=float, default=None, metavar="MB",
                    help="only run a device copy of this many MB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1 (the design for more GPUs "
                                   "is described, not built)", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    if args.copy_calibration is not None:
        copy_calibration(args.copy_calibration)
        return
    from mrcm_inputs import config5
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.perf_counter()
    case = config5()
    pb = case.problem
    log(f"workload {WORKLOAD}: inputs in {time.perf_counter() - t:.1f} s; steps {args.steps}, warmup {args.warmup}")
    prec = 1 if args.precision == "fp32ir" else 0
    res = run_gpu(case, prec, args.steps, args.warmup, args.refine, graph=not args.no_graph, tune=args.tune,
                  mean=not args.no_mean, transport=not (args.no_mean or args.no_transport),
                  cpu=not args.no_cpu_baseline)
    info = res["info"]
    log(f"{args.precision}: ms/step {res['ms_step']:.1f}; stages " +
        ", ".join(f"{k} {v['ms_per_step']:.1f}" for k, v in res["stages"].items()))
    if res["transport"]:
        tr = res["transport"]
        log(f"transport: {tr['ms_per_step']:.3f} ms/step ({tr['roofline']['achieved']:.0f} GB/s; dense q "
            f"{tr['ms_per_step_dense_q']:.3f}), CFL reduction "
            f"{tr['ms_cfl_reduction']:.3f} ms, mobility {tr['ms_mobility']:.3f} ms")
    impes = None
    if args.impes_darcy > 0 and not (args.no_mean or args.no_transport):
        impes = time_impes(case, args.impes_skip, args.impes_darcy)
        log(f"impes: C {impes['skip']}, {impes['darcy_solves']} Darcy solves, {impes['steps']} steps in "
            f"{impes['wall_s']:.2f} s (Darcy: first {impes['ms_darcy_first']:.0f} ms, later "
            f"{impes['ms_darcy_per_later_solve'] or 0:.0f} ms; Mean "
            f"{impes['ms_mean_per_solve']:.0f} ms per solve, {impes['ms_per_saturation_step']:.3f} ms per step)")
    secondary = None
    if not args.no_secondary:
        secondary = run_gpu(case, 1 - prec, args.steps, args.warmup, args.refine)
        log(f"other precision ms/step {secondary['ms_step']:.1f}")
    surrogate = None
    if not args.no_surrogate:
        net, train_info = train_surrogate()
        surrogate = run_gpu(case, 2, 1, 0, args.refine, net=net, profile=False)
        surrogate["train"] = train_info
        log(f"network-started CG ms/step {surrogate['ms_step']:.1f}")
    errs, t_ref = ({}, None) if args.no_block else block_errors(case, [0, 1], procs, args.refine)
    if errs:
        log(f"corner block vs oracle: {errs} (oracle {t_ref:.1f} s)")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, args.cpu_sample, procs)
        log(f"oracle sample: {cpu['value']:.0f} MBFs/s on {procs} processes")
    t_step = res["ms_step"] * 1e-3
    build_ms = sum(res["stages"].get(k, {}).get("ms_per_step", 0.0)
                   for k in ("coef", "factor", "rhs", "solve", "residual", "refine", "flux", "pcg", "fallback"))
    name = args.precision
    line = {
        "metric": "MBFs/s & Mcells/s per MRCM solve: FP32+IR & surrogate vs FP64, at rel err 1e-8",
        "value": info.n_mbfs / t_step,
        "unit": "MBFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "600x2200x85 channelised block (112.2M cells of 20x10x2 ft, contrast 1e8), "
                               "30x110x17 = 56,100 subdomains of 20x20x5, 2x1/2x1/2x2 patches, alpha 1, "
                               "MRCM whole solve, every factor resident",
                   "cells": pb.n, "subdomains": info.n_sub, "patches": info.n_patch, "mbfs": int(info.n_mbfs),
                   "interface_unknowns": res["iinfo"].n, "precision": name, "interface_refine": args.refine},
        "mcells_per_s": pb.n / t_step / 1e6,
        "build_ms": build_ms,
        "build_mbfs_per_s": info.n_mbfs / (build_ms * 1e-3) if build_ms > 0 else None,
        "stages_ms": {k: round(v["ms_per_step"], 3) for k, v in res["stages"].items()},
        "interface": {"unknowns": res["iinfo"].n, "separators": res["iinfo"].nodes, "levels": res["iinfo"].levels,
                      "largest_front": res["iinfo"].max_front, "front_bytes": res["iinfo"].front_bytes,
                      "factor_flops": res["iinfo"].factor_flops, "refine_steps": res["refine_iters"],
                      "rel_residual": res["interface_residual"]},
        "device_bytes": info.device_bytes + res["iinfo"].device_bytes,
        "mass_imbalance": res["mass_imbalance"],
        "rel_err_vs_oracle": {"what": "the workload's exact 60x220x85 corner block, whole solve vs the whole oracle",
                              **errs.get(name, {})} if errs else None,
        "graph": (None if res["graph_ms"] is None else
                  {"ms_per_step": res["graph_ms"], "value": info.n_mbfs / (res["graph_ms"] * 1e-3),
                   "what": "the same step recorded once by stream capture and replayed (mrcm_graph_launch)"}),
        "autotune": res["tuned"],
        "roofline": roofline_solve(res, prec),
        "roofline_factor": roofline_factor(res, prec),
        "roofline_interface": roofline_interface(res),
        "cpu_baseline": cpu,
        "mean_postprocess": res["mean"],
        "transport": res["transport"],
        "impes": impes,
    }
    if secondary is not None:
        line["other_precision"] = _form_line(secondary, info.n_mbfs, pb.n, 1 - prec,
                                             errs.get("fp32ir" if prec == 0 else "fp64"))
        line["other_precision"]["roofline"] = roofline_solve(secondary, 1 - prec)
        line["other_precision"]["roofline_factor"] = roofline_factor(secondary, 1 - prec)
    if surrogate is not None:
        line["surrogate"] = _form_line(surrogate, info.n_mbfs, pb.n, 2)
        line["surrogate"]["train"] = surrogate["train"]
        line["surrogate"]["steps"] = 1
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
