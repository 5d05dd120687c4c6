#!/usr/bin/env python3
"""MRCM benchmark: one step = one whole MRCM solve (Algorithm 2) on the GPU.

Workload: the 60x220x85 channelised reservoir block (cells of 20x10x2 ft),
3x11x17 = 561 subdomains of 20x20x5 cells, patches 2x1 on x/y-normal and 2x2
on z-normal interfaces (N_V = 3,880 patches, 15,520 MBFs), alpha = 1,
quarter-five-spot wells, synthetic seeded field.  Inputs are resident in HBM
before the timed region.

Reported: MBFs per second of whole MRCM solve (value), cells per second, the
build-only rate, stage times from HIP events, the roofline position of the
dominant kernel, the error against the FP64 CPU oracle, and the oracle's own
rate on this host (cpu_baseline).
"""
from __future__ import annotations

import argparse
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(case, precision, steps, warmup, refine, fp64_refine=1, pcg_max_iter=50, warm=None, net=None,
            graph=True, tune=False):
    """warm (PCG only): relative size of a mobility change.  The MBFs of the
    unchanged field start the conjugate gradients of every timed build on the
    field multiplied cell by cell by exp(warm * g), g standard normal (seed 7),
    as when a two-phase run rebuilds its MBFs between pressure solves.
    net (PCG only): a trained WarmStartNet; every timed build first gathers
    the network's inputs from the previous build, runs the network and uses
    its Galerkin-scaled output as the starting guess."""
    import torch
    import paper_2103_08513_amd as lib
    from paper_2103_08513_amd import _lib
    pb = case.problem
    dev = torch.device("cuda:0")
    kx, ky, kz, q = (torch.as_tensor(a, dtype=torch.float64, device=dev) for a in (pb.kx, pb.ky, pb.kz, pb.q))
    model = lib.MRCM(pb, case.partition, case.iface, alpha=case.alpha, precision=precision,
                     fp64_refine=fp64_refine, pcg_max_iter=pcg_max_iter)
    N = pb.n
    X = None
    x0 = None
    tuned = model.autotune(kx, ky, kz, q) if tune else None
    if warm is not None:
        model.build_mbfs(kx, ky, kz, q)
        torch.cuda.synchronize()
        x0 = torch.cat([torch.from_numpy(model.copy_mbfs(l).reshape(-1))
                        for l in range(model.info().n_sub)]).to(dev)
        lam = torch.as_tensor(np.exp(warm * np.random.default_rng(7).standard_normal(N)), device=dev)
        kx, ky, kz = kx * lam, ky * lam, kz * lam
    p = torch.empty(N, dtype=torch.float64, device=dev)
    U = torch.empty(6 * N, dtype=torch.float64, device=dev)

    nn_subs = None
    if net is not None:
        from paper_2103_08513_amd.surrogate import net_subdomains, warm_start
        model.build_mbfs(kx, ky, kz, q)
        nn_subs, nn_dims = net_subdomains(model)
        x0 = torch.zeros(model.mbf_layout()[-1], dtype=torch.float64, device=dev)

    def step():
        nonlocal X
        if nn_subs is not None:
            warm_start(model, net, nn_subs, nn_dims, x0)
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
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    # stage times from HIP events, over the same number of steps
    L.mrcm_profile_reset()
    L.mrcm_profile_enable(1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = _lib.CProfile()
    L.mrcm_profile_get(ctypes_byref(prof))
    L.mrcm_profile_enable(0)
    stages = {}
    for i, name in enumerate(_lib.STAGES):
        if prof.count[i]:
            stages[name] = {"ms_total": prof.ms[i], "count": int(prof.count[i]),
                            "ms_avg": prof.ms[i] / prof.count[i]}
    # the same step replayed from a recorded HIP graph (FP64 form only)
    graph_ms = None
    if precision == 0 and graph:
        nv = model.info().n_patch
        Xg = torch.empty(2 * nv, dtype=torch.float64, device=dev)
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
    # the interface residual once, outside the timed and profiled loops
    model.solve_interface(X, refine=refine, residual=True)
    torch.cuda.synchronize()
    info = model.info()
    # per-subdomain shapes from the library: (N_l, b_l, m_l, solve group)
    shapes = []
    for l in range(info.n_sub):
        si = model.subdomain(l)
        shapes.append((si.n_cells, si.band, si.n_rhs, si.solve_group))
    n_dims, w = model.interface_dims()
    out = dict(ms_step=ms_step, graph_ms=graph_ms, tuned=tuned, stages=stages, info=info, interface_n=n_dims, interface_w=w,
               p=p.cpu().numpy(), U=U.view(6, N).cpu().numpy(), X=X.cpu().numpy(),
               interface_residual=model.interface_residual, sub_shapes=shapes)
    model.close()
    return out


def train_surrogate(seeds=(1, 2), epochs=3):
    """The warm-start network trained (outside any timed region) on the MBFs of
    the FP64 path for channelised fields of other seeds than the workload's."""
    import torch
    import paper_2103_08513_amd as lib
    from mrcm_inputs import config2
    from paper_2103_08513_amd.surrogate import WarmStartNet, features, net_subdomains
    net = WarmStartNet(seed=0)
    inps, tgts = [], []
    t0 = time.perf_counter()
    for seed in seeds:
        c = config2(seed=seed)
        pb = c.problem
        m = lib.MRCM(pb, c.partition, c.iface, alpha=c.alpha, precision=lib.FP64)
        m.build_mbfs(*(torch.as_tensor(a, dtype=torch.float64, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)))
        subs, dims = net_subdomains(m)
        i, t = features(m, subs, dims)
        inps.append(i)
        tgts.append(t)
        m.close()
    inp, tgt = torch.cat(inps), torch.cat(tgts)
    hist = net.train(inp, tgt, dims, epochs=epochs, batch=256, lr=3e-3, seed=0)
    torch.cuda.synchronize()
    info = {"params": net.n_params(), "channels": list(net.channels), "dilations": list(net.dilations),
            "train_fields": [f"channelised 60x220x85, seed {s}" for s in seeds], "samples": int(inp.shape[0]),
            "epochs": epochs, "loss_by_epoch": hist, "train_seconds": time.perf_counter() - t0}
    log(f"network trained: {info['params']} parameters, loss {[round(h, 3) for h in hist]}")
    del inp, tgt, inps, tgts
    return net, info


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)


def cpu_baseline(case):
    """The CPU oracle as it stands, one thread, whole MRCM solve of the workload."""
    from threadpoolctl import threadpool_limits
    from oracle.mrcm import mrcm_solve
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        r = mrcm_solve(case)
        t = time.perf_counter() - t
    return r, t


def solve_algorithmic_bytes(shapes, es, group=None):
    """Bytes one k_solve launch must move: the band factor and the inverses of
    its 16x16 diagonal blocks read once per sweep (forward and backward), the
    right-hand sides read once and the solutions written once (FP64).  With
    `group`, only the subdomains of that solve group (the launch timed as the
    'solve' stage when the first solve is split)."""
    nbytes = 0.0
    for l_n, l_b, l_m, l_g in shapes:
        if group is not None and l_g != group:
            continue
        panels = (l_n + 15) // 16
        nbytes += 2.0 * es * (l_n * (l_b + 1) + 256 * panels) + 2.0 * 8.0 * l_n * l_m
    return nbytes


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, if it was taken on the current kernel source."""
    import hashlib
    path = os.path.join(HERE, "profiles", f"{kernel}.{workload}.pmc.txt")
    src = os.path.join(HERE, "paper_2103_08513_amd", "csrc", "local_kernels.hip")
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
    if fields.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline_for(stage_name, res, info, precision):
    st = res["stages"].get(stage_name)
    if st is None:
        return None
    sec = st["ms_avg"] * 1e-3
    es = 4 if precision == 1 else 8
    if stage_name == "factor":
        flops = info.factor_flops
        peak = PEAK_FP32_TFLOPS if precision == 1 else PEAK_FP64_TFLOPS
        ach = flops / sec / 1e12
        return {"kernel": "k_factor", "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None, "ms_avg": st["ms_avg"],
                "algorithmic_flops": flops}
    if stage_name == "solve":
        # the 'solve' stage is one launch: group 0 when the solve is split
        # (some subdomain in group 1), otherwise all subdomains
        split = any(sh[3] == 1 for sh in res["sub_shapes"])
        nbytes = solve_algorithmic_bytes(res["sub_shapes"], es, 0 if split else None)
        ach = nbytes / sec / 1e9
        traffic = measured_traffic("k_solve", "60x220x85") if precision == 0 else None
        return {"kernel": "k_solve", "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "ms_avg": st["ms_avg"],
                "algorithmic_bytes": nbytes}
    if stage_name == "pcg":
        # FP32 inner iterations: 22 flops per row (7-point product 12, two
        # dot products 4, three vector updates 6); the FP64 residuals of the
        # restarts are left out.  All subdomains of the workload have the same
        # number of cells.
        rows = info.n_cells / info.n_sub
        flops = 22.0 * rows * info.pcg_iters
        ach = flops / sec / 1e12
        return {"kernel": "k_pcg", "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS, "traffic": None, "ms_avg": st["ms_avg"],
                "algorithmic_flops": flops}
    return None


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32ir"], default="fp64")
    ap.add_argument("--refine", type=int, default=0, help="FP64 refinement steps of the interface solve")
    ap.add_argument("--fp64-refine", type=int, default=1, help="FP64 refinement sweeps of the FP64 local solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other precision")
    ap.add_argument("--no-pcg", action="store_true", help="skip the conjugate-gradient form")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the network-started conjugate gradients")
    ap.add_argument("--no-graph", action="store_true", help="skip the replay of the recorded step")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default tunables)")
    ap.add_argument("--copy-calibration", type=float, default=None, metavar="MB",
                    help="only run a device copy of this many MB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the MRCM library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    if args.copy_calibration is not None:
        copy_calibration(args.copy_calibration)
        return
    from mrcm_inputs import config2
    case = config2()
    pb = case.problem
    prec = 1 if args.precision == "fp32ir" else 0
    log(f"workload 60x220x85, precision {args.precision}, steps {args.steps}, warmup {args.warmup}")
    res = run_gpu(case, prec, args.steps, args.warmup, args.refine, args.fp64_refine, graph=not args.no_graph,
                  tune=not args.no_tune)
    info = res["info"]
    if res["graph_ms"] is not None:
        log(f"graph replay ms/step {res['graph_ms']:.3f}")
    log(f"ms/step {res['ms_step']:.3f}; stages " +
        ", ".join(f"{k} {v['ms_avg']:.3f}" for k, v in res["stages"].items()))
    secondary = None
    if not args.no_secondary:
        other = 1 - prec
        r2 = run_gpu(case, other, args.steps, args.warmup, args.refine, args.fp64_refine)
        secondary = r2
        log(f"other precision ms/step {r2['ms_step']:.3f}")
    pcg_runs = []
    if not args.no_pcg:
        # the conjugate-gradient form at the default budget (50 inner
        # iterations per column, band-Cholesky fallback) and with a budget
        # that lets every column converge
        for budget, warm in ((50, None), (1000, None), (1000, 0.05)):
            r = run_gpu(case, 2, min(args.steps, 3), 1, args.refine, pcg_max_iter=budget, warm=warm)
            r["budget"] = budget
            r["warm"] = warm
            r["surrogate"] = None
            pcg_runs.append(r)
            log(f"pcg budget {budget}, warm start {warm}: ms/step {r['ms_step']:.3f}, fallback {r['info'].pcg_fallback}, "
                f"iterations {r['info'].pcg_iters}")
        if not args.no_surrogate:
            net, train_info = train_surrogate()
            r = run_gpu(case, 2, min(args.steps, 3), 1, args.refine, pcg_max_iter=1000, net=net)
            r["budget"] = 1000
            r["warm"] = None
            r["surrogate"] = train_info
            pcg_runs.append(r)
            log(f"pcg with the network's start: ms/step {r['ms_step']:.3f}, iterations {r['info'].pcg_iters}")
    cpu = None
    err = {}
    if not args.no_cpu_baseline:
        log("oracle (CPU, FP64) whole solve ...")
        from oracle.norms import rel_l2
        ref, t_cpu = cpu_baseline(case)
        cpu = {"value": info.n_mbfs / t_cpu, "unit": "MBFs/s", "cores": 1, "kind": "oracle",
               "sample": "whole MRCM solve of the 60x220x85 workload (561 subdomains, 15,520 MBFs), "
                         "single thread", "seconds": t_cpu, "mcells_per_s": pb.n / t_cpu / 1e6}
        err = {"p": rel_l2(res["p"], ref.p), "U": rel_l2(res["U"], ref.U), "pi": rel_l2(res["X"], ref.pi)}
        if secondary is not None:
            secondary["err"] = {"p": rel_l2(secondary["p"], ref.p), "U": rel_l2(secondary["U"], ref.U)}
        for r in pcg_runs:
            if r["warm"] is None:
                r["err"] = {"p": rel_l2(r["p"], ref.p), "U": rel_l2(r["U"], ref.U)}
    t_step = res["ms_step"] * 1e-3
    build_ms = sum(res["stages"].get(k, {}).get("ms_avg", 0.0) *
                   (res["stages"].get(k, {}).get("count", 0) / max(1, args.steps))
                   for k in ("coef", "factor", "rhs", "solve", "residual", "refine", "flux"))
    # dominant hot-path kernel: k_solve (one launch per solve and per
    # refinement sweep); the factorisation's position is reported beside it
    roof = roofline_for("solve", res, info, prec)
    roof_factor = roofline_for("factor", res, info, prec)
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
        "config": {"workload": "60x220x85 channelised block, 561 subdomains of 20x20x5, "
                               "2x1/2x1/2x2 patches, alpha 1, MRCM whole solve",
                   "cells": pb.n, "subdomains": info.n_sub, "patches": info.n_patch,
                   "mbfs": int(info.n_mbfs), "precision": args.precision},
        "mcells_per_s": pb.n / t_step / 1e6,
        "autotune": res["tuned"],
        "graph": (None if res["graph_ms"] is None else
                  {"ms_per_step": res["graph_ms"], "value": info.n_mbfs / (res["graph_ms"] * 1e-3),
                   "what": "the same step recorded once by stream capture and replayed (mrcm_graph_launch)"}),
        "build_mbfs_per_s": info.n_mbfs / (build_ms * 1e-3) if build_ms > 0 else None,
        "build_ms": build_ms,
        "stages_ms": {k: round(v["ms_avg"] * v["count"] / args.steps, 4) for k, v in res["stages"].items()},
        "interface": {"unknowns": res["interface_n"], "bandwidth": res["interface_w"],
                      "rel_residual": res["interface_residual"]},
        "rel_err_vs_oracle": err,
        "roofline": roof,
        "roofline_factor": roof_factor,
        "cpu_baseline": cpu,
    }
    if prec == 1 or secondary is not None:
        ir_info = info if prec == 1 else secondary["info"]
        line["ir"] = {"sweeps": int(ir_info.ir_iters), "residual": ir_info.ir_residual}
    if secondary is not None:
        sp = "fp32ir" if prec == 0 else "fp64"
        line["other_precision"] = {
            "precision": sp, "ms_per_step": secondary["ms_step"],
            "value": info.n_mbfs / (secondary["ms_step"] * 1e-3),
            "stages_ms": {k: round(v["ms_avg"] * v["count"] / args.steps, 4)
                          for k, v in secondary["stages"].items()},
            "rel_err_vs_oracle": secondary.get("err"),
            "roofline": roofline_for("solve", secondary, secondary["info"], 1 - prec),
            "roofline_factor": roofline_for("factor", secondary, secondary["info"], 1 - prec),
        }
    if pcg_runs:
        line["pcg"] = [{
            "budget": r["budget"], "ms_per_step": r["ms_step"],
            "warm_start": (None if r["warm"] is None else
                           f"MBFs of the unchanged field; timed builds on k * exp({r['warm']} g), "
                           "g standard normal per cell"),
            "surrogate": r["surrogate"],
            "value": info.n_mbfs / (r["ms_step"] * 1e-3),
            "fallback_subdomains": int(r["info"].pcg_fallback),
            "inner_iterations": int(r["info"].pcg_iters),
            "columns": int(r["info"].n_rhs),
            "stages_ms": {k: round(v["ms_avg"] * v["count"] / min(args.steps, 3), 4)
                          for k, v in r["stages"].items()},
            "rel_err_vs_oracle": r.get("err"),
            "roofline": roofline_for("pcg", r, r["info"], 2),
        } for r in pcg_runs]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
