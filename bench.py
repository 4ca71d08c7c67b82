"""Benchmark of the FP64 FD-MP5 / global-LF / SSPRK(5,4) hot path on one MI355X.

Workload: 3D ideal MHD, 4096 independent blocks of 32^3 : 16^3 : 8^3 cells
(1 : 2 : 4 by count; 25,160,192 interior cells), ghosts filled from a seeded
8-mode field (amplitude 0.1) on rho = 1, p = 1, B = (1, 0, 0), CFL 0.4.

A step is one full SSPRK(5,4) step over every block (5 fused stage launches
plus the on-device dt computation), inputs resident in HBM.  The headline
value is the faster batched form (persistent launches, one per stage or one
per block-size class and stage, after autotuning both; steps replayed from HIP
graphs); the plain per-block launch on the same block list is timed beside it.
One JSON line is printed.

    python bench.py [--gpus 1] [--steps 20] [--warmup 2]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MHD cell-updates/s (batched vs per-block, FP64) + adjoint/forward time ratio"

# Operation counts of one cell in one stage, counted by the oracle's
# counting scalar (oracle/count_ops.py writes the record): arithmetic
# operations (+, -, *, /, sqrt, one each) and comparisons / selections (min,
# max, minmod, median, |x|, branch tests), each executed by the GPU as one
# FP64 VALU lane-operation; "median_form" is MP5 without its early exit (what
# the fused kernel evaluates), "early_exit" the published algorithm's own
# data-dependent count.
OPCOUNT_RECORD = os.path.join("profiles", "oracle_op_count_mhd3d_uneven4096.json")
# Algorithmic HBM bytes per cell per SSPRK(5,4) step: 17 state passes x 8
# variables x 8 bytes (low-storage form: 2+3+4+5+3 passes).
BYTES_PER_CELL_STEP_MHD3D = 17 * 8 * 8   # 8 variables (2D and 3D MHD alike)
# 2D Euler: 17 passes x 4 variables x 8 bytes.
BYTES_PER_CELL_STEP_EULER2D = 17 * 4 * 8
# FP64 VALU: 256 CU x 4 SIMD x 16 FP64 lanes x 2.4 GHz, one operation (an
# add, multiply, fused multiply-add, min, max, compare or select) per lane
# and cycle; 78.6 TFLOP/s counts a fused multiply-add as two flops.
PEAK_FP64_VALU_TOPS = 39.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
STAGES = 5


def strip_comments(src):
    """C++ source without comments and with whitespace collapsed (comment
    edits leave the code, and so the measurements taken on it, unchanged)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash(read=None):
    """Hash of the code (comments and whitespace aside) of the stage kernel
    and the runtime that launches it."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_math.h", "runtime.cpp", "amrvac_internal.h"):
        path = os.path.join("paper_1407_2052_amd", "csrc", f)
        if read is None:
            with open(os.path.join(ROOT, path)) as fh:
                src = fh.read()
        else:
            src = read(path)
        h.update(strip_comments(src).encode())
    return h.hexdigest()[:16]


def measured_traffic(variant, form):
    """HBM bytes per stage (the stage's launches together) from committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (calibrated against a plain copy),
    if they were taken on the current kernel source, on the tile shape and in
    the launch form ("per_class" or "single") that is being timed.  The record
    holds the timed pair of its run and, for the per-class form, every tile
    shape (the autotuner runs each of them per class in the same program)."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_mhd3d_uneven4096_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    if rec.get("variant") == variant and rec.get("form") == form:
        return rec.get("bytes_per_stage")
    if form == "per_class":   # every shape, from the autotuner's per-class pass of the same run
        return rec.get("variants", {}).get(variant, {}).get("bytes_per_stage")
    return None


def measured_traffic_other(leg, variant):
    """HBM bytes per stage of another workload's forward (`leg`: a key of
    FORWARD_LEGS) on tile shape `variant`, from the same committed record:
    every shape of that list's autotuning pass, profiled in a run of its own
    (`bench.py --forward-leg LEG`), if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_mhd3d_uneven4096_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("others", {}).get(leg, {}).get("variants", {}).get(variant, {}).get("bytes_per_stage")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(bs_full, min_seconds=10.0, max_steps=4, single_seconds=5.0):
    """The oracle as it stands, on a bounded sample of the same block list:
    512 blocks drawn with the same 1:2:4 size mix, SSPRK(5,4) steps until at
    least `min_seconds` of wall time, OpenMP over blocks on every core; then
    one thread on 64 of those blocks (same mix) for at least
    `single_seconds`."""
    import numpy as np
    import oracle

    rng = np.random.default_rng(11)
    sizes = bs_full.n[:, 0]

    def sample(counts):
        idx = []
        for s, k in zip((32, 16, 8), counts):
            pool = np.where(sizes == s)[0]
            idx.extend(rng.choice(pool, min(k, len(pool)), replace=False).tolist())
        idx = np.array(sorted(idx))
        sub = bs_full.copy()
        sub.u = [bs_full.u[i] for i in idx]
        sub.n, sub.dx, sub.xlo, sub.nbr = bs_full.n[idx], bs_full.dx[idx], bs_full.xlo[idx], bs_full.nbr[idx]
        return sub

    def run(sub, seconds):
        t0 = time.perf_counter()
        steps = 0
        cur = sub
        while steps < max_steps:
            cur, _ = oracle.run(cur, oracle.SSPRK54, 1, cfl=0.4)
            steps += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return steps, time.perf_counter() - t0

    sub = sample((73, 146, 293))
    cells = sub.interior_cells()
    threads = oracle.num_threads()
    steps, el = run(sub, min_seconds)
    out = {"value": cells * steps / el, "unit": "cell-updates/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{sub.nb} of the 4096 blocks (32^3:16^3:8^3 = 73:146:293, {cells} cells), "
                     f"{steps} SSPRK(5,4) steps, {el:.1f} s wall, OpenMP over blocks"}
    if single_seconds > 0:
        sub1 = sample((9, 18, 37))
        cells1 = sub1.interior_cells()
        oracle.set_threads(1)
        try:
            steps1, el1 = run(sub1, single_seconds)
        finally:
            oracle.set_threads(threads)
        out["single_thread"] = {"value": cells1 * steps1 / el1, "unit": "cell-updates/s",
                                "sample": f"{sub1.nb} blocks (9:18:37, {cells1} cells), {steps1} "
                                          f"SSPRK(5,4) steps, {el1:.1f} s wall, one thread"}
    return out


def adjoint_ratio(nsteps, ckpt, warm=80, ckpt_also=None, per_block_steps=2):
    """Adjoint / forward wall-time ratio on 3D ideal MHD, 256^3 periodic as
    4096 blocks of 16^3 (16-mode velocity and field perturbations, plasma
    beta 1), fixed dt from the CFL rule on the initial state: `warm` steps
    forward (untimed), then `nsteps` timed forward steps, then the adjoint of
    those nsteps (checkpoints every `ckpt` steps, recompute included) with
    lambda_N = rho_N - 1 in the density slot.  The plain per-block launch is
    timed on the same window start.  Then the same forward steps
    with only the blocks near the box centre active (dynamic grid
    activation, safety belt of one block)."""
    import numpy as np
    import torch
    from paper_1407_2052_amd import amrvac, inputs

    print("bench: generating 3D MHD 256^3 periodic (4096 x 16^3)", file=sys.stderr, flush=True)
    bs = inputs.mhd_turbulence_3d()
    cells = bs.interior_cells()
    ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED)
    _, cm = ctx.fd_rhs()
    dt = 0.4 / sum(cm[d] / bs.dx[0, d] for d in range(3))
    # the forward is timed on its fastest tile shape (the adjoint's own
    # kernels have fixed shapes; its pass to the checkpoints uses this one)
    fvar, _ = ctx.autotune(amrvac.SSPRK54, 2)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    print(f"bench: {warm} forward steps to the adjoint window", file=sys.stderr, flush=True)
    ctx.ssprk_step(amrvac.SSPRK54, warm, dt=dt, t=None)
    torch.cuda.synchronize()
    u_w = flat.clone()

    def timed(fn):
        torch.cuda.synchronize()
        e[0].record(stream)
        fn()
        e[1].record(stream)
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]) / 1e3

    fwd = timed(lambda: ctx.ssprk_step(amrvac.SSPRK54, nsteps, dt=dt, t=None))
    ctx.sync()
    lam_n = [torch.zeros_like(v) for v in views]
    for l, v in zip(lam_n, views):
        l[0, 3:-3, 3:-3, 3:-3] = v[0, 3:-3, 3:-3, 3:-3] - 1.0
    out = {"workload": "3D ideal MHD 256^3 periodic, 4096 x 16^3, SSPRK(5,4), steps "
                       f"{warm + 1}-{warm + nsteps} after {warm} forward steps",
           "steps": nsteps, "forward_tile_shape": fvar, "forward_s": fwd,
           "forward_cell_updates_per_s": cells * nsteps / fwd}
    for k in [ckpt] + ([ckpt_also] if ckpt_also else []):
        flat.copy_(u_w)
        lam = [l.clone() for l in lam_n]
        print(f"bench: adjoint of {nsteps} steps (checkpoints every {k})", file=sys.stderr, flush=True)
        adj = timed(lambda: ctx.ssprk_adjoint(amrvac.SSPRK54, dt, nsteps, k, lam))
        key = "" if k == ckpt else f"_ckpt{k}"
        out["ckpt_every" + key] = k
        out["adjoint_s" + key] = adj
        out["ratio" + key] = adj / fwd
    # the same window with RK3 + LIM03 (the paper's other FD combination)
    ctx3, flat3, views3 = amrvac.context_for(bs, amrvac.EXEC_BATCHED, recon=amrvac.LIM03)
    flat3.copy_(u_w)
    fvar3, _ = ctx3.autotune(amrvac.RK3, 2)
    ctx3.ssprk_step(amrvac.RK3, 1, dt=dt, t=None)          # graph capture
    flat3.copy_(u_w)
    fwd3 = timed(lambda: ctx3.ssprk_step(amrvac.RK3, nsteps, dt=dt, t=None))
    ctx3.sync()
    flat3.copy_(u_w)
    lam = [l.clone() for l in lam_n]
    print(f"bench: RK3 + LIM03 adjoint of {nsteps} steps (checkpoints every {ckpt})", file=sys.stderr, flush=True)
    adj3 = timed(lambda: ctx3.ssprk_adjoint(amrvac.RK3, dt, nsteps, ckpt, lam))
    ctx3.close()
    del flat3, views3, lam
    out["lim03_rk3"] = {"steps": nsteps, "ckpt_every": ckpt, "forward_tile_shape": fvar3, "forward_s": fwd3,
                        "adjoint_s": adj3,
                        "ratio": adj3 / fwd3}
    # the plain per-block launch on the same list (one launch per block per stage)
    flat.copy_(u_w)
    ctx.set_exec(amrvac.EXEC_PER_BLOCK)
    ctx.ssprk_step(amrvac.SSPRK54, 1, dt=dt, t=None)      # first launches
    flat.copy_(u_w)
    print(f"bench: per-block launch on the 256^3 list, {per_block_steps} steps", file=sys.stderr, flush=True)
    pb = timed(lambda: ctx.ssprk_step(amrvac.SSPRK54, per_block_steps, dt=dt, t=None))
    ctx.sync()
    ctx.set_exec(amrvac.EXEC_BATCHED)
    out["per_block"] = {"steps": per_block_steps, "cell_updates_per_s": cells * per_block_steps / pb,
                        "batched_over_per_block": (cells * nsteps / fwd) / (cells * per_block_steps / pb)}
    # dynamic grid activation: blocks whose centre lies within 0.25 of the
    # box centre are active, plus a safety belt of one block
    centres = bs.xlo + 0.5 * bs.n * bs.dx
    want = (np.sqrt(((centres - 0.5) ** 2).sum(axis=1)) < 0.25).astype(np.uint8)
    n_act, flags = amrvac.activation_flags(bs.nbr, want, 1)
    flat.copy_(u_w)
    ctx.set_active(flags)
    ctx.ssprk_step(amrvac.SSPRK54, 1, dt=dt, t=None)      # graph capture
    masked = timed(lambda: ctx.ssprk_step(amrvac.SSPRK54, nsteps, dt=dt, t=None))
    ctx.sync()
    out["activation"] = {"active_blocks": int(n_act), "blocks": bs.nb, "active_fraction": n_act / bs.nb,
                         "step_time_fraction": masked / fwd,
                         "active_cell_updates_per_s": n_act * 16 ** 3 * nsteps / masked}
    ctx.close()
    return out


def adjoint_ratio_2d(nsteps=200, ckpt=20):
    """Adjoint / forward wall-time ratio on 2D Euler 256^2 periodic (256
    blocks of 16^2, 8-mode density perturbation, v = 0, p = 1), fixed dt from
    the CFL rule on the initial state, J = 1/2 sum (rho_N - rho*)^2."""
    import torch
    from paper_1407_2052_amd import amrvac, inputs

    bs = inputs.hydro_random_2d()
    target = inputs.hydro_target_density()
    cells = bs.interior_cells()
    ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED)
    _, cm = ctx.fd_rhs()
    dt = 0.4 / sum(cm[d] / bs.dx[0, d] for d in range(2))
    fvar, _ = ctx.autotune(amrvac.SSPRK54, 2)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    u0 = flat.clone()
    ctx.ssprk_step(amrvac.SSPRK54, 1, dt=dt, t=None)      # graph capture
    flat.copy_(u0)

    def timed(fn):
        torch.cuda.synchronize()
        e[0].record(stream)
        fn()
        e[1].record(stream)
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]) / 1e3

    fwd = timed(lambda: ctx.ssprk_step(amrvac.SSPRK54, nsteps, dt=dt, t=None))
    ctx.sync()
    lam = [torch.zeros_like(v) for v in views]
    for b, (l, v) in enumerate(zip(lam, views)):
        l[0, 0, 3:-3, 3:-3] = v[0, 0, 3:-3, 3:-3] - torch.from_numpy(target[b].reshape(v.shape[2] - 6, v.shape[3] - 6)).to(v.device)
    flat.copy_(u0)
    print(f"bench: 2D Euler adjoint of {nsteps} steps (checkpoints every {ckpt})", file=sys.stderr, flush=True)
    adj = timed(lambda: ctx.ssprk_adjoint(amrvac.SSPRK54, dt, nsteps, ckpt, lam))
    ctx.close()
    return {"workload": "2D Euler 256^2 periodic, 256 x 16^2, SSPRK(5,4)", "steps": nsteps, "ckpt_every": ckpt,
            "forward_tile_shape": fvar,
            "forward_s": fwd, "adjoint_s": adj, "ratio": adj / fwd,
            "forward_cell_updates_per_s": cells * nsteps / fwd}


def forward_mhd2d(nsteps, warmup):
    """SSPRK(5,4) + MP5 forward steps of 2D ideal MHD on smooth Orszag-Tang
    data, 512^2 periodic in 1024 blocks of 16^2 (autotuned, batched)."""
    import torch
    from paper_1407_2052_amd import amrvac, inputs
    bs = inputs.orszag_tang_2d(512, 16)
    cells = bs.interior_cells()
    ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED)
    var, _ = ctx.autotune(amrvac.SSPRK54, 2)
    stream = torch.cuda.current_stream()
    ctx.ssprk_step(amrvac.SSPRK54, warmup, cfl=0.4, t=None)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.ssprk_step(amrvac.SSPRK54, nsteps, cfl=0.4, t=None)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.sync()
    el = e0.elapsed_time(e1) / 1e3
    ctx.close()
    return {"workload": "2D ideal MHD, smooth Orszag-Tang data, 512^2 periodic, 1024 x 16^2, SSPRK(5,4) + MP5",
            "tile_shape": var, "steps": nsteps, "ms_per_step": 1e3 * el / nsteps,
            "cell_updates_per_s": cells * nsteps / el, "cells": cells}


FORWARD_LEGS = {
    "mhd3d_periodic256": "3D ideal MHD 256^3 periodic, 4096 x 16^3",
    "euler2d_256": "2D Euler 256^2 periodic, 256 x 16^2",
    "mhd2d_512": "2D ideal MHD, smooth Orszag-Tang data, 512^2 periodic, 1024 x 16^2",
}


def forward_leg(leg, nsteps, warmup):
    """Only the SSPRK(5,4) + MP5 forward of one of the other lists (autotuned,
    batched), for profiling that list's stage kernel in a run of its own."""
    import torch
    from paper_1407_2052_amd import amrvac, inputs
    bs = {"mhd3d_periodic256": inputs.mhd_turbulence_3d, "euler2d_256": inputs.hydro_random_2d,
          "mhd2d_512": lambda: inputs.orszag_tang_2d(512, 16)}[leg]()
    cells = bs.interior_cells()
    ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED)
    var, _ = ctx.autotune(amrvac.SSPRK54, 2)
    stream = torch.cuda.current_stream()
    ctx.ssprk_step(amrvac.SSPRK54, warmup, cfl=0.4, t=None)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.ssprk_step(amrvac.SSPRK54, nsteps, cfl=0.4, t=None)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.sync()
    el = e0.elapsed_time(e1) / 1e3
    ctx.close()
    return {"leg": leg, "workload": FORWARD_LEGS[leg], "tile_shape": var, "steps": nsteps,
            "ms_per_step": 1e3 * el / nsteps, "cell_updates_per_s": cells * nsteps / el, "cells": cells}


def stage_roofline(key, cells, stage_s, bytes_per_cell_step):
    """FP64 VALU roofline of one fused stage launch: the oracle-counted
    operations per cell (median form) x cells / the launch time, against
    PEAK_FP64_VALU_TOPS; beside it the method's own early-exit count, the
    arithmetic flops alone against the FP64 peak, and the algorithmic HBM
    rate against 8 TB/s and the 60 % target."""
    with open(os.path.join(ROOT, OPCOUNT_RECORD)) as fh:
        rec = json.load(fh)[key]["per_cell_stage"]
    med, ee = rec["median_form"], rec["early_exit"]
    ops = med["flops"] + med["comparisons"]
    ops_ee = ee["flops"] + ee["comparisons"]
    achieved = ops * cells / stage_s / 1e12
    hbm = bytes_per_cell_step * cells / STAGES / stage_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TOPS, "unit": "TOP/s",
            "frac": achieved / PEAK_FP64_VALU_TOPS, "traffic": None,
            "ops_per_cell_stage": ops, "ops_source": f"{OPCOUNT_RECORD} [{key}] median form (flops + comparisons)",
            "method_early_exit": {"ops_per_cell_stage": ops_ee,
                                  "achieved": ops_ee * cells / stage_s / 1e12,
                                  "frac": ops_ee * cells / stage_s / 1e12 / PEAK_FP64_VALU_TOPS},
            "fp64_flops": {"per_cell_stage": med["flops"], "achieved_TFLOPs": med["flops"] * cells / stage_s / 1e12,
                           "frac_of_78_6": med["flops"] * cells / stage_s / 1e12 / PEAK_FP64_TFLOPS},
            "stage_ms": 1e3 * stage_s,
            "hbm_algorithmic_GBs": hbm, "hbm_frac": hbm / PEAK_HBM_GBS, "hbm_target_frac": 0.6,
            "hbm_target_met": hbm / PEAK_HBM_GBS >= 0.6}


def class_sweep(bs, amrvac):
    """Autotune each size class of a block list whose faces are all fixed
    (so every class is a valid list on its own) and print the per-shape step
    times per class and summed over the classes."""
    import numpy as np
    if np.any(bs.nbr >= 0):
        print("bench: class sweep skipped (the list has block neighbours)", file=sys.stderr, flush=True)
        return
    total = {}
    best_sum = 0.0
    for size in sorted({int(n) for n in bs.n[:, 0]}, reverse=True):
        idx = [i for i in range(bs.nb) if int(bs.n[i, 0]) == size]
        sub = bs.copy()
        sub.u = [bs.u[i] for i in idx]
        sub.n, sub.dx, sub.xlo, sub.nbr = bs.n[idx], bs.dx[idx], bs.xlo[idx], bs.nbr[idx]
        ctx, flat, views = amrvac.context_for(sub, amrvac.EXEC_BATCHED)
        _, ms = ctx.autotune(amrvac.SSPRK54, 2)
        for name, m in zip(ctx.variants(), ms):
            if m >= 0:
                total[name] = total.get(name, 0.0) + m
                print(f"bench: class-sweep {size}^3 ({len(idx)} blocks) {name} {m:.3f} ms/step",
                      file=sys.stderr, flush=True)
        best_sum += min(m for m in ms if m >= 0)
        ctx.close()
        del flat, views
    for name, m in sorted(total.items(), key=lambda kv: kv[1]):
        print(f"bench: class-sweep sum {name} {m:.3f} ms/step", file=sys.stderr, flush=True)
    print(f"bench: class-sweep sum best-per-class {best_sum:.3f} ms/step", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--per-block-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-block", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--ckpt", type=int, default=5)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-warm", type=int, default=80,
                    help="forward steps before the timed adjoint window (3D MHD 256^3)")
    ap.add_argument("--ckpt-also", type=int, default=20,
                    help="also time the adjoint with this checkpoint interval (0: no)")
    ap.add_argument("--adjoint-2d-steps", type=int, default=200,
                    help="steps of the 2D Euler adjoint leg")
    ap.add_argument("--no-hall", action="store_true",
                    help="skip the Hall-MHD leg on the 256^3 periodic list")
    ap.add_argument("--no-glm", action="store_true",
                    help="skip the GLM-MHD leg on the same block list")
    ap.add_argument("--no-lim03", action="store_true",
                    help="skip the RK3 + LIM03 leg on the same block list")
    ap.add_argument("--no-mhd2d", action="store_true",
                    help="skip the 2D MHD 512^2 forward leg")
    ap.add_argument("--no-single", action="store_true",
                    help="skip timing the batched launch form that the headline does not use (both forms are "
                         "still autotuned to choose the headline's)")
    ap.add_argument("--class-sweep", action="store_true",
                    help="also run the autotuner on each block-size class of the uneven list on its own "
                         "(per-class tile-shape times on stderr)")
    ap.add_argument("--forward-leg", choices=sorted(FORWARD_LEGS),
                    help="run only the forward of this other list (autotune, warm-up, timed steps), for "
                         "profiling its stage kernel in a run of its own; prints one JSON line")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run one plain device-to-device copy of this many bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; multi-GPU runs (--gpus > 1) are not supported "
              "(blocks would be split into Morton ranges per GPU with face-halo exchange and a "
              "max all-reduce of c_max per stage, which is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1407_2052_amd import amrvac, inputs

    if args.forward_leg:
        torch.cuda.set_device(0)
        out = forward_leg(args.forward_leg, args.steps, args.warmup)
        if args.copy_probe > 0:
            a = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
            b = torch.empty_like(a)
            torch.cuda.synchronize()
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        print(json.dumps(out), flush=True)
        return

    print("bench: generating 3D MHD uneven block list (4096 blocks)", file=sys.stderr, flush=True)
    bs = inputs.uneven_3d()
    cells = bs.interior_cells()
    torch.cuda.set_device(0)
    ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED)
    stream = torch.cuda.current_stream()
    # the two batched launch forms (one launch per block-size class and stage,
    # or one per stage over the whole list), each with its autotuned tile
    # shape; the headline runs the faster pair, the other is timed beside it
    forms = {"per_class": amrvac.EXEC_BATCHED, "single": amrvac.EXEC_BATCHED_SINGLE}
    tuned = {}
    for fname, fexec in forms.items():
        print(f"bench: autotuning the tile shape ({fname} launches)", file=sys.stderr, flush=True)
        ctx.set_exec(fexec)
        fvar, fms = ctx.autotune(amrvac.SSPRK54, 2)
        for name, ms in zip(ctx.variants(), fms):
            if ms >= 0:
                print(f"bench: autotune {fname} {name} {ms:.3f} ms/step", file=sys.stderr, flush=True)
        tuned[fname] = (fvar, min(ms for ms in fms if ms >= 0))
    form = min(tuned, key=lambda f: tuned[f][1])
    other = "single" if form == "per_class" else "per_class"

    def use_form(f):
        ctx.set_exec(forms[f])
        ctx.set_variant(ctx.variants().index(tuned[f][0]))

    use_form(form)
    variant = tuned[form][0]

    if args.class_sweep:
        class_sweep(bs, amrvac)

    def timed(nsteps, warmup):
        if warmup:
            ctx.ssprk_step(amrvac.SSPRK54, warmup, cfl=0.4, t=None)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.ssprk_step(amrvac.SSPRK54, nsteps, cfl=0.4, t=None)
        e1.record(stream)
        torch.cuda.synchronize()
        ctx.sync()
        return e0.elapsed_time(e1) / 1e3

    print(f"bench: batched warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)
    el = timed(args.steps, args.warmup)
    value = cells * args.steps / el
    ms_per_step = 1e3 * el / args.steps
    stage_s = el / (args.steps * STAGES)   # average stage-launch duration (step control included)

    per_block = None
    if not args.no_per_block:
        # on the tile shape tuned for the per-class launches (small launches,
        # like the per-class ones, suit it better than the one-launch shape)
        print(f"bench: per-block launch, timed {args.per_block_steps}", file=sys.stderr, flush=True)
        use_form("per_class")
        ctx.set_exec(amrvac.EXEC_PER_BLOCK)
        elp = timed(args.per_block_steps, 1)
        per_block = {"value": cells * args.per_block_steps / elp, "ms_per_step": 1e3 * elp / args.per_block_steps,
                     "steps": args.per_block_steps, "tile_shape": tuned["per_class"][0]}
        use_form(form)

    # the other batched launch form with its own autotuned tile shape
    launch_forms = {f: {"tile_shape": tuned[f][0], "autotune_ms_per_step": tuned[f][1]} for f in forms}
    launch_forms[form].update({"ms_per_step": ms_per_step, "value": value, "unit": "cell-updates/s"})
    launch_forms["headline"] = form
    if not args.no_single:
        print(f"bench: batched, {other} launches", file=sys.stderr, flush=True)
        use_form(other)
        elo = timed(args.steps, args.warmup)
        launch_forms[other].update({"ms_per_step": 1e3 * elo / args.steps, "value": cells * args.steps / elo,
                                    "unit": "cell-updates/s"})
    ctx.close()
    del flat, views

    lim03 = None
    if not args.no_lim03:
        # the paper's other FD combination (RK3 + LIM03) on the same list
        print("bench: RK3 + LIM03 on the same block list", file=sys.stderr, flush=True)
        ctx, flat, views = amrvac.context_for(bs, amrvac.EXEC_BATCHED, recon=amrvac.LIM03)
        lvar, _ = ctx.autotune(amrvac.RK3, 2)
        ctx.ssprk_step(amrvac.RK3, args.warmup, cfl=0.4, t=None)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.ssprk_step(amrvac.RK3, args.steps, cfl=0.4, t=None)
        e1.record(stream)
        torch.cuda.synchronize()
        ctx.sync()
        ell = e0.elapsed_time(e1) / 1e3
        ctx.close()
        del flat, views
        lim03 = {"scheme": "RK3 + LIM03", "tile_shape": lvar, "steps": args.steps,
                 "ms_per_step": 1e3 * ell / args.steps, "cell_updates_per_s": cells * args.steps / ell,
                 "ssprk54_mp5_over_rk3_lim03_step_time": ms_per_step / (1e3 * ell / args.steps)}

    glm = None
    if not args.no_glm:
        # GLM-MHD (psi as a ninth variable) on the same list, psi = 0.01 sin(...)
        print("bench: GLM-MHD SSPRK(5,4) + MP5 on the same block list", file=sys.stderr, flush=True)
        gbs = inputs.as_glm(bs)
        for b in range(gbs.nb):
            P = gbs.u[b].shape[1:]
            x = gbs.xlo[b, 0] + (np.arange(P[2]) - 2.5) * gbs.dx[b, 0]
            gbs.u[b][8] = 0.01 * np.sin(2 * np.pi * x)[None, None, :]
        ctx, flat, views = amrvac.context_for(gbs, amrvac.EXEC_BATCHED)
        gvar, _ = ctx.autotune(amrvac.SSPRK54, 2)
        ctx.ssprk_step(amrvac.SSPRK54, args.warmup, cfl=0.4, t=None)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.ssprk_step(amrvac.SSPRK54, args.steps, cfl=0.4, t=None)
        e1.record(stream)
        torch.cuda.synchronize()
        ctx.sync()
        elg = e0.elapsed_time(e1) / 1e3
        ctx.close()
        del flat, views, gbs
        glm = {"scheme": "SSPRK(5,4) + MP5, GLM-MHD (9 variables)", "tile_shape": gvar, "steps": args.steps,
               "ms_per_step": 1e3 * elg / args.steps, "cell_updates_per_s": cells * args.steps / elg,
               "step_time_over_mhd": (1e3 * elg / args.steps) / ms_per_step}

    hall = None
    if not args.no_hall:
        # Hall MHD needs neighbours on every face: the 256^3 periodic list,
        # timed with eta_h = 0.01 and as ideal MHD
        print("bench: Hall MHD (eta_h = 0.01) and ideal MHD on the 256^3 periodic list", file=sys.stderr, flush=True)
        hbs = inputs.mhd_turbulence_3d()
        hcells = hbs.interior_cells()
        res = {}
        for eta in (0.01, 0.0):
            ctx, flat, views = amrvac.context_for(hbs, amrvac.EXEC_BATCHED, eta_h=eta)
            hvar, _ = ctx.autotune(amrvac.SSPRK54, 2)
            ctx.ssprk_step(amrvac.SSPRK54, args.warmup, cfl=0.4, t=None)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.ssprk_step(amrvac.SSPRK54, args.steps, cfl=0.4, t=None)
            e1.record(stream)
            torch.cuda.synchronize()
            ctx.sync()
            res[eta] = (e0.elapsed_time(e1) / args.steps, hvar)
            ctx.close()
            del flat, views
        del hbs
        hall = {"workload": "3D Hall MHD 256^3 periodic, 4096 x 16^3, eta_h = 0.01, SSPRK(5,4) + MP5",
                "tile_shape": res[0.01][1], "steps": args.steps, "ms_per_step": res[0.01][0],
                "cell_updates_per_s": hcells / (res[0.01][0] / 1e3),
                "ideal_mhd_ms_per_step": res[0.0][0], "step_time_over_ideal": res[0.01][0] / res[0.0][0]}

    if args.copy_probe > 0:
        # a plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of this
        # dispatch calibrate the counters against bytes really moved
        n = args.copy_probe // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    adjoint = adjoint_2d = None
    if not args.no_adjoint:
        adjoint = adjoint_ratio(args.adjoint_steps, args.ckpt, args.adjoint_warm,
                                args.ckpt_also if args.ckpt_also > 0 else None,
                                max(1, args.per_block_steps))
        adjoint_2d = adjoint_ratio_2d(args.adjoint_2d_steps)

    mhd2d = None
    if not args.no_mhd2d:
        print("bench: 2D MHD 512^2 forward", file=sys.stderr, flush=True)
        mhd2d = forward_mhd2d(args.steps, args.warmup)

    roofline = stage_roofline("mhd3d_uneven4096", cells, stage_s, BYTES_PER_CELL_STEP_MHD3D)
    roofline["traffic"] = measured_traffic(variant, form)
    roofline["kernel"] = f"k_stage<3,MHD> (fused SSPRK stage), {variant}, {form} launches"
    others = {}
    if adjoint:
        c5 = adjoint["forward_cell_updates_per_s"]
        others["mhd3d_periodic256_forward"] = stage_roofline(
            "mhd3d_periodic256", 16 ** 3 * 4096, 16 ** 3 * 4096 / c5 / STAGES, BYTES_PER_CELL_STEP_MHD3D)
        others["mhd3d_periodic256_forward"]["kernel"] = f"k_stage<3,MHD>, {adjoint['forward_tile_shape']}"
        others["mhd3d_periodic256_forward"]["traffic"] = measured_traffic_other(
            "mhd3d_periodic256", adjoint["forward_tile_shape"])
    if adjoint_2d:
        c4 = adjoint_2d["forward_cell_updates_per_s"]
        others["euler2d_256_forward"] = stage_roofline(
            "euler2d_256", 256 * 256, 256 * 256 / c4 / STAGES, BYTES_PER_CELL_STEP_EULER2D)
        others["euler2d_256_forward"]["kernel"] = f"k_stage<2,HD>, {adjoint_2d['forward_tile_shape']}"
        others["euler2d_256_forward"]["traffic"] = measured_traffic_other("euler2d_256", adjoint_2d["forward_tile_shape"])
    if mhd2d:
        others["mhd2d_512_forward"] = stage_roofline(
            "mhd2d_512", mhd2d["cells"], mhd2d["cells"] / mhd2d["cell_updates_per_s"] / STAGES,
            BYTES_PER_CELL_STEP_MHD3D)
        others["mhd2d_512_forward"]["kernel"] = f"k_stage<2,MHD>, {mhd2d['tile_shape']}"
        others["mhd2d_512_forward"]["traffic"] = measured_traffic_other("mhd2d_512", mhd2d["tile_shape"])

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(bs)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D ideal MHD, 4096 uneven blocks 32^3:16^3:8^3 (1:2:4), fixed ghosts "
                               "from a seeded 8-mode field, SSPRK(5,4)+MP5+global LF, CFL 0.4",
                   "blocks": bs.nb, "cells": cells,
                   "exec": ("batched persistent, one launch per block-size class and stage, steps replayed from HIP graphs"
                            if form == "per_class" else
                            "batched persistent, one launch per stage over the whole list, steps replayed from HIP graphs")
                           + " (the faster autotuned batched form)",
                   "tile_shape": variant,
                   "parallelism": "single GPU"},
        "per_stage": {"ms": 1e3 * stage_s, "cell_updates_per_s": cells / stage_s},
        "per_block": per_block,
        "batched_over_per_block": (value / per_block["value"]) if per_block else None,
        "batched_launch_forms": launch_forms,
        "adjoint_forward_ratio": adjoint["ratio"] if adjoint else None,
        "adjoint": adjoint,
        "adjoint_2d_euler": adjoint_2d,
        "mhd2d_512": mhd2d,
        "lim03": lim03,
        "glm": glm,
        "hall": hall,
        "roofline": roofline,
        "rooflines_other": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
