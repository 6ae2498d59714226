"""Benchmark: the D2Q9 finite-volume time step on one MI355X.

Headline workload: periodic Taylor-Green vortex on a 4096 x 4096 uniform mesh,
DUGKS, FP64 (the only single-GPU case whose 2.4 GB of traffic per step exceeds
the 256 MB Infinity Cache, so that HBM bandwidth is what is measured).  One
"step" is one full time step of the path (moments, equilibrium and collision
transforms, reconstruction and half-step trace at every face, wall / ghost
handling, interface moments and back-transform, flux divergence and update),
with the library's non-finite check every `--check-every` steps inside the timed
region.  Inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0): the metric and its value, the roofline of the timed kernel
(algorithmic and measured bytes), the variants and the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
HEADLINE_TILE = (205, 1)        # rows per block, waves per block of the timed 4096^2 step, and
HEADLINE_TIME_BLOCK = 4        # steps per launch (fixed so that the committed counter profile
                               # describes the same launches)
HEADLINE_PAIRS = 0             # two steps per launch: one wave (0) or a pair of waves (1) per item
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_dugks_fp64_taylor_green_4096.txt")
BYTES = {"f64": 144, "f32": 72, "bf16": 36, "f16": 36}   # algorithmic bytes per cell-step (9 reads + 9 writes)
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 (FMA) x 2.4 GHz
DUGKS_FLOP_PER_CELL_STEP = 600  # algorithmic FP operations of one DUGKS cell update (each face once)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=4096, help="mesh side of the headline workload")
    p.add_argument("--check-every", type=int, default=100)
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=6, help="oracle steps of the CPU baseline on all cores")
    p.add_argument("--cpu-steps-one", type=int, default=2, help="oracle steps of the CPU baseline on one thread")
    p.add_argument("--burn-in", type=float, default=0.5,
                   help="seconds of GPU burn-in on the headline workload before its warm-up")
    p.add_argument("--precision-steps", type=int, default=2000,
                   help="steps after which the reduced-precision forms report their velocity error")
    p.add_argument("--only", default="", help="comma list of variant names to run")
    p.add_argument("--tile", default="", help="rows,waves_per_block for every run (skips the autotuner)")
    p.add_argument("--batch-shape", default="",
                   help="time_block,rows,wave_per_item[,wave_pairs] (0/1) of the batch (skips its autotuner)")
    p.add_argument("--time-block", type=int, default=HEADLINE_TIME_BLOCK,
                   help="steps per launch with --tile on doubly periodic meshes (1 to 4)")
    p.add_argument("--pairs", type=int, default=HEADLINE_PAIRS,
                   help="with --tile and two steps per launch: a pair of waves per work item (1) or one (0)")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    p.add_argument("--cavity-residual", action="store_true",
                   help="instead of the throughput benchmark: run the 256^2 tanh cavity (Re 1000) toward "
                        "a steady state and report the residual history")
    p.add_argument("--stability-map", action="store_true",
                   help="instead of the throughput benchmark: the stable band of dt/tau against CFL for "
                        "the uniform 32^2 and 64^2 cavity, both schemes, one batch per scheme")
    p.add_argument("--map-steps", type=int, default=20000, help="steps after which a case counts as stable")
    p.add_argument("--boundary-layer-paper", action="store_true",
                   help="instead of the throughput benchmark: the flat plate of Sec. 3.3 on the paper's "
                        "meshes, both schemes, profiles against the Blasius solution")
    p.add_argument("--flow-throughs", type=float, default=4.0, help="run length of the flat plate, in L / U0")
    p.add_argument("--scheme", default="dugks", choices=["dugks", "bkg"])
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    p.add_argument("--target", type=float, default=1e-8, help="residual target (per 1000 steps)")
    p.add_argument("--budget-s", type=float, default=600.0, help="wall-time budget of the residual run")
    p.add_argument("--beta", type=float, default=0.0,
                   help="tanh parameter of the cavity mesh (0: largest adjacent ratio 1.05)")
    p.add_argument("--save", default="", help="save the final f~ (npy) of the residual run")
    p.add_argument("--resume", default="", help="start the residual run from a saved f~ (npy)")
    p.add_argument("--start-step", type=int, default=0, help="step count of the resumed state")
    return p.parse_args()


def burn_in(ctx, scheme, seconds, stream):
    """Step the workload until `seconds` of wall time have passed (synchronised every few
    steps), so that the timed region does not start on a GPU still clocking up after the
    host-side setup.  Returns the wall time spent and the steps taken."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        ctx.step(scheme, 8)
        torch.cuda.synchronize()
        n += 8
    return time.perf_counter() - t0, n


def trial_steps_for(ctx, scheme, stream, target_ms=20.0, cap=4000):
    """Trial length of the autotuner: enough steps that one trial lasts about `target_ms`
    at the current launch shape (short trials make the choice noisy)."""
    import torch
    ctx.step(scheme, 4)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.step(scheme, 16)
    e1.record(stream)
    torch.cuda.synchronize()
    per = max(e0.elapsed_time(e1) / 16, 1e-4)
    return int(min(cap, max(16, math.ceil(target_ms / per))))


def timed_steps(ctx, scheme, steps, warmup, stream):
    """Warm up, then time `steps` steps with HIP events on the library's stream."""
    import torch
    ctx.step(scheme, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(scheme, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall * 1e3


def run_single(name, w, scheme, compute, storage, steps, warmup, check_every, stream, tile=None,
               time_block=1, burn_s=0.0, pairs=0):
    """Time `steps` steps of one workload; a fixed launch shape, or the autotuner's choice
    of shape and time block (one or two steps per launch).
    burn_s: wall time of GPU burn-in right before the warm-up (stepping the workload, whose
    state then carries on into the timed steps)."""
    from paper_1511_00242_amd import lbfv as L
    ctx = L.Context(w.xf, w.yf, w.tau, w.dt, rt=w.rt, bcs=w.bcs, compute=compute, storage=storage,
                    check_every=check_every, stream=stream.cuda_stream)
    ctx.bind_torch_buffers()
    ctx.init_equilibrium(w.rho, w.ux, w.uy)
    tune = None
    if tile:
        ctx.set_time_block(time_block)
        ctx.set_tile(*tile)
        ctx.set_wave_pairs(pairs)
    else:
        trial = trial_steps_for(ctx, scheme, stream)
        ctx.autotune(scheme, trial, os.environ.get("LBFV_TUNE_CACHE"))
        tune = {"trial_steps": trial}
    burn = None
    if burn_s > 0:
        # straight into the warm-up and the timed steps: an idle gap (a re-initialisation,
        # say) would let the clock drop again
        sec, n = burn_in(ctx, scheme, burn_s, stream)
        burn = {"seconds": round(sec, 3), "steps": n}
    ms, wall_ms = timed_steps(ctx, scheme, steps, warmup, stream)
    rows, wpb = ctx.get_tile()
    tb = ctx.get_time_block()
    pr = ctx.get_wave_pairs()
    tot = ctx.totals()                       # also re-checks for non-finite values
    ctx.close()
    cells = w.nx * w.ny
    per = ms / steps
    out = dict(name=name, ms_per_step=per, mlups=cells / (per * 1e-3) / 1e6, wall_ms=wall_ms,
               tile=[rows, wpb], time_block=tb, wave_pairs=int(pr), mass=tot[0])
    if tune:
        out["autotune"] = tune
    if burn:
        out["burn_in"] = burn
    return out


def run_batch(steps, warmup, stream, shape=""):
    import torch
    from paper_1511_00242_amd import inputs as I
    from paper_1511_00242_amd import lbfv as L
    cases = I.batch_cases()
    b = L.Batch(cases, stream=stream.cuda_stream)
    for i, w in enumerate(cases):
        b.init_equilibrium(i, w.rho, w.ux, w.uy)
    if shape:
        parts = [int(x) for x in shape.split(",")]
        tb, rows, per_item = parts[:3]
        b.set_time_block(tb)
        b.set_shape(rows=rows)
        b.set_grid_form(per_item)
        b.set_wave_pairs(parts[3] if len(parts) > 3 else 0)
    else:
        b.autotune(L.LBFV_DUGKS, 20)          # time block, row-block height, grid (state kept)
    graph_steps, rows = b.get_shape()
    tb = b.get_time_block()
    per_item = b.get_grid_form()
    pairs = b.get_wave_pairs()
    cells, items = b.info()
    b.step(L.LBFV_DUGKS, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(L.LBFV_DUGKS, steps)             # `steps` is a multiple of the steps of one graph
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b.close()
    # the same cases stepped one at a time: the plain FP64 kernel, and the FP32 deviation kernel
    t_seq = {}
    for label, compute, storage in (("fp64", L.LBFV_FP64, L.LBFV_STORE_NATIVE),
                                    ("fp32dev", L.LBFV_FP32, L.LBFV_STORE_DEV_FP32)):
        t_seq[label] = 0.0
        for w in cases:
            ctx = L.Context(w.xf, w.yf, w.tau, w.dt, bcs=w.bcs, compute=compute, storage=storage,
                            check_every=0, stream=stream.cuda_stream)
            ctx.init_equilibrium(w.rho, w.ux, w.uy)
            ctx.dugks_step(4)
            torch.cuda.synchronize()
            e0.record(stream)
            ctx.dugks_step(32)
            e1.record(stream)
            torch.cuda.synchronize()
            t_seq[label] += e0.elapsed_time(e1) / 32
            ctx.close()
    return dict(name="batch96_dugks_fp32dev", cases=len(cases), cells=cells, work_items=items, rows=rows,
                graph_launches=graph_steps, time_block=tb, wave_pairs=int(pairs),
                grid="wave_per_item" if per_item else "resident_waves",
                ms_per_step=ms, mlups=cells / (ms * 1e-3) / 1e6, alg_gbs=cells * BYTES["f32"] / (ms * 1e-3) / 1e9,
                alg_frac_of_hbm_peak=cells * BYTES["f32"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                seq_fp64_ms_per_step=t_seq["fp64"], speedup_vs_seq_fp64=t_seq["fp64"] / ms,
                seq_fp32dev_ms_per_step=t_seq["fp32dev"], speedup_vs_seq_fp32dev=t_seq["fp32dev"] / ms)


def cavity_residual(a, stream):
    """Config 1: lid-driven cavity 256^2 on the tanh mesh, U_lid 0.1, Re 1000, from rest,
    advanced in chunks of 1000 steps until ||u - u_prev|| / ||u|| over a chunk falls below
    the target or the wall-time budget is spent."""
    import torch
    from paper_1511_00242_amd import inputs as I
    from paper_1511_00242_amd import lbfv as L
    w = I.cavity(256)
    if a.beta > 0:
        w.xf = I.tanh_faces(256, a.beta)
        w.yf = w.xf.copy()
        w.dt = I.cfl_dt(w.xf, w.yf, 0.5)
    scheme = L.LBFV_DUGKS if a.scheme == "dugks" else L.LBFV_BKG
    comp, sto = (L.LBFV_FP64, L.LBFV_STORE_NATIVE) if a.precision == "fp64" else (L.LBFV_FP32, L.LBFV_STORE_DEV_FP32)
    ctx = L.Context(w.xf, w.yf, w.tau, w.dt, bcs=w.bcs, compute=comp, storage=sto, check_every=1000,
                    stream=stream.cuda_stream)
    if a.resume:
        ctx.set_f(np.load(a.resume))
    else:
        ctx.init_equilibrium(w.rho, w.ux, w.uy)
    ctx.autotune(scheme, 200)
    m0 = ctx.totals()[0]
    ctx.residual()
    steps, hist, res = a.start_step, [], 1.0
    t0 = time.perf_counter()
    gpu_ms = 0.0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    while time.perf_counter() - t0 < a.budget_s:
        e0.record(stream)
        ctx.step(scheme, 1000 * 50)
        e1.record(stream)
        torch.cuda.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        # the residual is defined over one 1000-step chunk: take it from the last chunk
        ctx.residual()
        ctx.step(scheme, 1000)
        res = ctx.residual()
        steps += 51000
        hist.append((steps, res))
        print(f"[cavity] step {steps} residual {res:.3e} ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)
        if res < a.target:
            break
    m1 = ctx.totals()[0]
    if a.save:
        np.save(a.save, ctx.get_f())
    rows, wpb = ctx.get_tile()
    tb, pairs = ctx.get_time_block(), ctx.get_wave_pairs()
    ctx.close()
    cells = 256 * 256
    return {"workload": "cavity_256x256_tanh_re1000", "scheme": a.scheme, "precision": a.precision,
            "mesh_beta": a.beta or I.tanh_beta_for_ratio(256, 1.05), "dt": w.dt, "tau": w.tau,
            "steps": steps, "lid_transits": steps * w.dt * 0.1, "residual": res, "target": a.target,
            "reached": res < a.target, "gpu_s": gpu_ms / 1e3,
            "mlups": cells * 50000 * len(hist) / (gpu_ms * 1e-3) / 1e6 if gpu_ms else None,
            "mass_rel_drift": abs(m1 - m0) / m0, "tile": [rows, wpb], "time_block": tb, "wave_pairs": int(pairs),
            "history": [[s_, r_] for s_, r_ in hist[:: max(1, len(hist) // 40)]] + [[steps, res]]}


def stability_map(a, stream):
    """Stable range of the lid-driven cavity (Sec. 3.2, uniform N x N meshes, U_w = 0.1, L = 1)
    over CFL and dt/tau: every (N, CFL, dt/tau) point is one case of an FP64 batch, advanced
    from rest for `map_steps` steps; a case is unstable if any cell then holds a non-finite
    value.  For each (scheme, N, CFL) the band of dt/tau over which the grid points are
    stable is reported (the longest run of stable points), with the whole row of flags."""
    import torch
    from paper_1511_00242_amd import inputs as I
    from paper_1511_00242_amd import lbfv as L
    sizes = (32, 64)
    cfls = [round(0.1 * k, 1) for k in range(1, 13)]
    ratios = [float(r) for r in np.geomspace(0.1, 1000.0, 41)]
    grid = [(n, c, r) for n in sizes for c in cfls for r in ratios]
    out = {"workload": "cavity_uniform_stability_map", "sizes": list(sizes), "cfl": cfls,
           "dt_over_tau": ratios, "steps": a.map_steps, "precision": "fp64", "schemes": {}}
    t0 = time.perf_counter()
    for sname, scheme in (("dugks", L.LBFV_DUGKS), ("bkg", L.LBFV_BKG)):
        cases = []
        for n, cfl, r in grid:
            xf = I.uniform_faces(n)
            dt = I.cfl_dt(xf, xf, cfl)
            z = np.zeros((n, n))
            cases.append(I.Workload(f"cavity_{n}_cfl{cfl}_r{r:.3g}", xf, xf.copy(), dt / r, dt,
                                    [("wall", 0.0, 0.0), ("wall", 0.0, 0.0), ("wall", 0.0, 0.0),
                                     ("wall", 0.1, 0.0)], z + 1.0, z, z.copy()))
        b = L.Batch(cases, compute=L.LBFV_FP64, storage=L.LBFV_STORE_NATIVE, stream=stream.cuda_stream)
        for i, w in enumerate(cases):
            b.init_equilibrium(i, w.rho, w.ux, w.uy)
        done = 0
        while done < a.map_steps:
            k = min(5000, a.map_steps - done)
            b.step(scheme, k)
            torch.cuda.synchronize()
            done += k
            print(f"[stability] {sname}: {done}/{a.map_steps} steps ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        bad = b.nonfinite()
        b.close()
        table = {}
        for n in sizes:
            for cfl in cfls:
                flags = [bool(bad[grid.index((n, cfl, r))] == 0) for r in ratios]
                # the longest run of stable grid points: the stable band of dt/tau
                best, start = (0, 0), None
                for k, ok in enumerate(flags + [False]):
                    if ok and start is None:
                        start = k
                    if not ok and start is not None:
                        if k - start > best[1] - best[0]:
                            best = (start, k)
                        start = None
                band = [ratios[best[0]], ratios[best[1] - 1]] if best[1] > best[0] else None
                table[f"N{n}_cfl{cfl}"] = {"stable_dt_over_tau": band,
                                           "stable": "".join("s" if f else "u" for f in flags)}
        out["schemes"][sname] = table
    out["wall_s"] = time.perf_counter() - t0
    return out


def boundary_layer_paper(a, stream):
    """Sec. 3.3: laminar flat plate at Re_L = 1e5 on the paper's meshes (dy_min 0.1, 0.05,
    0.02; CFL 0.5), DUGKS and BKG in FP64 from the uniform free stream for a fixed number
    of flow-through times; u / U0 and v / (U0 / (2 sqrt(Re_x))) at the two stations of the
    paper against the Blasius solution at the cell centres with eta <= 8."""
    import torch
    from paper_1511_00242_amd import inputs as I
    from paper_1511_00242_amd import lbfv as L
    eta_b, u_b, v_b, _ = I.blasius()
    out = {"workload": "flat_plate_paper_mesh_re1e5", "flow_throughs": a.flow_throughs, "cases": {}}
    t0 = time.perf_counter()
    for dy in (0.1, 0.05, 0.02):
        w = I.boundary_layer_paper(dy)
        steps = int(round(a.flow_throughs * w.meta["length"] / w.meta["u0"] / w.dt))
        for sname, scheme in (("dugks", L.LBFV_DUGKS), ("bkg", L.LBFV_BKG)):
            ctx = L.Context(w.xf, w.yf, w.tau, w.dt, bcs=w.bcs, check_every=10000, stream=stream.cuda_stream)
            ctx.init_equilibrium(w.rho, w.ux, w.uy)
            ctx.step(scheme, steps - 1000)
            ctx.residual()
            ctx.step(scheme, 1000)
            res = ctx.residual()
            _, ux, uy = ctx.moments()
            ctx.close()
            yc = 0.5 * (w.yf[1:] + w.yf[:-1])
            xc = 0.5 * (w.xf[1:] + w.xf[:-1])
            case = {"steps": steps, "dt_over_tau": w.dt / w.tau, "residual_per_1000": res,
                    "cells": [w.nx, w.ny]}
            for st, i in (("x1", 40 + 29), ("x2", 40 + 50)):
                x = xc[i]
                eta = yc * math.sqrt(w.meta["u0"] / (w.meta["nu"] * x))
                vs = w.meta["u0"] / (2.0 * math.sqrt(w.meta["u0"] * x / w.meta["nu"]))
                m = eta <= 8.0
                du = ux[m, i] / w.meta["u0"] - np.interp(eta[m], eta_b, u_b)
                dv = uy[m, i] / vs - np.interp(eta[m], eta_b, v_b)
                case[st] = {"x": x, "cells_in_eta8": int(m.sum()),
                            "cells_in_layer": int((eta <= 4.91).sum()),
                            "u_rms_err": float(np.sqrt(np.mean(du ** 2))), "u_max_err": float(np.max(np.abs(du))),
                            "v_rms_err": float(np.sqrt(np.mean(dv ** 2))), "v_max_err": float(np.max(np.abs(dv)))}
            out["cases"][f"{sname}_dy{dy:g}"] = case
            print(f"[flat plate] {sname} dy_min {dy}: {steps} steps, residual {res:.2e}, "
                  f"u rms err x1 {case['x1']['u_rms_err']:.4f} x2 {case['x2']['u_rms_err']:.4f} "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    return out


HEADLINE_KERNEL = "_ZN4lbfv12stepc_kernelIddLi0ELb0ELi4EEEvNS_10StepParamsIT_EEiiii"   # stepc_kernel<double,double,DUGKS,4>


def kernel_isa_hash():
    """sha256 of the headline kernel's machine code and kernel descriptor in the loaded
    library: a counter profile stays valid exactly as long as the binary kernel it measured."""
    from paper_1511_00242_amd import codeobj
    from paper_1511_00242_amd import lbfv as L
    return codeobj.kernel_isa_sha256(L._LIB_PATH, HEADLINE_KERNEL)


def profiled_traffic(tile, time_block, ms_per_step, pairs=0):
    """HBM traffic of the headline kernel from the committed rocprofv3 counter summary:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same counters read for a
    plain 1 GiB device copy.  None when the kernel's machine code or the launch shape changed
    since."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None, None
    kv = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        isa = kernel_isa_hash()
        if (isa is None or kv.get("kernel_isa_sha256") != isa or kv.get("tile") != f"{tile[0]},{tile[1]}"
                or kv.get("time_block", "1") != str(time_block) or kv.get("wave_pairs", "0") != str(pairs)):
            return None, None
        b = (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
             + float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])) * 1024.0
    except (KeyError, ValueError):
        return None, None
    # one dispatch advances `time_block` steps
    return b / (time_block * ms_per_step * 1e-3) / 1e9, b


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, steps_all, steps_one):
    """The FP64 oracle as it stands, on the host's cores, over a bounded sample of the
    workload: both schemes, on all the cores this process may use and on one thread.
    `value` is DUGKS on all cores (the headline's scheme)."""
    from oracle import oracle as O
    from paper_1511_00242_amd import inputs as I
    nproc = os.cpu_count() or 1
    # the cores this process may use: its affinity mask, capped by OMP_NUM_THREADS where the
    # host sets one (a shared host grants each job a share of its cores that way)
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    threads = max(1, min(allowed, int(os.environ.get("OMP_NUM_THREADS", allowed))))
    w = I.taylor_green(n)
    legs = {}
    total = 0.0
    for sname, scheme in (("dugks", O.DUGKS), ("bkg", O.BKG)):
        for th, steps in ((threads, steps_all), (1, steps_one)):
            c = O.Case(w.xf, w.yf, w.rt, w.tau, w.dt, w.bcs, threads=th)
            f = c.init_equilibrium(w.rho, w.ux, w.uy)
            t0 = time.perf_counter()
            c.run(f, scheme, steps)
            el = time.perf_counter() - t0
            total += el
            legs[f"{sname}_{th}_threads"] = {"mlups": n * n * steps / el / 1e6, "threads": th, "steps": steps,
                                             "seconds": round(el, 2)}
            print(f"[bench] cpu oracle {sname} {th} threads: {n * n * steps / el / 1e6:.2f} MLUPS ({el:.1f} s)",
                  file=sys.stderr, flush=True)
    head = legs[f"dugks_{threads}_threads"]
    return {"value": head["mlups"], "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": (f"taylor_green {n}x{n} FP64, DUGKS and BKG: {steps_all} steps on {threads} threads, "
                       f"{steps_one} steps on 1 thread ({total:.1f} s in all)"),
            "nproc": nproc, "affinity_cpus": allowed, "cpu_model": cpu_model(), "legs": legs}


def read_oracle_fixture(path):
    """(cells [(j, i)], f~ [9, n]) of a long-horizon fixture written by the oracle alone
    (tests/golden/make_long_horizon.py); None if it is not there."""
    if not os.path.exists(path):
        return None
    cells, vals = [], []
    for line in open(path):
        p = line.split()
        if not p or p[0].startswith("#") or p[0] in ("steps", "totals", "ext"):
            continue
        cells.append((int(p[0]), int(p[1])))
        vals.append([float(v) for v in p[2:]])
    return cells, np.array(vals).T


EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)   # D2Q9 unit directions, Sec. 2.1
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)


def precision_errors(w, runs, stream, n=2000):
    """The precision workload's accuracy at its parity point: every form advanced `n` steps
    from the initial state at the launch shape its timing run used; u against the GPU FP64
    run of the same scheme over every cell, and against the oracle at the cells of its
    long-horizon fixture (c = 1 at RT = 1/3, so u = sum e f / sum f).  Returns
    {name: {...}} for the reduced-precision forms."""
    from paper_1511_00242_amd import lbfv as L
    fields = {}
    for name, sch, comp, sto, tile, tb in runs:
        ctx = L.Context(w.xf, w.yf, w.tau, w.dt, rt=w.rt, bcs=w.bcs, compute=comp, storage=sto,
                        check_every=0, stream=stream.cuda_stream)
        ctx.init_equilibrium(w.rho, w.ux, w.uy)
        ctx.set_time_block(tb)
        ctx.set_tile(*tile)
        ctx.step(sch, n)
        _, ux, uy = ctx.moments()
        ctx.close()
        fields[name] = (sch, comp, np.stack([ux, uy]))
    out = {}
    for name, (sch, comp, u) in fields.items():
        if comp == L.LBFV_FP64:
            continue
        ref = next(v[2] for v in fields.values() if v[0] == sch and v[1] == L.LBFV_FP64)
        d = u - ref
        e = {"steps": n, "u_rel_l2_vs_gpu_fp64": float(np.linalg.norm(d) / np.linalg.norm(ref)),
             "u_max_vs_gpu_fp64": float(np.max(np.abs(d)) / np.max(np.abs(ref)))}
        fx = read_oracle_fixture(os.path.join(ROOT, "tests", "golden",
                                              f"long_tg{w.nx}_{'dugks' if sch == L.LBFV_DUGKS else 'bkg'}.txt"))
        if fx is not None:
            cells, f9 = fx
            rho = f9.sum(axis=0)
            uo = np.stack([EX @ f9 / rho, EY @ f9 / rho])
            jj = np.array([c[0] for c in cells]); ii = np.array([c[1] for c in cells])
            ug = u[:, jj, ii]
            e["u_rel_l2_vs_oracle_sampled"] = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
            e["u_max_vs_oracle_sampled"] = float(np.max(np.abs(ug - uo)) / np.max(np.abs(uo)))
            e["oracle_cells"] = len(cells)
        out[name] = e
        print(f"[bench] {name} after {n} steps: u vs GPU FP64 {e['u_rel_l2_vs_gpu_fp64']:.2e}"
              + (f", vs oracle ({e['oracle_cells']} cells) {e['u_rel_l2_vs_oracle_sampled']:.2e}"
                 if "oracle_cells" in e else ""), file=sys.stderr, flush=True)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_1511_00242_amd import inputs as I
    from paper_1511_00242_amd import lbfv as L
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.stability_map:
        print(json.dumps(stability_map(a, stream)), flush=True)
        return
    if a.boundary_layer_paper:
        print(json.dumps(boundary_layer_paper(a, stream)), flush=True)
        return
    if a.cavity_residual:
        print(json.dumps(cavity_residual(a, stream)), flush=True)
        return
    steps = max(2, a.steps)
    tile = tuple(int(x) for x in a.tile.split(",")) if a.tile else None
    if a.copy_probe_mb:
        n = a.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 3 copies of {a.copy_probe_mb} MiB", file=sys.stderr, flush=True)
        del src, dst

    w = I.taylor_green(a.n)
    head = run_single("dugks_fp64", w, L.LBFV_DUGKS, L.LBFV_FP64, L.LBFV_STORE_NATIVE, steps, a.warmup,
                      a.check_every, stream, tile or HEADLINE_TILE, a.time_block if tile else HEADLINE_TIME_BLOCK,
                      burn_s=a.burn_in, pairs=a.pairs if tile else HEADLINE_PAIRS)
    print(f"[bench] dugks fp64 {a.n}^2: {head['ms_per_step']:.4f} ms/step {head['mlups']:.0f} MLUPS",
          file=sys.stderr, flush=True)
    # the roofline figure divides by the step kernel's own average duration: the same launches
    # without the periodic check reductions
    kern = run_single("dugks_fp64_kernel", w, L.LBFV_DUGKS, L.LBFV_FP64, L.LBFV_STORE_NATIVE, steps,
                      a.warmup, 0, stream, tuple(head["tile"]), head["time_block"], pairs=head["wave_pairs"],
                      burn_s=a.burn_in)
    cells = w.nx * w.ny
    gbs = cells * BYTES["f64"] / (kern["ms_per_step"] * 1e-3) / 1e9
    traffic_gbs, traffic_bytes = profiled_traffic(head["tile"], head["time_block"], kern["ms_per_step"],
                                                  head["wave_pairs"])

    variants = {}
    if not a.no_variants:
        only = set(x for x in a.only.split(",") if x)
        specs = [("bkg_fp64", L.LBFV_BKG, L.LBFV_FP64, L.LBFV_STORE_NATIVE, "f64"),
                 ("dugks_fp32dev", L.LBFV_DUGKS, L.LBFV_FP32, L.LBFV_STORE_DEV_FP32, "f32"),
                 ("bkg_fp32dev", L.LBFV_BKG, L.LBFV_FP32, L.LBFV_STORE_DEV_FP32, "f32"),
                 ("dugks_bf16dev", L.LBFV_DUGKS, L.LBFV_FP32, L.LBFV_STORE_DEV_BF16, "bf16"),
                 ("dugks_fp16dev", L.LBFV_DUGKS, L.LBFV_FP32, L.LBFV_STORE_DEV_FP16, "f16")]
        for name, sch, comp, sto, dt in specs:
            if only and name not in only:
                continue
            r = run_single(name, w, sch, comp, sto, steps, a.warmup, a.check_every, stream, tile, a.time_block,
                           pairs=a.pairs)
            # bytes the method defines per step over the time per step; with two steps per
            # launch the state is read and written once per two steps, so this can pass the
            # HBM peak
            r["alg_gbs"] = cells * BYTES[dt] / (r["ms_per_step"] * 1e-3) / 1e9
            r["alg_frac_of_hbm_peak"] = r["alg_gbs"] / HBM_PEAK_GBS
            r["speedup_vs_dugks_fp64"] = head["ms_per_step"] / r["ms_per_step"]
            if sch == L.LBFV_BKG and "bkg_fp64" in variants:
                r["speedup_vs_same_scheme_fp64"] = variants["bkg_fp64"]["ms_per_step"] / r["ms_per_step"]
            elif sch == L.LBFV_DUGKS:
                r["speedup_vs_same_scheme_fp64"] = head["ms_per_step"] / r["ms_per_step"]
            variants[name] = r
            print(f"[bench] {name}: {r['ms_per_step']:.4f} ms/step {r['mlups']:.0f} MLUPS", file=sys.stderr,
                  flush=True)
        # accuracy of the reduced-precision forms at the precision workload's parity point
        if a.precision_steps > 0 and any(k in variants for k, *_ in specs[1:]):
            runs = [("dugks_fp64", L.LBFV_DUGKS, L.LBFV_FP64, L.LBFV_STORE_NATIVE, head["tile"], head["time_block"])]
            for name, sch, comp, sto, _ in specs:
                if name in variants:
                    runs.append((name, sch, comp, sto, variants[name]["tile"], variants[name]["time_block"]))
            if "bkg_fp64" not in variants and "bkg_fp32dev" in variants:
                runs.append(("bkg_fp64", L.LBFV_BKG, L.LBFV_FP64, L.LBFV_STORE_NATIVE, [0, 0], 1))
            for name, e in precision_errors(w, runs, stream, a.precision_steps).items():
                variants[name]["accuracy"] = e
        # the smaller workloads (L2 / Infinity-Cache resident, launch bound): MLUPS only
        small = [("tg32_dugks_fp64", I.taylor_green(32), L.LBFV_DUGKS),
                 ("cavity256_dugks_fp64", I.cavity(256), L.LBFV_DUGKS),
                 ("cavity256_bkg_fp64", I.cavity(256), L.LBFV_BKG),
                 ("bl512x256_dugks_fp64", I.boundary_layer(), L.LBFV_DUGKS),
                 ("bl512x256_bkg_fp64", I.boundary_layer(), L.LBFV_BKG)]
        for name, ws, sch in small:
            if only and name not in only:
                continue
            # microseconds per step: at least 2000 timed steps (tens of milliseconds)
            r = run_single(name, ws, sch, L.LBFV_FP64, L.LBFV_STORE_NATIVE, max(10 * steps, 2000),
                           max(a.warmup, 200), a.check_every * 10, stream, tile, a.time_block, pairs=a.pairs)
            variants[name] = r
            print(f"[bench] {name}: {r['ms_per_step'] * 1e3:.2f} us/step {r['mlups']:.0f} MLUPS", file=sys.stderr,
                  flush=True)
        if not only or "batch" in only:
            r = run_batch(200, 200, stream, a.batch_shape)
            variants["batch"] = r
            print(f"[bench] batch: {r['ms_per_step']:.4f} ms/step {r['mlups']:.0f} MLUPS", file=sys.stderr,
                  flush=True)
        if "bkg_fp64" in variants:
            variants["dugks_over_bkg_cost_fp64"] = head["ms_per_step"] / variants["bkg_fp64"]["ms_per_step"]

    out = {
        "metric": "MLUPS and % HBM peak per step (DUGKS, BKG; FP64 vs FP32/batched)",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic Taylor-Green field, no dataset)",
        "config": {"workload": f"taylor_green_{a.n}x{a.n}_dugks_fp64", "nx": a.n, "ny": a.n,
                   "scheme": "dugks", "precision": "fp64", "boundary": "periodic",
                   "check_every": a.check_every, "tile_rows_waves": head["tile"],
                   "steps_per_launch": head["time_block"], "wave_pairs": head["wave_pairs"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic_gbs,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "traffic_frac": traffic_gbs / HBM_PEAK_GBS if traffic_gbs else None,
                     "limiter": ("vector ALU and power: the state crosses HBM once per launch of "
                                 f"{head['time_block']} steps" if head["time_block"] > 1 else "HBM"),
                     "kernel": (f"lbfv::stepc_kernel<double,double,DUGKS,{head['time_block']}>" if head["time_block"] >= 3
                                else ("lbfv::step2p_kernel<double,double,DUGKS>" if head["wave_pairs"]
                                      else "lbfv::step2_kernel<double,double,DUGKS>") if head["time_block"] == 2
                                else "lbfv::step_kernel<double,double,DUGKS>"),
                     "steps_per_launch": head["time_block"],
                     "kernel_ms": kern["ms_per_step"],
                     "alu": {"achieved": cells * DUGKS_FLOP_PER_CELL_STEP / (kern["ms_per_step"] * 1e-3) / 1e12,
                             "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": cells * DUGKS_FLOP_PER_CELL_STEP / (kern["ms_per_step"] * 1e-3) / 1e12
                             / FP64_VECTOR_PEAK_TFLOPS,
                             "flop_per_cell_step": DUGKS_FLOP_PER_CELL_STEP},
                     "bytes_per_cell_step": BYTES["f64"]},
        "burn_in": head.get("burn_in"),
        "variants": variants,
        "context": {"paper_cpu_mlups_64x64": {"dugks": 2.08, "bkg": 3.90,
                                              "hardware": "Xeon E5-2670v3 (paper Sec. 3.1)"}},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.n, a.cpu_steps, a.cpu_steps_one)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
