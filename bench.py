"""Throughput of the fused cascaded double-distribution LBM step on one MI355X.

Workload: the differentially heated 512^3 cavity at Ra = 1e6, Pr = 0.71,
u0 = 0.05, D3Q15 flow + D3Q7 scalar, FP32 arithmetic, distributions stored in
FP32 (headline) and in shifted FP16 (second line of the same record),
started from rest.  One step = one launch of the fused stream-collide kernel
over all cells (pull streaming, walls, Boussinesq coupling, both cascaded
collisions, store).

Prints one JSON line.  `value` is whole-job MLUPS (million lattice-cell
updates per second) with the state resident in HBM; `roofline` relates the
step kernel's algorithmic bytes per launch ((15 + 7) values read and written
per cell) to its average launch time measured with HIP events on the stream
the kernel runs on; `cpu_baseline` times the CPU oracle on a bounded sample
of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled flow+thermal MLUPS & % HBM roofline; steps-to-steady learned vs plain"
HBM_PEAK_GBS = 8000.0
# uniform scalar source of the heat-source line (lattice units per cell and
# step); it selects the general collision kernels
SOURCE_R = 1e-6


def recorded_traffic(n, precision):
    """HBM bytes per launch of the step kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs recorded under profiles/ (scaled by the copy-probe
    calibration), or None when the workload differs or the kernel sources
    have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "step_traffic_cavity512.json")
    if n != 512 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, "paper_1710_04751_amd", "csrc", f), "rb").read()
                   for f in ("lbm_device.hpp", "lbm_index.hpp", "lbm_step.hpp", "lbm_step.hip"))
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    entry = rec.get(precision)
    return None if entry is None else round(entry["traffic_bytes"])


def algorithmic_bytes_per_cell(precision, qt=7):
    vb = {"fp32": 4, "fp16": 2, "fp64": 8}[precision]
    return 2 * (15 + qt) * vb


def time_variant(n, ra, precision, steps, warmup, block=None, log=print, R=0.0, sr=0, qt=7,
                 shape=None):
    """Time the step on an n^3 cavity, or on an nx x ny x nz box when shape
    is given (the lattice parameters of the n^3 cavity either way)."""
    import torch
    from paper_1710_04751_amd import solver as S

    stream = torch.cuda.Stream()
    params = S.make_params(n, ra, precision=precision, R=R, round_stochastic=sr, thermal_q=qt)
    if shape:
        params.nx, params.ny, params.nz = shape
    if block:
        params.block_x, params.block_y = block
    cav = S.Cavity(params, stream=stream)
    kname = cav.kernel_name()
    if block:
        chosen = list(block)
    else:  # block shape chosen by the library's autotuner (its trial steps are warm-up)
        chosen = list(cav.autotune(steps_per_trial=20))
        log(f"  {precision}: autotuned block {chosen[0]}x{chosen[1]}")
    cav.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    done = 0
    chunk = max(1, min(steps, 2000))
    while done < steps:
        k = min(chunk, steps - done)
        cav.step(k)
        done += k
        if done < steps:
            stream.synchronize()  # progress line; the gap is one launch latency
            log(f"  {precision}: {done}/{steps} steps")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # sanity of the state after the timed region
    status, _ = cav.residual()
    s2, dT = cav.residual()
    nu = cav.nusselt()
    ncell = params.nx * params.ny * params.nz
    launch_ms = ms / steps
    mlups = ncell * steps / (ms * 1e-3) / 1e6
    bpc = algorithmic_bytes_per_cell(precision, qt)
    achieved = bpc * ncell / (launch_ms * 1e-3) / 1e9
    out = {
        "precision": precision, "kernel": kname, "steps": steps, "warmup": warmup,
        "ms_per_step": launch_ms, "wall_s": wall, "mlups": mlups,
        "bytes_per_cell_update": bpc, "achieved_GBs": achieved,
        "frac_hbm_peak": achieved / HBM_PEAK_GBS, "finite": status == 0,
        "nu_hot_wall": nu.nu_hot_wall, "block": chosen,
    }
    cav.close()
    del cav
    torch.cuda.empty_cache()
    return out


def copy_calibration(nbytes=4 << 30, reps=5, log=print):
    """Plain device copy of a known size (the library's copy probe): the
    reference for bandwidth and for scaling the FETCH_SIZE / WRITE_SIZE
    counters of the step kernel (each launch reads and writes nbytes)."""
    import torch
    from paper_1710_04751_amd import capi
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    capi.lbm_copy_probe(b.data_ptr(), a.data_ptr(), nbytes)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        capi.lbm_copy_probe(b.data_ptr(), a.data_ptr(), nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    log(f"copy probe: {nbytes >> 30} GiB in {ms:.3f} ms -> {gbs:.1f} GB/s read+write")
    return {"bytes_per_launch_each_way": nbytes, "ms": ms, "GBs": gbs}


def batched_params(count=64, seed=1710, precision="fp32"):
    """The uneven batch: edge lengths uniform over {32, 48, 64, 80, 96}, Ra
    log-uniform in [1e3, 1e6] (seeded), Pr = 0.71, u0 = 0.05, D3Q7.  Small
    boxes at high Ra need relaxation rates up to 1.98, so the batch uses the
    stable rate set (bulk rate 1, Maxwellian fourth-order equilibrium,
    c_sphi^2 = 1/4)."""
    from paper_1710_04751_amd import solver as S
    from paper_1710_04751_amd import workloads as W
    return [S.make_params(n, ra, precision=precision, **W.STABLE_RATES)
            for n, ra in W.batched_cavities(count, seed)]


def time_batched(steps, log=print):
    """Aggregate MLUPS of the batch in one persistent graph-replayed launch
    per step (autotuned shape) against the same cavities stepped by
    separate single-cavity launches, cavity after cavity."""
    import torch
    from paper_1710_04751_amd import solver as S

    params = batched_params()
    cells = sum(p.nx * p.ny * p.nz for p in params)
    batch = S.Batch(params)
    threads, bpc = batch.autotune(steps_per_trial=6)
    batch.step(100)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    info = batch.launch_info()
    batch.close()
    del batch
    torch.cuda.empty_cache()
    stream = torch.cuda.Stream()
    cavs = [S.Cavity(p, stream=stream) for p in params]
    for c in cavs:
        c.step(10)
    torch.cuda.synchronize()
    e0.record(stream)
    for c in cavs:
        c.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    for c in cavs:
        c.close()
    del cavs
    torch.cuda.empty_cache()
    mb = cells * steps / (ms_b * 1e-3) / 1e6
    ms = cells * steps / (ms_s * 1e-3) / 1e6
    log(f"batched: {len(params)} cavities, {cells} cells: {mb:.0f} MLUPS in one launch per step "
        f"(threads {threads}, {bpc} blocks/CU, graph {info['graph_steps']}) vs {ms:.0f} MLUPS "
        f"sequential ({mb / ms:.2f}x)")
    return {"workload": "64 cavities, N in {32,48,64,80,96}, Ra log-uniform 1e3-1e6, seed 1710, "
                        "D3Q7, FP32", "cavities": len(params), "cells": cells, "steps": steps,
            "value": round(mb, 1), "unit": "MLUPS", "sequential_MLUPS": round(ms, 1),
            "speedup": round(mb / ms, 3), "threads": threads, "blocks_per_cu": bpc,
            "graph_steps": info["graph_steps"]}


def time_batched_steady(sequential=False, log=print):
    """Every cavity of the batch run to steady state (the steady rule of
    workloads.STEADY_RULE, step limit 400,000) in the batch, retiring
    members as they stop; optionally once more cavity after cavity with
    single-cavity launches.  Aggregate MLUPS = sum over cavities of cells x
    steps taken / wall time."""
    import torch
    from paper_1710_04751_amd import capi
    from paper_1710_04751_amd import solver as S
    from paper_1710_04751_amd import workloads as W

    params = batched_params()
    cells = [p.nx * p.ny * p.nz for p in params]
    rule = dict(W.STEADY_RULE)
    cap = 400_000
    batch = S.Batch(params)
    threads, bpc = batch.autotune(steps_per_trial=6)
    for m in batch.members:  # autotuning advanced the members: start from rest
        m.init_rest()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_b, how_b, res_b = batch.run_to_steady(max_steps=cap, **rule)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    done_b = [m.steps_done() for m in batch.members]
    upd_b = sum(c * s for c, s in zip(cells, done_b))
    batch.close()
    del batch
    torch.cuda.empty_cache()
    names = {capi.LBM_STEADY_TOL: "tol", capi.LBM_STEADY_PLATEAU: "plateau",
             capi.LBM_STEADY_MAX_STEPS: "max_steps", capi.LBM_STEADY_UNSTABLE: "unstable",
             capi.LBM_STEADY_STALLED: "stalled"}
    ended = [names[h] for h in how_b]
    conv = [i for i, e in enumerate(ended) if e in ("tol", "plateau")]
    stalled = [i for i, e in enumerate(ended) if e == "stalled"]
    members = W.batched_cavities()
    log(f"batched to steady: {wall_b:.1f} s, {upd_b / wall_b / 1e6:.0f} MLUPS, "
        f"{len(conv)} steady, {len(stalled)} stalled")
    out = {"value": round(upd_b / wall_b / 1e6, 1), "unit": "MLUPS", "wall_s": round(wall_b, 2),
           "cell_updates": upd_b, "rule": rule, "max_steps": cap,
           "ended": {e: ended.count(e) for e in sorted(set(ended))},
           "steps_to_steady": steps_b, "steps_run": done_b,
           "steady_members": [{"n": members[i][0], "Ra": round(members[i][1], 1),
                               "steps": steps_b[i]} for i in conv],
           "stalled_members": [{"n": members[i][0], "Ra": round(members[i][1], 1),
                                "steps_run": done_b[i], "last_residual": res_b[i]}
                               for i in stalled],
           "threads": threads, "blocks_per_cu": bpc}
    if not sequential:
        return out
    stream = torch.cuda.Stream()
    wall_s, upd_s, steps_s = 0.0, 0, []
    for i, p in enumerate(params):
        cav = S.Cavity(p, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, how, _ = cav.run_to_steady(max_steps=cap, **rule)
        torch.cuda.synchronize()
        wall_s += time.perf_counter() - t0
        upd_s += cells[i] * cav.steps_done()
        steps_s.append(st)
        cav.close()
        if i % 8 == 7:
            log(f"sequential to steady: {i + 1}/{len(params)} cavities, {wall_s:.1f} s")
    ms = upd_s / wall_s / 1e6
    log(f"to steady: batched {out['value']:.0f} MLUPS ({wall_b:.1f} s) vs sequential {ms:.0f} "
        f"MLUPS ({wall_s:.1f} s)")
    out.update({"sequential_MLUPS": round(ms, 1), "sequential_wall_s": round(wall_s, 2),
                "speedup_wall": round(wall_s / wall_b, 3),
                "steps_to_steady_sequential": steps_s})
    return out


GOLDEN_128 = os.path.join(ROOT, "tests", "golden", "cavity128_ra1e6_d3q7_2500.npz")


def block_planes(mac, planes):
    """4x4x4 block means of 512^3 fields [5][512][512][512] taken at the
    128^3 cell planes y = planes[0] and z = planes[1]: ([5][z][x], [5][y][x])."""
    import torch
    yb, zb = planes
    a = mac[:, :, 4 * yb:4 * yb + 4, :].reshape(5, 128, 4, 4, 128, 4).mean(dim=(2, 3, 5))
    b = mac[:, 4 * zb:4 * zb + 4, :, :].reshape(5, 4, 128, 4, 128, 4).mean(dim=(1, 3, 5))
    return a, b


def field_errors(a, b):
    """Errors per field of [5][...] arrays: max and root-mean-square of a - b,
    each normalised by max |b| (rho by max |rho - 1|, the velocity components
    by the largest reference velocity component)."""
    names = ("rho", "ux", "uy", "uz", "T")
    umax = max(float(b[i].abs().max()) for i in (1, 2, 3))
    out = {}
    for i, k in enumerate(names):
        if k == "rho":
            scale = float((b[i] - 1.0).abs().max())
        elif k == "T":
            scale = float(b[i].abs().max())
        else:
            scale = umax
        d = a[i] - b[i]
        out[k] = float(d.abs().max()) / scale
        out[k + "_rms"] = float(d.pow(2).mean().sqrt()) / scale
    return out


def precision_study(steps=10_000, log=print):
    """512^3, Ra 1e6, D3Q7 from rest for 10,000 steps with FP32 and with
    FP16 storage (FP32 arithmetic), the stable rate set of the 128^3 FP64
    oracle run at the same Ra, Pr, u0 and physical time (2,500 steps):
    errors of the 4x4x4 block means against the oracle on the mid-planes,
    and FP16 against FP32 over every cell."""
    import numpy as np
    import torch
    from paper_1710_04751_amd import solver as S
    from paper_1710_04751_amd import workloads as W

    if not os.path.exists(GOLDEN_128):
        log("precision study: 128^3 reference missing, skipped")
        return None
    ref = np.load(GOLDEN_128)
    planes = (int(ref["plane_y"]), int(ref["plane_z"]))
    ry = torch.from_numpy(ref["y64"].astype(np.float64)).cuda()
    rz = torch.from_numpy(ref["z64"].astype(np.float64)).cuda()
    out, full = {}, {}
    for prec in ("fp32", "fp16", "fp16_sr"):
        sr = 1 if prec == "fp16_sr" else 0
        cav = S.Cavity(S.make_params(512, 1e6, precision=prec[:4], round_stochastic=sr,
                                     **W.STABLE_RATES))
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(2000, steps - done)
            cav.step(k)
            torch.cuda.synchronize()
            done += k
            log(f"precision study {prec}: {done}/{steps} steps")
        secs = time.perf_counter() - t0
        m = cav.macros(fp64=False)
        mac = torch.stack([m[k] for k in ("rho", "ux", "uy", "uz", "T")])
        del m
        cav.close()
        del cav
        torch.cuda.empty_cache()
        a, b = block_planes(mac, planes)
        e_y, e_z = field_errors(a.double(), ry), field_errors(b.double(), rz)
        out[prec] = {"vs_oracle128": {k: max(e_y[k], e_z[k]) for k in e_y},
                     "seconds": round(secs, 2), "steps": steps}
        full[prec] = mac
        log(f"precision study {prec}: vs 128^3 oracle {out[prec]['vs_oracle128']}")
    d = field_errors(full["fp16"], full["fp32"])
    out["fp16_vs_fp32"] = d
    out["fp16_sr_vs_fp32"] = field_errors(full["fp16_sr"], full["fp32"])
    log(f"precision study: fp16 (stochastic rounding) vs fp32 {out['fp16_sr_vs_fp32']}")
    log(f"precision study: fp16 vs fp32 over all cells {d}")
    out["workload"] = ("512^3, Ra 1e6, D3Q7, from rest, 10,000 steps, stable rate set; reference "
                       "128^3 FP64 oracle, 2,500 steps (same t u0 / L), mid-planes y = 64, z = 64 "
                       "of the 128^3 grid against 4x4x4 block means")
    del full
    torch.cuda.empty_cache()
    return out


def warm_start(log=print):
    """The learned warm start at 64^3: steady training/test sets from the
    batched solver, GPU training of the network, then every test cavity
    solved from its prediction; steps to the steady rule warm vs cold."""
    from paper_1710_04751_amd import warmstart as WS
    from paper_1710_04751_amd import workloads as W
    t0 = time.perf_counter()
    r = WS.study(log=log)
    keys = ("grid", "train", "test", "ra_range", "train_converged", "test_converged",
            "cold_no_steady_state", "lowest_ra_without_steady_state", "highest_ra_converged",
            "warm_converged_without_cold_steady_state", "epochs", "batch", "train_seconds",
            "train_tflops", "final_train_loss", "val_loss", "cold_steps_median",
            "warm_steps_median", "cold_steps_mean", "warm_steps_mean", "steps_ratio_median",
            "nu_rel_diff_max", "fallbacks", "cold_solve_s", "warm_solve_s")
    out = {k: r[k] for k in keys}
    out["workload"] = ("64^3 cavities, Ra log-uniform in [1e3, 1e6], 200 training (seed 17101) "
                       "and 50 held-out (seed 17102) Rayleigh numbers, D3Q7, FP32 solver, "
                       f"rate set {W.STABLE_RATES}, u0 0.05, steady rule {W.STEADY_RULE}, "
                       "step limit 300,000; network BF16/FP32-accumulate on the matrix cores; "
                       "steps medians over the held-out cavities whose cold solve meets the "
                       "rule (fallbacks charged warm + cold steps)")
    out["unit"] = "steps to the steady rule"
    out["no_steady_state_test"] = [
        {"Ra": round(10 ** u["log10_ra"], 1), "cold": u["cold_how"],
         "cold_steps_run": u["cold_steps_run"], "cold_last_residual": u["cold_last_residual"],
         "warm": u["warm_how"]} for u in r["no_steady_state"]]
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    log(f"warm start: median steps {out['warm_steps_median']:.0f} warm vs "
        f"{out['cold_steps_median']:.0f} cold, max |dNu|/Nu {out['nu_rel_diff_max']:.1e}, "
        f"{out['cold_no_steady_state']} of {out['train'] + out['test']} without a steady state "
        f"from rest, training {out['train_tflops']:.1f} TFLOP/s")
    return out


def nn_throughput(steps=20, grid=64, batch=8, log=print):
    """Training and inference throughput of the warm-start network on the
    matrix cores: seeded initial parameters, random targets, `steps` timed
    training steps (forward, backward, Adam) and forward passes."""
    import numpy as np
    import torch
    from paper_1710_04751_amd.network import WarmStartNet, init_params

    net = WarmStartNet(grid, batch)
    net.set_params(torch.from_numpy(init_params(1)))
    g = torch.Generator(device="cuda").manual_seed(5)
    targets = 0.1 * torch.randn(batch, 4, grid, grid, grid, device="cuda", generator=g)
    lra = list(np.linspace(3.0, 5.0, batch))
    idx = list(range(batch))
    for _ in range(3):
        net.train_step(lra, targets, idx, want_loss=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.train_step(lra, targets, idx, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    t_train = e0.elapsed_time(e1) / steps * 1e-3
    e0.record()
    for _ in range(steps):
        net.forward(lra)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / steps * 1e-3
    f_fwd, f_train = net.flops(batch)
    net.close()
    out = {"grid": grid, "batch": batch, "steps": steps,
           "train_step_ms": round(t_train * 1e3, 3),
           "train_TFLOPs": round(f_train / t_train / 1e12, 2),
           "forward_ms": round(t_fwd * 1e3, 3), "forward_TFLOPs": round(f_fwd / t_fwd / 1e12, 2),
           "peak_TFLOPs_bf16": 2500.0, "dtype": "bf16 operands, fp32 accumulate"}
    log(f"network: train step {out['train_step_ms']} ms ({out['train_TFLOPs']} TFLOP/s), "
        f"forward {out['forward_ms']} ms ({out['forward_TFLOPs']} TFLOP/s)")
    return out


def cpu_baseline(n_full, ra, seconds_hint=15.0, log=print):
    """The oracle on a bounded sample of the workload: a 64^3 block of cells
    with the 512^3 case's lattice parameters, a few steps, all host threads."""
    import numpy as np
    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    used = O.set_threads(threads)
    p = O.cavity_params(n_full, ra)
    side = 64
    p.nx = p.ny = p.nz = side
    F, G = O.rest_state(p)
    O.run(p, 1, F, G)  # warm
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds_hint:
        F, G, _ = O.run(p, 2, F, G)
        steps += 2
    dt = time.perf_counter() - t0
    mlups = side ** 3 * steps / dt / 1e6
    log(f"cpu oracle: {side}^3 x {steps} steps in {dt:.1f}s on {used} threads -> {mlups:.3f} MLUPS")
    # the same on one core (2 steps)
    O.set_threads(1)
    t1 = time.perf_counter()
    F, G, _ = O.run(p, 2, F, G)
    d1 = time.perf_counter() - t1
    O.set_threads(threads)
    single = side ** 3 * 2 / d1 / 1e6
    log(f"cpu oracle, one core: {single:.3f} MLUPS")
    # the small parity case in full: 16^3, Ra 1e3, 2000 steps from rest (8.2 M cell updates)
    from paper_1710_04751_amd import workloads as W
    c = W.SMALL_PARITY
    ps = O.cavity_params(c.n, c.Ra, Pr=c.Pr, u0=c.u0)
    Fs, Gs = O.rest_state(ps)
    t2 = time.perf_counter()
    O.run(ps, c.steps, Fs, Gs)
    d2 = time.perf_counter() - t2
    small = {"workload": f"{c.n}^3, Ra {c.Ra:g}, {c.steps} steps from rest, D3Q7, FP64",
             "cell_updates": c.n ** 3 * c.steps, "seconds": round(d2, 3),
             "MLUPS": round(c.n ** 3 * c.steps / d2 / 1e6, 4), "threads": used}
    log(f"cpu oracle, {small['workload']}: {d2:.2f} s, {small['MLUPS']} MLUPS")
    return {"value": mlups, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "single_core_MLUPS": round(single, 4), "small_cavity_2000_steps": small,
            "sample": f"{side}^3 cells with the {n_full}^3 Ra={ra:g} lattice parameters, "
                      f"{steps} steps from rest ({dt:.1f} s) on {used} threads, then 2 steps on "
                      f"one core ({d1:.1f} s), FP64 oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--Ra", type=float, default=1e6)
    ap.add_argument("--fp16-steps", type=int, default=None,
                    help="timed steps of the FP16-storage line (default: --steps)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--block", type=str, default=None, help="bx,by of the step kernel")
    ap.add_argument("--no-nn", action="store_true", help="skip the network throughput leg")
    ap.add_argument("--sr-steps", type=int, default=2000,
                    help="timed steps of the FP16 stochastic-rounding line; 0 skips it")
    ap.add_argument("--q15-steps", type=int, default=1000,
                    help="timed steps of the D3Q15-scalar line; 0 skips it")
    ap.add_argument("--source-steps", type=int, default=1000,
                    help="timed steps of the heat-source line (general kernels); 0 skips it")
    ap.add_argument("--fp64-steps", type=int, default=500,
                    help="timed steps of the FP64 line (352 B per update); 0 skips it")
    ap.add_argument("--slab-steps", type=int, default=0,
                    help="timed FP32 steps on one z-slab of an 8-way split of the n^3 cavity "
                         "(n x n x n/8, the share of one GPU); 0 (default) skips it")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 512^3 FP32/FP16 comparison with the 128^3 oracle reference")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned warm-start study at 64^3 (about 3 minutes)")
    ap.add_argument("--no-batched-steady", action="store_true",
                    help="skip running every cavity of the batch to steady state")
    ap.add_argument("--batched-steady-sequential", action="store_true",
                    help="also run every cavity of the batch to steady state with "
                         "single-cavity launches, one after another (a few minutes)")
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "z-slab decomposition is described in the design notes, not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    block = tuple(int(v) for v in args.block.split(",")) if args.block else None
    copy = copy_calibration(log=log)
    log(f"bench: {args.n}^3 Ra={args.Ra:g} D3Q7, {args.steps} timed steps, warmup {args.warmup}")
    main_line = time_variant(args.n, args.Ra, "fp32", args.steps, args.warmup, block, log)
    log(json.dumps(main_line))
    f16_steps = args.fp16_steps if args.fp16_steps is not None else args.steps
    f16 = time_variant(args.n, args.Ra, "fp16", f16_steps, args.warmup, block, log)
    log(json.dumps(f16))
    f16sr = None
    if args.sr_steps > 0:
        f16sr = time_variant(args.n, args.Ra, "fp16", args.sr_steps, args.warmup, block, log, sr=1)
        log(json.dumps(f16sr))
    q15 = None
    if args.q15_steps > 0:
        q15 = time_variant(args.n, args.Ra, "fp32", args.q15_steps, args.warmup, block, log, qt=15)
        log(json.dumps(q15))
    src = None
    if args.source_steps > 0:
        src = time_variant(args.n, args.Ra, "fp32", args.source_steps, args.warmup, block, log,
                           R=SOURCE_R)
        log(json.dumps(src))
    f64 = None
    if args.fp64_steps > 0:
        f64 = time_variant(args.n, args.Ra, "fp64", args.fp64_steps, args.warmup, block, log)
        log(json.dumps(f64))
    slab = None
    if args.slab_steps > 0:
        slab = time_variant(args.n, args.Ra, "fp32", args.slab_steps, args.warmup, block, log,
                            shape=(args.n, args.n, args.n // 8))
        log(json.dumps(slab))
    batched = None if args.no_batched else time_batched(args.batched_steps, log=log)
    if batched is not None and not args.no_batched_steady:
        batched["to_steady"] = time_batched_steady(args.batched_steady_sequential, log=log)
    nn = None if args.no_nn else nn_throughput(log=log)
    precision = None if args.no_precision else precision_study(log=log)
    warm = None if args.no_warm_start else warm_start(log=log)
    cpu = None if args.no_cpu else cpu_baseline(args.n, args.Ra, log=log)

    rec = {
        "metric": METRIC,
        "value": round(main_line["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_line["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"cavity{args.n}_ra{args.Ra:g}_d3q7",
            "cells": args.n ** 3, "Ra": args.Ra, "Pr": 0.71, "u0": 0.05,
            "flow_lattice": "D3Q15", "thermal_lattice": "D3Q7", "storage": "fp32",
            "start": "rest", "kernel": main_line["kernel"], "block": main_line["block"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(main_line["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_line["frac_hbm_peak"], 4),
            "traffic": recorded_traffic(args.n, "fp32"),
        },
        "fp16_storage": {
            "value": round(f16["mlups"], 1), "unit": "MLUPS", "steps": f16_steps,
            "rounding": "nearest (fast; see precision_vs_oracle for its error)",
            "ms_per_step": f16["ms_per_step"], "kernel": f16["kernel"],
            "roofline": {"bound": "hbm", "achieved": round(f16["achieved_GBs"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(f16["frac_hbm_peak"], 4),
                         "traffic": recorded_traffic(args.n, "fp16")},
            "stochastic_rounding": None if f16sr is None else {
                "value": round(f16sr["mlups"], 1), "unit": "MLUPS", "steps": args.sr_steps,
                "rounding": "stochastic (the accurate FP16 form)",
                "ms_per_step": f16sr["ms_per_step"], "frac": round(f16sr["frac_hbm_peak"], 4)},
        },
        "thermal_d3q15": None if q15 is None else {
            "value": round(q15["mlups"], 1), "unit": "MLUPS", "steps": args.q15_steps,
            "storage": "fp32", "ms_per_step": q15["ms_per_step"], "kernel": q15["kernel"],
            "bytes_per_cell_update": q15["bytes_per_cell_update"],
            "roofline": {"bound": "hbm", "achieved": round(q15["achieved_GBs"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(q15["frac_hbm_peak"], 4),
                         "traffic": recorded_traffic(args.n, "fp32_q15")},
        },
        "heat_source": None if src is None else {
            "value": round(src["mlups"], 1), "unit": "MLUPS", "steps": args.source_steps,
            "R": SOURCE_R, "storage": "fp32", "ms_per_step": src["ms_per_step"],
            "kernel": src["kernel"],
            "roofline": {"bound": "hbm", "achieved": round(src["achieved_GBs"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(src["frac_hbm_peak"], 4),
                         "traffic": recorded_traffic(args.n, "fp32_source")},
        },
        "fp64": None if f64 is None else {
            "value": round(f64["mlups"], 1), "unit": "MLUPS", "steps": args.fp64_steps,
            "storage": "fp64", "ms_per_step": f64["ms_per_step"], "kernel": f64["kernel"],
            "bytes_per_cell_update": f64["bytes_per_cell_update"],
            "roofline": {"bound": "hbm", "achieved": round(f64["achieved_GBs"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(f64["frac_hbm_peak"], 4),
                         "traffic": recorded_traffic(args.n, "fp64")},
        },
        "slab": None if slab is None else {
            "shape": [args.n, args.n, args.n // 8], "value": round(slab["mlups"], 1),
            "unit": "MLUPS", "steps": args.slab_steps, "storage": "fp32",
            "ms_per_step": slab["ms_per_step"], "block": slab["block"],
            "roofline": {"bound": "hbm", "achieved": round(slab["achieved_GBs"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(slab["frac_hbm_peak"], 4), "traffic": None},
            # populations with e_z = +1 or -1 that cross one slab face per step
            # (5 flow + 1 scalar), FP32: what each neighbour exchange would carry
            "face_bytes_per_step": 6 * args.n * args.n * 4,
        },
        "batched": batched,
        "network": nn,
        "precision_vs_oracle": precision,
        "warm_start": warm,
        "copy_probe": {"GBs": round(copy["GBs"], 1), "bytes": copy["bytes_per_launch_each_way"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
