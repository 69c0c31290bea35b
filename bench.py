"""Benchmark: Larger-than-Life cell-updates/s on one MI355X, CAT int8-MFMA vs the LDS direct stencil.

A bench step is one full run of the workload: ``ltl_step(100)`` on the Bosco-type rule
R5 C0 M1 S34..58 B34..45 N_M over a 4096 x 4096 uint8 grid (Bernoulli(0.5), seed 2, dead
ghost halo), inputs resident in HBM. Prints one JSON line.

Also reported (not the headline value): the batched workload (512 instances of log-uniform
sides in [128, 2048], r uniform in 1..16, per-instance rules; one ``ltl_batch_step(32)``
hipGraph per bench step), and with --sweep the radius sweep r = 1..16 on 16384^2 for the
int8, fp16 and fp8 (r <= 7) CAT variants and the direct stencil.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--sweep] [--no-cpu] [--no-batch] [--autotune]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s vs radius r=1..16, CAT int8-MFMA vs direct stencil, bit-exact"
INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 MFMA
HBM_PEAK_GBS = 8000.0
OPS_PER_CELL = 256       # two 16x16x64 int8 MFMAs per 256 cells, 2 ops per multiply-add
DEFAULT_TUNING = "4,160,224,8"   # steps per launch, tile rows, tile cols, waves
KERNEL_SRC = [os.path.join(ROOT, "paper_2406_17284_amd", "csrc", f) for f in ("cat_device.h", "cat_kernel.hip")]
BATCH_TUNING = "3,160,160,8"   # the autotuner's pick for the 512-instance batch on MI355X
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "cat_step_i8_bosco4096_traffic.json")
MFMA_RECORD = os.path.join(ROOT, "profiles", "cat_step_i8_bosco4096_sq.json")


def kernel_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


SHAPE_KEYS = ("steps_per_launch", "tile_rows", "tile_cols", "waves", "persistent")


def parse_tuning(text):
    """'T,tile_rows,tile_cols,waves[,persistent]' -> keyword arguments of set_tuning."""
    vals = [int(x) for x in text.split(",")]
    return dict(zip(SHAPE_KEYS, vals))


def recorded_traffic(tuning):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter record, if it was
    taken on this kernel source and launch shape; else None."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    shape = [tuning[k] for k in SHAPE_KEYS]
    if rec.get("kernel_sha256") != kernel_hash() or rec.get("tuning") != shape:
        return None
    return rec["hbm_bytes_per_launch"]


def recorded_mfma_ops(tuning):
    """int8 MFMA ops issued per launch (SQ_INSTS_VALU_MFMA_MOPS_I8 x 512) from the committed
    counter record, if it was taken on this kernel source and launch shape; else None."""
    try:
        with open(MFMA_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    shape = [tuning[k] for k in SHAPE_KEYS]
    if rec.get("kernel_sha256") != kernel_hash() or rec.get("tuning") != shape:
        return None
    return rec["mfma_ops_per_launch"]


def timed_runs(sim, n_per_run, runs, torch):
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(runs):
        sim.step(n_per_run)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batch(args, ltl, inputs, torch):
    """The batched workload: 512 automata advanced together, 32 steps per bench step."""
    insts = inputs.batch_instances()
    steps = 32
    dev = [inputs.bernoulli_grid_torch(x.H, x.W, 0.5, x.seed, device="cuda") for x in insts]
    rules = [x.rule for x in insts]
    cells = sum(x.H * x.W for x in insts)
    res = {"workload": "512 instances, sides log-uniform in [128, 2048], r uniform in 1..16, S/B uniform in "
                       "[0.2, 0.5] x (2r+1)^2, M1, Bernoulli(0.5), 32 steps per bench step (one hipGraph)",
           "cells": cells}
    bt = ltl.Batch(dev, rules, "cat_i8")
    if args.autotune:
        bt.autotune(probe_steps=4)
    else:
        T, th, tw, wv = (int(x) for x in args.batch_tuning.split(","))
        bt.set_tuning(steps_per_launch=T, tile_rows=th, tile_cols=tw, waves=wv)
    for _ in range(max(1, args.warmup)):
        bt.step(steps)
    secs, _ = timed_runs(bt, steps, args.steps, torch)
    res["value"] = cells * steps * args.steps / secs
    res["unit"] = "cell-updates/s"
    res["ms_per_bench_step"] = secs / args.steps * 1e3
    res["tuning"] = bt.tuning()
    bt.close()

    db = ltl.Batch(dev, rules, "direct")
    db.step(steps)
    dsecs, _ = timed_runs(db, steps, 1, torch)
    res["direct_stencil_cell_updates_per_s"] = cells * steps / dsecs
    db.close()

    # cross-check: a fresh CAT batch and the direct batch after the same 32 steps, all instances
    a = ltl.Batch(dev, rules, "cat_i8")
    b = ltl.Batch(dev, rules, "direct")
    a.step(steps)
    b.step(steps)
    res["cat_vs_direct_equal"] = all(torch.equal(a.read(i), b.read(i)) for i in range(len(insts)))
    a.close()
    b.close()
    return res


def bench_life(ltl, inputs, torch):
    """The small workload: Life (R1 C0 M1 S3..4 B3..3) on 256^2, 64 steps per run, autotuned;
    launch-latency bound (one 256^2 grid is a few tiles). Returns the result object, the
    initial grid and the GPU grid after one run (for the oracle check)."""
    w = inputs.WORKLOADS["life256"]
    g_np = inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)
    g = torch.from_numpy(g_np).cuda()
    s = ltl.Simulation(g, w.rule, "cat_i8")
    tuning = s.autotune(probe_steps=w.steps)
    s.step(w.steps)
    runs = 20
    secs, _ = timed_runs(s, w.steps, runs, torch)
    s.close()
    s = ltl.Simulation(g, w.rule, "cat_i8", tuning={k: tuning[k] for k in SHAPE_KEYS})
    s.step(w.steps)
    final = s.read().cpu().numpy()
    s.close()
    res = {"workload": f"life256: R1 C0 M1 S3..4 B3..3 N_M, 256x256, Bernoulli(0.5) seed {w.seed}, "
                       f"{w.steps} steps per run", "tuning": tuning, "us_per_run": secs / runs * 1e6,
           "value": w.H * w.W * w.steps * runs / secs, "unit": "cell-updates/s"}
    return res, g_np, final


def bench_decay(args, ltl, inputs, torch):
    """The multi-state workload: R16 C8 M0 S300..500 B330..420, 32768^2, 20 steps per bench step
    (the CAT step time does not depend on the grid's contents)."""
    w = inputs.WORKLOADS["decay32768"]
    g = inputs.bernoulli_grid_torch(w.H, w.W, w.p, w.seed, device="cuda")
    res = {"workload": "decay32768: R16 C8 M0 S300..500 B330..420 N_M, 32768x32768, Bernoulli(0.5), 20 steps"}
    for method in ("cat_i8", "direct"):
        s = ltl.Simulation(g, w.rule, method)
        if method == "cat_i8":
            s.autotune(probe_steps=4)
            res["tuning"] = s.tuning()
        s.step(w.steps)
        secs, _ = timed_runs(s, w.steps, 1 if method == "direct" else max(1, min(args.steps, 3)), torch)
        runs = 1 if method == "direct" else max(1, min(args.steps, 3))
        res[method] = w.H * w.W * w.steps * runs / secs
        s.close()
    res["unit"] = "cell-updates/s"
    return res


XGMI_LINK_GBS = 153.0   # one xGMI link of an MI355X, one direction (published figure)


def bench_shard(args, ltl, inputs, torch):
    """One GPU's share of the radius-sweep grid split N = `args.shard` ways: the CAT int8 rate on
    a (side/N) x side row strip and on a 2-D block of the same size (side/a x side/b, a * b = N,
    a >= b closest) next to the whole grid's, and the halo a strip would trade with each
    neighbour per launch (r * T rows of `side` bytes, one xGMI link per neighbour). The exchange
    time is the link model, not a measurement: this library runs on one GPU."""
    side, n = args.sweep_side, args.shard
    rows = side // n
    b = max(d for d in range(1, n + 1) if n % d == 0 and d * d <= n)
    a = n // b
    full = inputs.bernoulli_grid_torch(side, side, 0.5, 3, device="cuda")
    strip = full[:rows].contiguous()
    block = full[:side // a, :side // b].contiguous()
    res = {"workload": f"{rows}x{side} row strip and {side // a}x{side // b} block (1/{n}) of the {side}x{side} "
                       "sweep grid, sweep rules, 50 steps",
           "xgmi_link_GBs_model": XGMI_LINK_GBS, "per_r": {}}
    for r in (1, 5, 16):
        rule = inputs.sweep_rule(r)
        row = {}
        for name, g in (("strip", strip), ("block", block), ("whole", full)):
            s = ltl.Simulation(g, rule, "cat_i8")
            s.autotune(probe_steps=10)
            s.step(50)
            secs, _ = timed_runs(s, 50, 1, torch)
            row[name + "_cell_updates_per_s"] = g.shape[0] * g.shape[1] * 50 / secs
            if name == "strip":
                T = s.tuning()["steps_per_launch"]
                row["strip_tuning"] = s.tuning()
                launch_s = secs / (50 / T)
            s.close()
        halo = r * T * side
        row["halo_bytes_per_edge_per_launch"] = halo
        row["launch_us"] = launch_s * 1e6
        row["exchange_us_model"] = halo / (XGMI_LINK_GBS * 1e9) * 1e6
        res["per_r"][str(r)] = row
    return res


def mfma_issued(tuning, avg_launch_s, cells, r):
    """Counter-measured MFMA utilisation of the timed kernel: int8 ops the MFMAs issue per
    launch (committed SQ counter record) over launch time x peak, and the useful fraction:
    the band non-zeros, 4(2r+1) ops per cell-update, over the ops issued per cell-update."""
    ops = recorded_mfma_ops(tuning)
    if ops is None:
        return None
    steps = tuning["steps_per_launch"]
    issued_per_cell = ops / (cells * steps)
    return {"ops_per_launch": ops, "frac_of_peak": ops / avg_launch_s / (INT8_PEAK_TOPS * 1e12),
            "issued_ops_per_cell_update": issued_per_cell,
            "useful_ops_per_cell_update": 4 * (2 * r + 1),
            "useful_frac": 4 * (2 * r + 1) / issued_per_cell}


def gpu_energy_reader(torch):
    """Returns a function giving the GPU's energy counter in joules (amdsmi), or raises."""
    import amdsmi
    amdsmi.amdsmi_init()
    handles = amdsmi.amdsmi_get_processor_handles()
    if not handles:
        raise RuntimeError("amdsmi sees no GPU")
    handle = handles[0]
    if len(handles) > 1:   # several visible to amdsmi: pick the one HIP runs on, by PCI bus id
        props = torch.cuda.get_device_properties(0)
        bus = getattr(props, "pci_bus_id", None)
        for h in handles:
            bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)
            if bus is not None and int(bdf.split(":")[1], 16) == bus:
                handle = h
                break

    def read():
        e = amdsmi.amdsmi_get_energy_count(handle)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6
    return read


def bench_energy(args, ltl, inputs, torch):
    """Energy efficiency (cell-updates per joule) at the largest workload grid: Bosco R5 on
    32768^2, 1000-step runs of CAT int8 and a shorter run of the direct stencil, the GPU's own
    energy counter read before and after each (idle draw measured over the same kind of span)."""
    try:
        energy = gpu_energy_reader(torch)
        energy()
    except Exception as e:   # no energy counter on this machine: report why instead
        return {"error": f"{type(e).__name__}: {e}"}
    side, rule = 32768, inputs.BOSCO_M1
    g = inputs.bernoulli_grid_torch(side, side, 0.5, 6, device="cuda")
    res = {"workload": "Bosco R5 C0 M1 S34..58 B34..45 N_M on 32768x32768, Bernoulli(0.5) seed 6, dead halo",
           "source": "amdsmi energy accumulator of the GPU (whole board), before/after synchronized runs"}
    torch.cuda.synchronize()
    e0, t0 = energy(), time.perf_counter()
    time.sleep(2.0)
    e1, t1 = energy(), time.perf_counter()
    res["idle_W"] = (e1 - e0) / (t1 - t0)
    for method, steps, reps in (("cat_i8", 1000, 3), ("direct", 100, 2)):
        s = ltl.Simulation(g, rule, method)
        if method == "cat_i8":
            s.set_tuning(**parse_tuning(args.tuning))
        s.step(steps // 10)
        torch.cuda.synchronize()
        e0, t0 = energy(), time.perf_counter()
        for _ in range(reps):
            s.step(steps)
        torch.cuda.synchronize()
        e1, t1 = energy(), time.perf_counter()
        joules, secs = e1 - e0, t1 - t0
        n = side * side * steps * reps
        res[method] = {"steps": steps * reps, "seconds": secs, "joules": joules, "avg_W": joules / secs,
                       "cell_updates_per_s": n / secs, "cell_updates_per_J": n / joules,
                       "cell_updates_per_J_above_idle": n / max(1e-9, joules - res["idle_W"] * secs)}
        s.close()
    res["cat_over_direct_per_J"] = res["cat_i8"]["cell_updates_per_J"] / res["direct"]["cell_updates_per_J"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)   # long enough for the GPU clocks to settle
    ap.add_argument("--sweep", action="store_true", help="also time the radius sweep r=1..16 on 16384^2")
    ap.add_argument("--sweep-side", type=int, default=16384)
    ap.add_argument("--sweep-rmax", type=int, default=16, help="largest radius of the sweep (int8 and direct reach 32)")
    ap.add_argument("--life", action="store_true",
                    help="also time the Life 256^2 workload (64 steps per run; its autotuning launches the "
                         "benchmark's kernel at other shapes, so it is off in the profiled default run)")
    ap.add_argument("--shard", type=int, default=0, metavar="N",
                    help="also time one GPU's row strip (1/N) of the sweep grid and the halo it would exchange")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-instance batched workload")
    ap.add_argument("--decay", action="store_true", help="also time the C=8 R16 decay workload on 32768^2")
    ap.add_argument("--energy", action="store_true",
                    help="also measure cell-updates per joule (CAT int8 and direct, Bosco R5 on 32768^2)")
    ap.add_argument("--batch-tuning", type=str, default=BATCH_TUNING, help="T,tile_rows,tile_cols,waves of the batch")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape with ltl_autotune")
    ap.add_argument("--tuning", type=str, default=DEFAULT_TUNING,
                    help="T,tile_rows,tile_cols,waves[,persistent] (default: the autotuner's pick on MI355X)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.calib_copy:
        import torch

        n = args.calib_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2406_17284_amd import inputs, ltl

    torch.cuda.set_device(0)
    w = inputs.WORKLOADS["bosco4096"]
    g0_np = inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)
    g0 = torch.from_numpy(g0_np).cuda()
    cells = w.H * w.W

    # ---- CAT int8
    sim = ltl.Simulation(g0, w.rule, "cat_i8")
    if args.autotune:
        sim.autotune(probe_steps=20)
    else:
        sim.set_tuning(**parse_tuning(args.tuning))
    tuning = sim.tuning()
    for _ in range(args.warmup):
        sim.step(w.steps)
    secs, wall = timed_runs(sim, w.steps, args.steps, torch)
    value = cells * w.steps * args.steps / secs
    launches_per_run = math.ceil(w.steps / tuning["steps_per_launch"])
    avg_launch_s = secs / (args.steps * launches_per_run)
    ops_per_launch = OPS_PER_CELL * cells * w.steps / launches_per_run
    achieved_tops = ops_per_launch / avg_launch_s / 1e12
    sim.close()

    # ---- direct stencil, same workload
    simd = ltl.Simulation(g0, w.rule, "direct")
    simd.step(w.steps)
    dsteps = max(1, min(args.steps, 3))
    dsecs, _ = timed_runs(simd, w.steps, dsteps, torch)
    direct_value = cells * w.steps * dsteps / dsecs
    simd.close()

    # ---- parity at the workload's own length: CAT vs direct on the GPU (and the oracle below)
    a = ltl.Simulation(g0, w.rule, "cat_i8")
    a.set_tuning(**{k: tuning[k] for k in SHAPE_KEYS})
    a.step(w.steps)
    b = ltl.Simulation(g0, w.rule, "direct")
    b.step(w.steps)
    cat_final = a.read().cpu().numpy()
    direct_final = b.read().cpu().numpy()
    a.close()
    b.close()
    parity = {"cat_vs_direct_equal": bool(np.array_equal(cat_final, direct_final))}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": "bosco4096: R5 C0 M1 S34..58 B34..45 N_M, 4096x4096 uint8, Bernoulli(0.5) seed 2, "
                        "dead ghost halo, 100 LTL steps per bench step",
            "method": "cat_i8",
            "tuning": tuning,
            "direct_stencil_cell_updates_per_s": direct_value,
            "direct_stencil_algorithmic_GBs": 2 * direct_value / 1e9,   # one byte read + one written per cell-update
            "cat_over_direct": value / direct_value,
            "wall_s": wall,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved_tops,
            "peak": INT8_PEAK_TOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tops / INT8_PEAK_TOPS,
            "traffic": recorded_traffic(tuning),
            "kernel": "cat_step_i8",
            "ops_per_cell_update": OPS_PER_CELL,
            "avg_launch_us": avg_launch_s * 1e6,
            "launches_per_bench_step": launches_per_run,
            "mfma_issued": mfma_issued(tuning, avg_launch_s, cells, w.rule.R),
        },
        "roofline_hbm": {
            "bound": "hbm",
            "achieved": 2 * cells / avg_launch_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": 2 * cells / avg_launch_s / 1e9 / HBM_PEAK_GBS,
            "bytes_per_launch": 2 * cells,
            "note": "algorithmic bytes: one read and one write of the grid per launch",
        },
        "parity": parity,
    }

    if args.sweep:
        sweep = {}
        side = args.sweep_side
        gs = inputs.bernoulli_grid_torch(side, side, 0.5, 3, device="cuda")
        for r in range(1, args.sweep_rmax + 1):
            rule = inputs.sweep_rule(r)
            row = {}
            for method in ("cat_i8", "cat_f16", "cat_f8", "direct"):
                if (method == "cat_f8" and r > 7) or (method == "cat_f16" and r > 16):
                    continue   # fp8-e4m3 counts are exact only for 2r+1 <= 16; fp16 covers r <= 16
                s = ltl.Simulation(gs, rule, method)
                if method != "direct":
                    s.autotune(probe_steps=10)
                s.step(50)
                secs_r, _ = timed_runs(s, 50, 1, torch)
                row[method] = side * side * 50 / secs_r
                s.close()
            sweep[str(r)] = row
        out["sweep"] = {"workload": f"{side}x{side}, r=1..{args.sweep_rmax} sweep rules, Bernoulli(0.5) seed 3, 50 steps",
                        "cell_updates_per_s": sweep}

    if args.shard > 1:
        out["shard"] = bench_shard(args, ltl, inputs, torch)

    # ---- the same workload on a torus (the paper's experimental boundary condition)
    sp = ltl.Simulation(g0, w.rule, "cat_i8", boundary="periodic")
    sp.set_tuning(**{k: tuning[k] for k in SHAPE_KEYS})
    sp.step(w.steps)
    psecs, _ = timed_runs(sp, w.steps, max(1, min(args.steps, 5)), torch)
    pd = ltl.Simulation(g0, w.rule, "direct", boundary="periodic")
    pc = ltl.Simulation(g0, w.rule, "cat_i8", boundary="periodic")
    pc.set_tuning(**{k: tuning[k] for k in SHAPE_KEYS})
    pd.step(w.steps)
    pc.step(w.steps)
    out["periodic"] = {"workload": "bosco4096 on a torus (periodic boundary)",
                       "value": cells * w.steps * max(1, min(args.steps, 5)) / psecs, "unit": "cell-updates/s",
                       "cat_vs_direct_equal": bool(torch.equal(pc.read(), pd.read()))}
    for x in (sp, pd, pc):
        x.close()

    if not args.no_batch:
        out["batched"] = bench_batch(args, ltl, inputs, torch)

    if args.life:
        out["life256"], life_init, life_final = bench_life(ltl, inputs, torch)
    if args.decay:
        out["decay"] = bench_decay(args, ltl, inputs, torch)
    if args.energy:
        out["energy"] = bench_energy(args, ltl, inputs, torch)

    if not args.no_cpu:
        import oracle

        threads = oracle.set_threads(0)
        t0 = time.perf_counter()
        one = oracle.run(g0_np, w.rule, 1)
        t1 = time.perf_counter() - t0
        n_cpu = int(max(1, min(w.steps - 1, 15.0 // max(t1, 1e-3))))
        t0 = time.perf_counter()
        res = oracle.run(one, w.rule, n_cpu)
        tc = time.perf_counter() - t0
        sample = f"bosco4096 grid, steps 2..{n_cpu + 1} of 100 ({n_cpu} steps, {t1 + tc:.1f} s total)"
        if n_cpu + 1 == w.steps:
            parity["cat_vs_oracle_equal"] = bool(np.array_equal(res, cat_final))
        # one thread, one step (the single-thread figure of the same oracle)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.run(one, w.rule, 1)
        t_single = time.perf_counter() - t0
        oracle.set_threads(threads)
        if args.life:
            lw = inputs.WORKLOADS["life256"]
            out["life256"]["cat_vs_oracle_equal"] = bool(np.array_equal(oracle.run(life_init, lw.rule, lw.steps),
                                                                         life_final))
        out["cpu_baseline"] = {"value": cells * n_cpu / tc, "unit": "cell-updates/s", "cores": threads,
                               "kind": "oracle", "sample": sample,
                               "single_thread_value": cells / t_single,
                               "cpu_model": cpu_model()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
