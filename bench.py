"""Benchmark: Larger-than-Life cell-updates/s on one MI355X, CAT int8-MFMA vs the LDS direct stencil.

Headline (``value``): the Bosco-type rule R5 C0 M1 S34..58 B34..45 N_M on a 4096 x 4096 uint8
grid (Bernoulli(0.5), seed 2, dead ghost halo), one bench step = ``ltl_step(100)`` with the
grid resident in HBM, the launch shape the library picks by itself (tuning table). Timing:
``--warmup`` untimed bench steps, then ``--steps`` repetitions, each restarting from the same
initial grid and timed with HIP events on the simulation's stream; the median is reported.

Also measured by default (each with its own median over repetitions restarting from its
initial grid, bit-exactness against the oracle's digests, and a CPU-oracle baseline):
  * sweep: the radius sweep r = 1..16 on 16384^2 (50 steps, sweep rules), CAT int8, int8 at
    one step per launch, fp16, fp8 (r <= 7) and the direct stencil;
  * life256: Life on 256^2, 64 steps;
  * batched: the 512-instance batch, 32 steps (one hipGraph);
  * decay: the C = 8 R16 rule on 32768^2, 20 steps;
  * periodic: the headline workload on a torus;
  * energy: cell-updates per joule of CAT int8 and the direct stencil, Bosco R5 on 32768^2.
Prints one JSON line on stdout (progress goes to stderr).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-life] [--no-batch] [--no-decay]
                  [--no-cpu] [--tuning T,rows,cols,waves[,persistent[,lds_pad]]] [--no-energy] [--shard N]
                  [--only sweep|batch|decay|life [--sweep-radii ...] [--sweep-methods ...]]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s vs radius r=1..16, CAT int8-MFMA vs direct stencil, bit-exact"
PEAK_TOPS = {"cat_i8": 5000.0, "cat_f8": 5000.0, "cat_f16": 2500.0}   # MI355X dense MFMA, per element type
HBM_PEAK_GBS = 8000.0
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9   # int32 lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
OPS_PER_CELL = 256       # two 16x16x64 int8 MFMAs per 256 cells, 2 ops per multiply-add
KERNEL_SRC = [os.path.join(ROOT, "paper_2406_17284_amd", "csrc", f) for f in ("cat_device.h", "cat_kernel.hip")]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "cat_step_i8_bosco4096_traffic.json")
MFMA_RECORD = os.path.join(ROOT, "profiles", "cat_step_i8_bosco4096_sq.json")
DIGESTS = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
SHAPE_KEYS = ("steps_per_launch", "tile_rows", "tile_cols", "waves", "persistent", "lds_pad")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def parse_tuning(text):
    """'T,tile_rows,tile_cols,waves[,persistent[,lds_pad]]' -> keyword arguments of set_tuning."""
    vals = [int(x) for x in text.split(",")]
    return dict(zip(SHAPE_KEYS, vals))


def _shape(tuning):
    return [int(tuning.get(k, 0)) for k in SHAPE_KEYS]


def _record(path, tuning, field):
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256") != kernel_hash() or list(rec.get("tuning", []))[:len(SHAPE_KEYS)] + \
            [0] * (len(SHAPE_KEYS) - len(rec.get("tuning", []))) != _shape(tuning):
        return None
    return rec[field]


def recorded_traffic(tuning):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter record, if it was
    taken on this kernel source and launch shape; else None."""
    return _record(TRAFFIC_RECORD, tuning, "hbm_bytes_per_launch")


def recorded_mfma_ops(tuning):
    """int8 MFMA ops issued per launch (SQ_INSTS_VALU_MFMA_MOPS_I8 x 512) from the committed
    counter record, if it was taken on this kernel source and launch shape; else None."""
    return _record(MFMA_RECORD, tuning, "mfma_ops_per_launch")


def mfma_issued(tuning, avg_launch_s, cells, r):
    """Counter-measured MFMA utilisation of the timed kernel: int8 ops the MFMAs issue per
    launch (committed SQ counter record) over launch time x peak, and the useful fraction:
    the band non-zeros, 4(2r+1) ops per cell-update, over the ops issued per cell-update."""
    ops = recorded_mfma_ops(tuning)
    if ops is None:
        return None
    steps = tuning["steps_per_launch"]
    issued_per_cell = ops / (cells * steps)
    return {"ops_per_launch": ops, "frac_of_peak": ops / avg_launch_s / (PEAK_TOPS["cat_i8"] * 1e12),
            "issued_ops_per_cell_update": issued_per_cell,
            "useful_ops_per_cell_update": 4 * (2 * r + 1),
            "useful_frac": 4 * (2 * r + 1) / issued_per_cell}


def cpu_model() -> str:
    """/proc/cpuinfo's model name with its family / model / stepping numbers (a virtualised host
    may report only the product line) and the CPUs this process may run on."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = (x.strip() for x in line.split(":", 1))
                    if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                        info[k] = v
                if not line.strip() and info:
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 0
    name = info.get("model name", "unknown")
    ids = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return f"{name} ({ids}; {usable} CPUs usable by this process)" if ids else f"{name} ({usable} CPUs usable)"


def load_digests():
    try:
        with open(DIGESTS) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def digest_of(t) -> str:
    import numpy as np
    import xxhash

    a = np.ascontiguousarray(t.cpu().numpy())
    return xxhash.xxh3_128_hexdigest(memoryview(a).cast("B"))


def golden(digests, name, step):
    """The oracle's digest of workload `name` after `step` steps, or None if not recorded."""
    w = digests.get(name)
    if not w:
        return None
    for e in w.get("steps", []):
        if e["step"] == step:
            return e["digest"]
    return None


# ------------------------------------------------------------------------------ timing
def time_reps(stream, run, reset, reps, torch):
    """Seconds of `reps` runs of `run()` (HIP events on `stream`), each after `reset()` restored
    the initial state outside the timed region."""
    out = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        ev0.record(stream)
        run()
        ev1.record(stream)
        torch.cuda.synchronize()
        out.append(ev0.elapsed_time(ev1) / 1e3)
    return out


def sim_reset(sim, g0):
    def reset():
        sim.current_padded()[:, :sim.W].copy_(g0)
    return reset


def batch_reset(b, g0s):
    def reset():
        for i, g in enumerate(g0s):
            b.current_padded(i)[:, :b.W[i]].copy_(g)
    return reset


def sim_rate(ltl, torch, g0, rule, method, steps, reps, tuning=None, boundary="dead", warmup=1):
    """Median seconds per `steps`-step run (restarting from g0 each time), the final grid after
    `steps` steps, the launch shape and the per-run times."""
    sim = ltl.Simulation(g0, rule, method, tuning=tuning, boundary=boundary)
    reset = sim_reset(sim, g0)
    for _ in range(warmup):
        reset()
        sim.step(steps)
    times = time_reps(sim.stream, lambda: sim.step(steps), reset, reps, torch)
    final = sim.read()
    tun = sim.tuning()
    sim.close()
    return statistics.median(times), final, tun, times


# ------------------------------------------------------------------------------ CPU oracle
def oracle_rates(oracle, inputs, grid_fn, rule, steps_all, steps_one, rows_one=None):
    """Cell-updates/s of the oracle on all host threads (steps_all steps of grid_fn()) and on one
    thread (steps_one steps of the first rows_one rows, extrapolated per cell-update)."""
    import numpy as np

    g = grid_fn()
    threads = oracle.set_threads(0)
    t0 = time.perf_counter()
    res = oracle.run(g, rule, steps_all)
    t_all = time.perf_counter() - t0
    sub = np.ascontiguousarray(g[:rows_one]) if rows_one else g
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run(sub, rule, steps_one)
    t_one = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": g.size * steps_all / t_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "single_thread_value": sub.size * steps_one / t_one, "seconds_all_cores": t_all,
            "seconds_single_thread": t_one}, res


# ------------------------------------------------------------------------------ legs
def bench_sweep(args, ltl, inputs, torch, digests, oracle):
    side, steps, reps = args.sweep_side, 50, args.leg_reps or 5
    g = inputs.bernoulli_grid_torch(side, side, 0.5, 3, device="cuda")
    cells = side * side
    per_r = {}
    t1_shape = dict(steps_per_launch=1, tile_rows=160, tile_cols=224, waves=8)
    radii = [int(x) for x in args.sweep_radii.split(",")] if args.sweep_radii else range(1, args.sweep_rmax + 1)
    methods = args.sweep_methods.split(",") if args.sweep_methods else ("cat_i8", "cat_i8_T1", "cat_f16", "cat_f8",
                                                                          "direct")
    if args.no_direct:
        methods = [m for m in methods if m != "direct"]
    for r in radii:
        w = inputs.sweep_workload(r, side)
        ref = golden(digests, w.name, steps) if side == 16384 else None
        row = {}
        for method in methods:
            m = "cat_i8" if method == "cat_i8_T1" else method
            # the one-step row (a fixed 8-wave shape) covers the radii of the flatness claim, 1..16
            if (m == "cat_f8" and r > 7) or (m == "cat_f16" and r > 16) or (method == "cat_i8_T1" and r > 16):
                continue
            med, final, tun, _ = sim_rate(ltl, torch, g, w.rule, m, steps, reps if m != "direct" else min(reps, 3),
                                          tuning=t1_shape if method == "cat_i8_T1" else None)
            rate = cells * steps / med
            ent = {"cell_updates_per_s": rate, "ms_per_run": med * 1e3}
            if m in PEAK_TOPS:
                launches = math.ceil(steps / tun["steps_per_launch"])
                ent["frac"] = OPS_PER_CELL * rate / (PEAK_TOPS[m] * 1e12)
                ent["avg_launch_us"] = med / launches * 1e6
                ent["tuning"] = [tun[k] for k in SHAPE_KEYS]
            else:
                ent["frac_valu"] = (2 * r + 1) ** 2 * rate / VALU_PEAK_OPS
            ent["bit_exact"] = None if ref is None else digest_of(final) == ref
            row[method] = ent
            del final
        if "cat_i8" in row and "direct" in row:
            row["cat_over_direct"] = row["cat_i8"]["cell_updates_per_s"] / row["direct"]["cell_updates_per_s"]
        per_r[str(r)] = row
        log(f"sweep r={r}: " + ", ".join(f"{m} {v['cell_updates_per_s']:.3e}" for m, v in row.items()
                                          if isinstance(v, dict)))
    res = {"workload": f"sweep{side}: {side}x{side}, radii {list(radii)} of the sweep rules (S=[0.25,0.45]N, "
                       f"B=[0.27,0.34]N floored), Bernoulli(0.5) seed 3, dead halo, {steps} steps per run",
           "reps": reps, "per_r": per_r}
    i8 = [per_r[k]["cat_i8"]["cell_updates_per_s"] for k in per_r if "cat_i8" in per_r[k]]
    t1 = [per_r[k]["cat_i8_T1"]["cell_updates_per_s"] for k in per_r if "cat_i8_T1" in per_r[k]]
    if i8:
        res["int8_max_over_min"] = max(i8) / min(i8)
    if t1:
        res["int8_T1_max_over_min"] = max(t1) / min(t1)
        res["int8_T1_shape"] = [t1_shape.get(k, 0) for k in SHAPE_KEYS]
    if all("cat_over_direct" in per_r[k] for k in per_r):
        wins = [int(k) for k in per_r if per_r[k]["cat_over_direct"] > 1]
        res["cat_beats_direct_from_r"] = min(wins) if wins else None
        res["cat_beats_direct_at_every_r"] = len(wins) == len(per_r)
    exact = [v.get("bit_exact") for k in per_r for v in per_r[k].values() if isinstance(v, dict)]
    res["bit_exact_all"] = all(e is True for e in exact) if all(e is not None for e in exact) else None
    del g
    if oracle is not None:
        # all cores: 2 steps of a 2048-row strip of the sweep grid per sampled radius; one
        # thread: 1 step of its first 128 rows (extrapolated per cell-update)
        cpu = {}
        for r in [x for x in (1, 5, 9, 16) if x in list(radii)] or [list(radii)[0]]:
            rule = inputs.sweep_rule(r)
            rates, _ = oracle_rates(oracle, inputs, lambda: inputs.bernoulli_grid(2048, side, 0.5, 3), rule, 2, 1,
                                    rows_one=128)
            cpu[str(r)] = rates
        res["cpu_baseline"] = {"per_r": cpu, "kind": "oracle", "unit": "cell-updates/s",
                               "cores": next(iter(cpu.values()))["cores"], "cpu_model": cpu_model(),
                               "sample": "per r in {1, 5, 9, 16}: all cores = 2 steps of a 2048 x 16384 strip; one "
                                         "thread = 1 step of a 128 x 16384 strip, extrapolated per cell-update"}
    return res


def bench_life(args, ltl, inputs, torch, digests):
    w = inputs.WORKLOADS["life256"]
    g = torch.from_numpy(inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)).cuda()
    med, final, tun, _ = sim_rate(ltl, torch, g, w.rule, "cat_i8", w.steps, 20, warmup=3)
    return {"workload": f"life256: R1 C0 M1 S3..4 B3..3 N_M, 256x256, Bernoulli(0.5) seed {w.seed}, dead halo, "
                        f"{w.steps} steps per run", "reps": 20, "tuning": [tun[k] for k in SHAPE_KEYS],
            "us_per_run": med * 1e6, "value": w.H * w.W * w.steps / med, "unit": "cell-updates/s"}, final


def bench_batch(args, ltl, inputs, torch, digests, oracle):
    insts = inputs.batch_instances()
    steps, reps = 32, args.leg_reps or 5
    dev = [inputs.bernoulli_grid_torch(x.H, x.W, 0.5, x.seed, device="cuda") for x in insts]
    rules = [x.rule for x in insts]
    cells = sum(x.H * x.W for x in insts)
    res = {"workload": "batch512: 512 instances, sides log-uniform in [128, 2048], r uniform in 1..16, S/B uniform "
                       "in [0.2, 0.5] x (2r+1)^2, M1, Bernoulli(0.5), dead halo, 32 steps per run (one hipGraph)",
           "cells": cells, "reps": reps}
    out = {}
    for method in ("cat_i8",) if args.no_direct else ("cat_i8", "direct"):
        b = ltl.Batch(dev, rules, method)
        reset = batch_reset(b, dev)
        reset()
        b.step(steps)
        times = time_reps(b.stream, lambda: b.step(steps), reset, reps if method == "cat_i8" else min(reps, 2), torch)
        med = statistics.median(times)
        out[method] = cells * steps / med
        if method == "cat_i8":
            res["ms_per_run"] = med * 1e3
            res["tuning"] = [b.tuning()[k] for k in SHAPE_KEYS]
            gold = digests.get("batch512", {}).get("instances")
            if gold:
                res["bit_exact"] = all(digest_of(b.read(i)) == gold[i]["digest"] for i in range(len(insts)))
            else:
                res["bit_exact"] = None
        b.close()
    res["value"] = out["cat_i8"]
    res["unit"] = "cell-updates/s"
    res["frac"] = OPS_PER_CELL * out["cat_i8"] / (PEAK_TOPS["cat_i8"] * 1e12)
    if "direct" in out:
        res["direct_stencil_cell_updates_per_s"] = out["direct"]
        res["cat_over_direct"] = out["cat_i8"] / out["direct"]
    if oracle is not None:
        import numpy as np

        # the first 16 instances: all cores over 32 steps, one thread over 2 steps
        sample = list(range(16))
        threads = oracle.set_threads(0)
        grids = [inputs.bernoulli_grid(insts[i].H, insts[i].W, 0.5, insts[i].seed) for i in sample]
        n = sum(g.size for g in grids)
        t0 = time.perf_counter()
        for g, i in zip(grids, sample):
            oracle.run(g, insts[i].rule, steps)
        t_all = time.perf_counter() - t0
        oracle.set_threads(1)
        t0 = time.perf_counter()
        for g, i in zip(grids, sample):
            oracle.run(np.ascontiguousarray(g), insts[i].rule, 2)
        t_one = time.perf_counter() - t0
        oracle.set_threads(threads)
        res["cpu_baseline"] = {"value": n * steps / t_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
                               "single_thread_value": n * 2 / t_one, "cpu_model": cpu_model(),
                               "sample": "instances 0..15 of the batch: all cores over 32 steps; one thread over 2 "
                                         "steps, extrapolated per cell-update"}
    return res


def bench_decay(args, ltl, inputs, torch, digests, oracle):
    w = inputs.WORKLOADS["decay32768"]
    g = inputs.bernoulli_grid_torch(w.H, w.W, w.p, w.seed, device="cuda")
    cells = w.H * w.W
    res = {"workload": f"decay32768: R16 C8 M0 S300..500 B330..420 N_M, 32768x32768, Bernoulli(0.5) seed {w.seed}, "
                       f"dead halo, {w.steps} steps per run", "reps": args.leg_reps or 5}
    ref = golden(digests, "decay32768", w.steps)
    med, final, tun, _ = sim_rate(ltl, torch, g, w.rule, "cat_i8", w.steps, args.leg_reps or 5)
    res["value"] = cells * w.steps / med
    res["unit"] = "cell-updates/s"
    res["ms_per_run"] = med * 1e3
    res["frac"] = OPS_PER_CELL * res["value"] / (PEAK_TOPS["cat_i8"] * 1e12)
    res["tuning"] = [tun[k] for k in SHAPE_KEYS]
    res["bit_exact"] = None if ref is None else digest_of(final) == ref
    res["alive_after_run"] = int((final == 1).sum().item())
    del final
    # At density 0.5 nearly every box count exceeds both ranges: the grid decays to all-dead
    # within about 8 steps. The kernel's work does not depend on the cells, but the same rule is
    # also timed at density 0.42, where births, survivals and decay go on for all 20 steps.
    g42 = inputs.bernoulli_grid_torch(w.H, w.W, 0.42, w.seed, device="cuda")
    ref42 = golden(digests, "decay32768_p042", w.steps)
    med42, final42, _, _ = sim_rate(ltl, torch, g42, w.rule, "cat_i8", w.steps, args.leg_reps or 5)
    res["live_density_042"] = {"value": cells * w.steps / med42, "unit": "cell-updates/s", "ms_per_run": med42 * 1e3,
                               "alive_after_run": int((final42 == 1).sum().item()),
                               "bit_exact": None if ref42 is None else digest_of(final42) == ref42}
    del final42, g42
    if not args.no_direct:
        med_d, final_d, _, _ = sim_rate(ltl, torch, g, w.rule, "direct", w.steps, 1, warmup=0)
        res["direct_stencil_cell_updates_per_s"] = cells * w.steps / med_d
        res["direct_bit_exact"] = None if ref is None else digest_of(final_d) == ref
        res["cat_over_direct"] = res["value"] / res["direct_stencil_cell_updates_per_s"]
        del final_d
    del g
    if oracle is not None:
        rates, _ = oracle_rates(oracle, inputs, lambda: inputs.bernoulli_grid(1024, w.W, 0.5, w.seed), w.rule, 2, 1,
                                rows_one=64)
        res["cpu_baseline"] = dict(rates, cpu_model=cpu_model(),
                                   sample="all cores = 2 steps of a 1024 x 32768 strip of the grid; one thread = 1 "
                                          "step of a 64 x 32768 strip, extrapolated per cell-update")
    return res


XGMI_LINK_GBS = 153.0   # one xGMI link of an MI355X, one direction (published figure)


def bench_shard(args, ltl, inputs, torch):
    """One GPU's share of the radius-sweep grid split N = `args.shard` ways: the CAT int8 rate on
    a (side/N) x side row strip and on a 2-D block of the same size next to the whole grid's, and
    the halo a strip would trade with each neighbour per launch (r * T rows of `side` bytes, one
    xGMI link per neighbour). The exchange time is the link model, not a measurement: this
    library runs on one GPU."""
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
            med, _, tun, _ = sim_rate(ltl, torch, g, rule, "cat_i8", 50, 3)
            row[name + "_cell_updates_per_s"] = g.shape[0] * g.shape[1] * 50 / med
            if name == "strip":
                T = tun["steps_per_launch"]
                row["strip_tuning"] = [tun[k] for k in SHAPE_KEYS]
                launch_s = med / (50 / T)
        halo = r * T * side
        row["halo_bytes_per_edge_per_launch"] = halo
        row["launch_us"] = launch_s * 1e6
        row["exchange_us_model"] = halo / (XGMI_LINK_GBS * 1e9) * 1e6
        res["per_r"][str(r)] = row
        log(f"shard r={r} done")
    return res


def gpu_energy_reader(torch):
    """Returns the amdsmi handle of the GPU HIP runs on, or raises."""
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
    return amdsmi, handle


class EnergyMeter:
    """Joules drawn by the GPU over a span: the board's energy accumulator where it advances,
    else the integral of the reported socket power sampled every 20 ms by a host thread."""

    def __init__(self, torch):
        import threading
        self.smi, self.h = gpu_energy_reader(torch)
        self.threading = threading

    def counter(self):
        e = self.smi.amdsmi_get_energy_count(self.h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6

    def power_w(self):
        p = self.smi.amdsmi_get_power_info(self.h)
        for key in ("current_socket_power", "average_socket_power", "socket_power"):
            v = p.get(key)
            if isinstance(v, (int, float)) and 0 < v < 10000:
                return float(v)
        raise RuntimeError(f"no socket power in {sorted(p)}")

    def measure(self, fn, min_seconds=4.0):
        """Runs fn() until at least min_seconds have passed (the accumulator advances in coarse
        steps); returns (seconds, runs, joules, source, sampled_joules)."""
        samples, stop = [], self.threading.Event()

        def sampler():
            while not stop.is_set():
                try:
                    samples.append((time.perf_counter(), self.power_w()))
                except Exception:
                    pass
                stop.wait(0.02)
        th = self.threading.Thread(target=sampler, daemon=True)
        c0, t0 = self.counter(), time.perf_counter()
        th.start()
        runs = 0
        while True:
            fn()
            runs += 1
            if time.perf_counter() - t0 >= min_seconds:
                break
        t1 = time.perf_counter()
        c1 = self.counter()
        stop.set()
        th.join()
        sampled = None
        if len(samples) >= 2:
            sampled = sum((b[0] - a[0]) * 0.5 * (a[1] + b[1]) for a, b in zip(samples, samples[1:]))
            sampled *= (t1 - t0) / max(1e-9, samples[-1][0] - samples[0][0])
        if c1 > c0:
            return t1 - t0, runs, c1 - c0, "energy accumulator", sampled
        if sampled is None:
            raise RuntimeError("the energy accumulator did not advance and no power samples were read")
        return t1 - t0, runs, sampled, "socket power sampled every 20 ms", sampled


def bench_energy(args, ltl, inputs, torch):
    """Energy efficiency (cell-updates per joule) at the largest workload grid: Bosco R5 on
    32768^2, CAT int8 (1000-step runs) and the direct stencil (100-step runs), each repeated
    for at least 4 s between readings of the GPU's energy counter (or integrated sampled power),
    and the idle draw over a span of the same length."""
    try:
        meter = EnergyMeter(torch)
        meter.counter()
    except Exception as e:   # no energy reading on this machine: report why instead
        return {"error": f"{type(e).__name__}: {e}"}
    side, rule = 32768, inputs.BOSCO_M1
    g = inputs.bernoulli_grid_torch(side, side, 0.5, 6, device="cuda")
    res = {"workload": "Bosco R5 C0 M1 S34..58 B34..45 N_M on 32768x32768, Bernoulli(0.5) seed 6, dead halo",
           "source": "amdsmi (whole board), around synchronized runs"}
    torch.cuda.synchronize()
    try:
        secs, _, joules, src, _ = meter.measure(lambda: time.sleep(0.5))
        res["idle_W"] = joules / secs
        res["idle_source"] = src
        for method, steps in (("cat_i8", 1000), ("direct", 100)):
            s = ltl.Simulation(g, rule, method)
            s.step(steps // 10)
            torch.cuda.synchronize()

            def run():
                s.step(steps)
                torch.cuda.synchronize()
            secs, runs, joules, src, sampled = meter.measure(run)
            n = side * side * steps * runs
            res[method] = {"steps": steps * runs, "seconds": secs, "joules": joules, "avg_W": joules / secs,
                           "energy_source": src,
                           "sampled_avg_W": None if sampled is None else sampled / secs,
                           "cell_updates_per_s": n / secs, "cell_updates_per_J": n / joules,
                           "cell_updates_per_J_above_idle": n / max(1e-9, joules - res["idle_W"] * secs)}
            s.close()
    except Exception as e:
        res["error"] = f"{type(e).__name__}: {e}"
        return res
    res["cat_over_direct_per_J"] = res["cat_i8"]["cell_updates_per_J"] / res["direct"]["cell_updates_per_J"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed repetitions of the headline run (median reported)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed headline runs first (GPU clocks settle)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the radius sweep r=1..16 on 16384^2")
    ap.add_argument("--sweep-side", type=int, default=16384)
    ap.add_argument("--sweep-rmax", type=int, default=16)
    ap.add_argument("--sweep-radii", type=str, default="", help="comma-separated radii of the sweep (default 1..rmax)")
    ap.add_argument("--sweep-methods", type=str, default="",
                    help="comma-separated subset of cat_i8, cat_i8_T1, cat_f16, cat_f8, direct")
    ap.add_argument("--no-life", action="store_true", help="skip the Life 256^2 workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-instance batched workload")
    ap.add_argument("--no-decay", action="store_true", help="skip the C=8 R16 decay workload on 32768^2")
    ap.add_argument("--no-periodic", action="store_true", help="skip the headline workload on a torus")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baselines")
    ap.add_argument("--shard", type=int, default=0, metavar="N",
                    help="also time one GPU's row strip (1/N) of the sweep grid and the halo it would exchange")
    ap.add_argument("--no-energy", action="store_true",
                    help="skip the cell-updates per joule leg (CAT int8 and direct, Bosco R5 on 32768^2)")
    ap.add_argument("--energy", action="store_true", help=argparse.SUPPRESS)   # the leg is on by default
    ap.add_argument("--tuning", type=str, default="",
                    help="T,tile_rows,tile_cols,waves[,persistent[,lds_pad]] for the headline (default: the "
                         "library's own pick from its tuning table)")
    ap.add_argument("--leg-reps", type=int, default=0, metavar="N",
                    help="timed repetitions of each sweep / batch / decay measurement (default: 5)")
    ap.add_argument("--no-direct", action="store_true",
                    help="leave out the direct-stencil comparison runs (profiler runs of the CAT kernels)")
    ap.add_argument("--only", choices=("sweep", "batch", "decay", "life"), default="",
                    help="run this one workload alone (no headline, no CPU baselines) and print its record; "
                         "for profiler runs whose kernel averages must cover that workload only")
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

    import torch

    from paper_2406_17284_amd import inputs, ltl

    oracle = None
    if not args.no_cpu:
        import oracle as oracle_mod

        oracle_mod.use_native()   # the oracle as it stands, compiled -O3 -march=native for this host
        oracle = oracle_mod

    torch.cuda.set_device(0)
    digests = load_digests()
    if args.only:
        legs = {"sweep": bench_sweep, "batch": bench_batch, "decay": bench_decay}
        if args.only == "life":
            rec, _ = bench_life(args, ltl, inputs, torch, digests)
        else:
            rec = legs[args.only](args, ltl, inputs, torch, digests, None)
        print(json.dumps({"only": args.only, "record": rec}), flush=True)
        return
    w = inputs.WORKLOADS["bosco4096"]
    g0_np = inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)
    g0 = torch.from_numpy(g0_np).cuda()
    cells = w.H * w.W
    t_wall0 = time.perf_counter()

    # ---- headline: CAT int8 on the Bosco workload
    sim = ltl.Simulation(g0, w.rule, "cat_i8", tuning=parse_tuning(args.tuning) if args.tuning else None)
    tuning = sim.tuning()
    for _ in range(args.warmup):
        sim.step(w.steps)
    reset = sim_reset(sim, g0)
    times = time_reps(sim.stream, lambda: sim.step(w.steps), reset, args.steps, torch)
    secs = statistics.median(times)
    cat_final = sim.read()
    sim.close()
    value = cells * w.steps / secs
    launches_per_run = math.ceil(w.steps / tuning["steps_per_launch"])
    avg_launch_s = secs / launches_per_run
    ops_per_launch = OPS_PER_CELL * cells * w.steps / launches_per_run
    achieved_tops = ops_per_launch / avg_launch_s / 1e12
    ref100 = golden(digests, "bosco4096", w.steps)
    log(f"headline: {value:.4e} cell-updates/s, {avg_launch_s * 1e6:.2f} us per launch")

    # ---- direct stencil, same workload
    if args.no_direct:
        direct_value = None
        parity = {"cat_vs_direct_equal": None}
    else:
        dsecs, direct_final, _, _ = sim_rate(ltl, torch, g0, w.rule, "direct", w.steps, 3)
        direct_value = cells * w.steps / dsecs
        parity = {"cat_vs_direct_equal": bool(torch.equal(cat_final, direct_final))}
        del direct_final
    parity["cat_vs_oracle_digest"] = None if ref100 is None else digest_of(cat_final) == ref100

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": "bosco4096: R5 C0 M1 S34..58 B34..45 N_M, 4096x4096 uint8, Bernoulli(0.5) seed 2, "
                        "dead ghost halo, 100 LTL steps per bench step",
            "method": "cat_i8",
            "timing": f"median of {args.steps} runs, each restarting from the initial grid, after {args.warmup} "
                      "untimed runs; HIP events on the simulation's stream",
            "tuning": [tuning[k] for k in SHAPE_KEYS],
            "tuning_source": "--tuning" if args.tuning else "library default (tuning table)",
            "run_ms_min_max": [min(times) * 1e3, max(times) * 1e3],
            "direct_stencil_cell_updates_per_s": direct_value,
            # one byte read + one written per cell-update
            "direct_stencil_algorithmic_GBs": None if direct_value is None else 2 * direct_value / 1e9,
            "direct_stencil_frac_valu": None if direct_value is None else
            (2 * w.rule.R + 1) ** 2 * direct_value / VALU_PEAK_OPS,
            "cat_over_direct": None if direct_value is None else value / direct_value,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved_tops,
            "peak": PEAK_TOPS["cat_i8"],
            "unit": "TFLOP/s",
            "frac": achieved_tops / PEAK_TOPS["cat_i8"],
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

    if not args.no_periodic:
        psecs, pfinal, _, _ = sim_rate(ltl, torch, g0, w.rule, "cat_i8", w.steps, 5, boundary="periodic")
        dpsecs, dpfinal, _, _ = sim_rate(ltl, torch, g0, w.rule, "direct", w.steps, 1, boundary="periodic", warmup=0)
        out["periodic"] = {"workload": "bosco4096 on a torus (periodic boundary, the paper's experimental setting)",
                           "value": cells * w.steps / psecs, "unit": "cell-updates/s",
                           "direct_stencil_cell_updates_per_s": cells * w.steps / dpsecs,
                           "cat_vs_direct_equal": bool(torch.equal(pfinal, dpfinal))}
        del pfinal, dpfinal
        log("periodic done")
    if not args.no_life:
        out["life256"], life_final = bench_life(args, ltl, inputs, torch, digests)
        log("life done")
    if not args.no_sweep:
        out["sweep"] = bench_sweep(args, ltl, inputs, torch, digests, oracle)
    if not args.no_batch:
        out["batched"] = bench_batch(args, ltl, inputs, torch, digests, oracle)
        log("batch done")
    if not args.no_decay:
        out["decay"] = bench_decay(args, ltl, inputs, torch, digests, oracle)
        log("decay done")
    if args.shard > 1:
        out["shard"] = bench_shard(args, ltl, inputs, torch)
    if not args.no_energy:
        out["energy"] = bench_energy(args, ltl, inputs, torch)
        log("energy done")

    if oracle is not None:
        # the headline workload: all 100 steps on every host thread (also the parity of the timed
        # grid against the oracle itself), one thread over 2 steps (extrapolated per cell-update)
        rates, ref = oracle_rates(oracle, inputs, lambda: g0_np, w.rule, w.steps, 2)
        import numpy as np

        parity["cat_vs_oracle_equal"] = bool(np.array_equal(ref, cat_final.cpu().numpy()))
        out["cpu_baseline"] = dict(rates, cpu_model=cpu_model(),
                                   sample="bosco4096: all cores over the 100 steps of a bench step; one thread over "
                                          "steps 1..2, extrapolated per cell-update")
        if not args.no_life:
            lw = inputs.WORKLOADS["life256"]
            lrates, lref = oracle_rates(oracle, inputs, lambda: inputs.bernoulli_grid(lw.H, lw.W, lw.p, lw.seed),
                                        lw.rule, lw.steps, lw.steps)
            out["life256"]["cat_vs_oracle_equal"] = bool(np.array_equal(lref, life_final.cpu().numpy()))
            out["life256"]["cpu_baseline"] = dict(lrates, sample="life256: all 64 steps, all cores and one thread")
    out["config"]["wall_s"] = time.perf_counter() - t_wall0
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
