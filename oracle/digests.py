"""Digests of oracle grids at the workloads' full sizes (test infrastructure only).

Writes ``tests/golden/oracle_digests.json``: for every workload below, the XXH3-128
digest (and the alive-cell count) of the oracle's H x W uint8 grid after every step.
The GPU parity tests hash the library's grids the same way and compare, so every
cell of every step of these full-size runs is checked against the plain definition
(direct box count with a dead ghost halo, then the transition), not only sampled
windows.

This script calls only the oracle (this package) and the seeded generators of
``paper_2406_17284_amd.inputs`` (which hold none of the method's arithmetic); no value
in the file comes from the HIP library.

Workloads (the seeded recipes of ``inputs``):
  bosco4096        R5 C0 M1 S34..58 B34..45, 4096^2, Bernoulli(0.5) seed 2, steps 1..100
  sweep16384_r{r}  sweep rule of radius r = 1..16, 16384^2, Bernoulli(0.5) seed 3, steps 1..50
  batch512         the 512-instance batch: per step 1..32 one digest of all instance grids
                   in instance order, and per instance the digest after step 32
  decay32768       R16 C8 M0 S300..500 B330..420, 32768^2, Bernoulli(0.5) seed 5, steps 1..20
  decay32768_p042  the same rule and seed at Bernoulli(0.42), where births, survivals and
                   decay chains all persist over the 20 steps (at 0.5 every alive cell dies
                   in step 1 and the grid is empty from step 8 on)

Usage: ``python -m oracle.digests [--threads N] [--only name,name,...]``. The full set
takes about two hours of oracle time on 6 cores; results are merged into the file
after each workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import xxhash

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import oracle  # noqa: E402
from paper_2406_17284_amd import inputs  # noqa: E402

OUT = os.path.join(_ROOT, "tests", "golden", "oracle_digests.json")
DIGEST = "xxh3_128 of the H x W uint8 grid, row-major, no padding"


def digest(grid: np.ndarray) -> str:
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    return xxhash.xxh3_128_hexdigest(memoryview(g).cast("B"))


def alive(grid: np.ndarray) -> int:
    return int(np.count_nonzero(grid == 1))


def single(name: str, H: int, W: int, rule, seed: int, p: float, steps: int) -> dict:
    g = inputs.bernoulli_grid(H, W, p, seed)
    per_step = []
    t0 = time.time()
    for k in range(1, steps + 1):
        g = oracle.step(g, rule)
        per_step.append({"step": k, "digest": digest(g), "alive": alive(g)})
        print(f"{name} step {k}/{steps} alive {per_step[-1]['alive']} ({time.time() - t0:.0f} s)", flush=True)
    return {"H": H, "W": W, "rule": rule.text(), "seed": seed, "p": p, "steps": per_step}


def batch(steps: int = 32) -> dict:
    insts = inputs.batch_instances()
    grids = [inputs.bernoulli_grid(x.H, x.W, 0.5, x.seed) for x in insts]
    per_step = []
    t0 = time.time()
    for k in range(1, steps + 1):
        grids = [oracle.step(g, x.rule) for g, x in zip(grids, insts)]
        h = xxhash.xxh3_128()
        for g in grids:
            h.update(memoryview(np.ascontiguousarray(g)).cast("B"))
        per_step.append({"step": k, "digest": h.hexdigest(), "alive": sum(alive(g) for g in grids)})
        print(f"batch512 step {k}/{steps} ({time.time() - t0:.0f} s)", flush=True)
    return {"count": len(insts), "seed": 4, "p": 0.5, "steps": per_step,
            "instances": [{"index": i, "H": x.H, "W": x.W, "rule": x.rule.text(), "seed": x.seed,
                           "digest": digest(g), "alive": alive(g)}
                          for i, (x, g) in enumerate(zip(insts, grids))]}


def jobs():
    bos = inputs.WORKLOADS["bosco4096"]
    dec = inputs.WORKLOADS["decay32768"]
    out = [("bosco4096", lambda: single("bosco4096", bos.H, bos.W, bos.rule, bos.seed, 0.5, bos.steps)),
           ("batch512", batch)]
    for r in range(1, 17):
        w = inputs.sweep_workload(r)
        out.append((w.name, lambda w=w: single(w.name, w.H, w.W, w.rule, w.seed, 0.5, w.steps)))
    out.append(("decay32768", lambda: single("decay32768", dec.H, dec.W, dec.rule, dec.seed, 0.5, dec.steps)))
    out.append(("decay32768_p042",
                lambda: single("decay32768_p042", dec.H, dec.W, dec.rule, dec.seed, 0.42, dec.steps)))
    return out


def load_existing() -> dict:
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save(data: dict) -> None:
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", default="")
    a = ap.parse_args(argv)
    if a.threads:
        oracle.set_threads(a.threads)
    only = set(x for x in a.only.split(",") if x)
    data = load_existing()
    data["_about"] = {"digest": DIGEST, "writer": "python -m oracle.digests (calls only oracle/ and inputs)"}
    for name, fn in jobs():
        if only and name not in only:
            continue
        t0 = time.time()
        data[name] = fn()
        data[name]["oracle_seconds"] = round(time.time() - t0, 1)
        save(data)
        print(f"== {name} done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
