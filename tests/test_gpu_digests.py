"""Full-grid parity at the workloads' full sizes: every cell of the GPU grid after every step
against the oracle's grid, through digests.

``tests/golden/oracle_digests.json`` holds the XXH3-128 digest of the oracle's H x W grid
after every step of each workload (written by ``python -m oracle.digests``, which calls only
the oracle and the seeded generators). Here the library's grids are hashed the same way:
  * stepping one step per call (one-step launches), every step is compared;
  * stepping the whole run in one call, in the launch shape the benchmark times (the
    library's own pick from its tuning table), the final grid is compared, and with calls of
    steps_per_launch steps the grid after every launch.
A digest mismatch names the first differing step; the sampled-window tests in
test_gpu_fullsize.py then localise the cells.
"""
import json
import os

import numpy as np
import pytest
import xxhash

from paper_2406_17284_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DIGESTS = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")


def load_digests():
    try:
        with open(DIGESTS) as f:
            return json.load(f)
    except OSError:
        return {}


GOLD = load_digests()


@pytest.fixture(scope="module")
def ltl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_17284_amd import ltl as mod
    mod.load()
    return mod


def digest(t) -> str:
    a = np.ascontiguousarray(t.cpu().numpy())
    return xxhash.xxh3_128_hexdigest(memoryview(a).cast("B"))


def steps_of(name):
    w = GOLD.get(name)
    if not w:
        pytest.skip(f"no oracle digests recorded for {name}")
    return {e["step"]: e["digest"] for e in w["steps"]}


def check_every_step(ltl, g0, rule, name, method, steps):
    gold = steps_of(name)
    sim = ltl.Simulation(g0, rule, method)
    for k in range(1, steps + 1):
        sim.step(1)
        assert digest(sim.read()) == gold[k], f"{name} {method}: first differing step {k}"
    sim.close()


def check_launches_and_final(ltl, g0, rule, name, method, steps):
    """Calls of steps_per_launch steps (digest after each launch), then a fresh run of all
    steps in one call (graph replay)."""
    gold = steps_of(name)
    sim = ltl.Simulation(g0, rule, method)
    T = sim.tuning()["steps_per_launch"] if method != "direct" else 1
    done = 0
    while done < steps:
        n = min(T, steps - done)
        sim.step(n)
        done += n
        assert digest(sim.read()) == gold[done], f"{name} {method} T={T}: first differing launch ends at step {done}"
    sim.close()
    sim = ltl.Simulation(g0, rule, method)
    sim.step(steps)
    assert digest(sim.read()) == gold[steps], f"{name} {method}: {steps} steps in one call"
    assert not sim.current_padded()[:, sim.W:].any()
    sim.close()


# ------------------------------------------------------------------ Bosco R5 4096^2, 100 steps
@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8", "direct"])
def test_bosco4096_every_step(ltl, method):
    w = inputs.WORKLOADS["bosco4096"]
    g0 = inputs.bernoulli_grid_torch(w.H, w.W, w.p, w.seed, device="cuda")
    check_every_step(ltl, g0, w.rule, "bosco4096", method, w.steps)


def test_bosco4096_benchmark_shape(ltl):
    w = inputs.WORKLOADS["bosco4096"]
    g0 = inputs.bernoulli_grid_torch(w.H, w.W, w.p, w.seed, device="cuda")
    check_launches_and_final(ltl, g0, w.rule, "bosco4096", "cat_i8", w.steps)


# ------------------------------------------------------------------ radius sweep 16384^2, 50 steps
SWEEP_SIDE = 16384


@pytest.fixture(scope="module")
def sweep_grid(ltl):
    return inputs.bernoulli_grid_torch(SWEEP_SIDE, SWEEP_SIDE, 0.5, 3, device="cuda")


@pytest.mark.parametrize("r", list(range(1, 17)))
def test_sweep_int8_every_step(ltl, sweep_grid, r):
    w = inputs.sweep_workload(r)
    check_every_step(ltl, sweep_grid, w.rule, w.name, "cat_i8", w.steps)


@pytest.mark.parametrize("r", list(range(1, 17)))
def test_sweep_benchmark_shapes(ltl, sweep_grid, r):
    """int8 in the benchmark's shape launch by launch and in one call; fp16, fp8 (r <= 7) and the
    direct stencil over the whole run in one call."""
    w = inputs.sweep_workload(r)
    check_launches_and_final(ltl, sweep_grid, w.rule, w.name, "cat_i8", w.steps)
    gold = steps_of(w.name)
    for method in ["cat_f16", "direct"] + (["cat_f8"] if r <= 7 else []):
        sim = ltl.Simulation(sweep_grid, w.rule, method)
        sim.step(w.steps)
        assert digest(sim.read()) == gold[w.steps], f"{w.name} {method}"
        sim.close()


# ------------------------------------------------------------------ 512-instance batch, 32 steps
@pytest.fixture(scope="module")
def batch_grids(ltl):
    insts = inputs.batch_instances()
    return insts, [inputs.bernoulli_grid_torch(x.H, x.W, 0.5, x.seed, device="cuda") for x in insts]


def batch_digest(batch, n):
    h = xxhash.xxh3_128()
    for i in range(n):
        h.update(memoryview(np.ascontiguousarray(batch.read(i).cpu().numpy())).cast("B"))
    return h.hexdigest()


def test_batch512_every_step(ltl, batch_grids):
    insts, grids = batch_grids
    gold = steps_of("batch512")
    b = ltl.Batch(grids, [x.rule for x in insts], "cat_i8")
    for k in range(1, 33):
        b.step(1)
        assert batch_digest(b, len(insts)) == gold[k], f"batch512: first differing step {k}"
    b.close()


@pytest.mark.parametrize("method", ["cat_i8", "direct"])
def test_batch512_benchmark_shape_every_instance(ltl, batch_grids, method):
    """The benchmark's configuration (32 steps in one call, one hipGraph): every instance."""
    insts, grids = batch_grids
    if "batch512" not in GOLD:
        pytest.skip("no oracle digests recorded for batch512")
    gold = GOLD["batch512"]["instances"]
    b = ltl.Batch(grids, [x.rule for x in insts], method)
    b.step(32)
    bad = [i for i in range(len(insts)) if digest(b.read(i)) != gold[i]["digest"]]
    b.close()
    assert not bad, f"instances differing from the oracle after 32 steps: {bad[:20]}"


# ------------------------------------------------------------------ C = 8 decay, 32768^2, 20 steps
@pytest.mark.parametrize("name,p", [("decay32768", 0.5), ("decay32768_p042", 0.42)])
def test_decay32768_every_step(ltl, name, p):
    w = inputs.WORKLOADS["decay32768"]
    steps_of(name)
    g0 = inputs.bernoulli_grid_torch(w.H, w.W, p, w.seed, device="cuda")
    check_every_step(ltl, g0, w.rule, name, "cat_i8", w.steps)


@pytest.mark.parametrize("name,p", [("decay32768", 0.5), ("decay32768_p042", 0.42)])
def test_decay32768_benchmark_shape(ltl, name, p):
    w = inputs.WORKLOADS["decay32768"]
    steps_of(name)
    g0 = inputs.bernoulli_grid_torch(w.H, w.W, p, w.seed, device="cuda")
    check_launches_and_final(ltl, g0, w.rule, name, "cat_i8", w.steps)
    gold = steps_of(name)
    sim = ltl.Simulation(g0, w.rule, "direct")
    sim.step(w.steps)
    assert digest(sim.read()) == gold[w.steps], f"{name} direct"
    sim.close()
