"""GPU parity of the dataflow form (tuning persistent = 2): one cooperative launch per step call,
every tile's workgroup resident, neighbouring tiles synchronised by per-tile round counters.

The bar is the same as for every other launch shape: every cell equal to the CPU oracle (and, at
the full Bosco 4096^2 size, to the oracle's digests), with steps split across calls, rounds whose
last one is shorter, dead and periodic boundaries, every epilogue and element type. Also the
refusals of shapes the form cannot run and the report of a wait that runs out (forced from the
host with a spin limit of zero polls: every workgroup still finishes)."""
import json
import os

import numpy as np
import pytest
import xxhash

import oracle
from paper_2406_17284_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ltl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_17284_amd import ltl as mod
    mod.load()
    return mod


def flow(T, rows, cols, waves=8):
    return dict(steps_per_launch=T, tile_rows=rows, tile_cols=cols, waves=waves, persistent=2)


def run(ltl, g0, rule, method, chunks, tuning, boundary="dead"):
    sim = ltl.Simulation(torch.from_numpy(np.ascontiguousarray(g0)).cuda(), rule, method, tuning=tuning,
                         boundary=boundary)
    assert sim.tuning()["persistent"] == 2
    for n in chunks:
        sim.step(n)
    got = sim.read().cpu().numpy()
    pad = sim.current_padded().cpu().numpy()
    sim.close()
    ref = oracle.run(g0, rule, sum(chunks), periodic=(boundary == "periodic"))
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"{method} {rule.text()} {tuning} {boundary} chunks={chunks}: {len(bad)} cells differ, "
                             f"first {bad[:5].tolist()}")
    assert not pad[:, g0.shape[1]:].any()


CASES = [
    # (rule, method, H, W, flow shape, step chunks, boundary)
    (inputs.BOSCO_M1, "cat_i8", 700, 900, flow(4, 160, 224), [13], "dead"),
    (inputs.BOSCO_M1, "cat_i8", 700, 900, flow(4, 160, 224), [3, 8, 1, 9], "dead"),
    (inputs.LIFE, "cat_i8", 256, 256, flow(8, 64, 64), [64], "dead"),
    (inputs.LIFE, "cat_i8", 300, 272, flow(6, 64, 96, 4), [17, 6], "periodic"),
    (inputs.Rule(2, 0, 1, 7, 13, 8, 11), "cat_i8", 333, 517, flow(5, 96, 128), [21], "dead"),
    (inputs.Rule(8, 0, 1, 72, 130, 78, 98), "cat_i8", 640, 704, flow(3, 128, 192), [10], "dead"),     # windowed epilogue
    (inputs.Rule(16, 0, 1, 272, 490, 294, 370), "cat_i8", 500, 640, flow(2, 128, 192), [7], "dead"),  # 16-bit epilogue
    (inputs.Rule(16, 8, 0, 300, 500, 330, 420), "cat_i8", 400, 512, flow(2, 128, 192), [9], "dead"),  # decay
    (inputs.Rule(5, 0, 1, 34, 58, 34, 45), "cat_i8", 480, 448, flow(4, 160, 224), [11], "periodic"),
    (inputs.Rule(7, 0, 1, 56, 101, 60, 76), "cat_f16", 300, 400, flow(3, 128, 96), [8], "dead"),
    (inputs.Rule(3, 0, 1, 12, 22, 13, 16), "cat_f8", 300, 400, flow(4, 128, 192), [9], "dead"),
    (inputs.Rule(20, 0, 1, 400, 700, 450, 560), "cat_i8", 400, 448, flow(1, 128, 160), [5], "dead"),  # radius > 16
    (inputs.Rule(4, 0, 1, 3, 6, 4, 5, "N"), "cat_i8", 300, 320, flow(4, 64, 128), [9], "dead"),        # cross
]


@pytest.mark.parametrize("rule,method,H,W,tuning,chunks,boundary", CASES)
def test_flow_matches_oracle(ltl, rule, method, H, W, tuning, chunks, boundary):
    p = 0.42 if rule.C > 2 else 0.5
    g0 = inputs.bernoulli_grid(H, W, p, seed=H * 7 + W)
    print(f"flow {method} {rule.text()} {H}x{W} {tuning} {chunks} {boundary}", flush=True)
    run(ltl, g0, rule, method, chunks, tuning, boundary)


def test_flow_each_step_and_after_other_shapes(ltl):
    """Single steps, then a switch between the dataflow form and the per-launch forms on one
    handle (the round counters only grow, so an earlier launch's values never satisfy a wait)."""
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(500, 600, 0.5, seed=9)
    sim = ltl.Simulation(torch.from_numpy(g0).cuda(), rule, "cat_i8", tuning=flow(4, 160, 224))
    ref = g0.copy()
    plan = [(1, flow(4, 160, 224)), (1, None), (5, flow(2, 128, 192)),
            (3, dict(steps_per_launch=3, tile_rows=160, tile_cols=224, waves=8, persistent=0)),
            (7, flow(4, 160, 224)), (4, dict(steps_per_launch=2, tile_rows=128, tile_cols=128, waves=8, persistent=1)),
            (9, flow(3, 96, 128))]
    for n, tun in plan:
        if tun is not None:
            sim.set_tuning(**tun)
        sim.step(n)
        ref = oracle.run(ref, rule, n)
        got = sim.read().cpu().numpy()
        assert np.array_equal(got, ref), f"after {n} steps with {tun}: {(got != ref).sum()} cells differ"
    sim.close()


def test_flow_bosco4096_digests(ltl):
    """The benchmark workload at full size in the dataflow form: the grid after every 4-step
    launch and after all 100 steps in one call against the oracle's digests."""
    with open(os.path.join(ROOT, "tests", "golden", "oracle_digests.json")) as f:
        gold = {e["step"]: e["digest"] for e in json.load(f)["bosco4096"]["steps"]}
    w = inputs.WORKLOADS["bosco4096"]
    g0 = inputs.bernoulli_grid_torch(w.H, w.W, w.p, w.seed, device="cuda")

    def digest(t):
        return xxhash.xxh3_128_hexdigest(memoryview(np.ascontiguousarray(t.cpu().numpy())).cast("B"))

    sim = ltl.Simulation(g0, w.rule, "cat_i8", tuning=flow(4, 160, 224))
    for k in range(1, 26):
        sim.step(4)
        assert digest(sim.read()) == gold[4 * k], f"first differing launch ends at step {4 * k}"
    sim.close()
    sim = ltl.Simulation(g0, w.rule, "cat_i8", tuning=flow(4, 160, 224))
    sim.step(100)
    assert digest(sim.read()) == gold[100]
    sim.close()


def test_flow_refusals(ltl):
    g = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    sim = ltl.Simulation(g, inputs.BOSCO_M1, "cat_i8")
    # more tiles than the device holds at once (4096 / 64 squared = 4096 tiles)
    with pytest.raises(ltl.LtlError) as e:
        sim.set_tuning(**flow(1, 64, 64, 4))
    assert e.value.code == ltl.LTL_ERR_ARG
    # a margin wider than the tile (r = 5, T = 8: 64 > 32 rows)
    with pytest.raises(ltl.LtlError):
        sim.set_tuning(**flow(8, 32, 224))
    with pytest.raises(ltl.LtlError):   # persistent must be 0, 1 or 2
        sim.set_tuning(steps_per_launch=4, tile_rows=160, tile_cols=224, waves=8, persistent=3)
    sim.close()
    # torus with a partial edge tile narrower than the margin (4096 = 18 x 224 + 64; L = 32 fits,
    # 4000 = 17 x 224 + 192 fits; 3600 = 16 x 224 + 16 does not)
    g = torch.zeros((512, 3600), dtype=torch.uint8, device="cuda")
    sim = ltl.Simulation(g, inputs.BOSCO_M1, "cat_i8", boundary="periodic")
    with pytest.raises(ltl.LtlError):
        sim.set_tuning(**flow(4, 160, 224))
    sim.close()
    # and the direct method has no dataflow form
    with pytest.raises(ltl.LtlError):
        ltl.Simulation(torch.zeros((64, 64), dtype=torch.uint8, device="cuda"), inputs.LIFE, "direct",
                       tuning=dict(steps_per_launch=1, tile_rows=64, tile_cols=64, waves=4, persistent=2))


def test_flow_timeout_is_reported(ltl, monkeypatch):
    """A spin limit of zero polls makes every wait that finds a neighbour not yet done count as
    timed out; the launch still ends normally and the next call reports the error."""
    monkeypatch.setenv("LTL_FLOW_SPIN_LIMIT", "0")
    g0 = inputs.bernoulli_grid_torch(4096, 4096, 0.5, 2, device="cuda")
    reported = False
    for attempt in range(3):   # a timeout needs one wait that is not already satisfied
        sim = ltl.Simulation(g0, inputs.BOSCO_M1, "cat_i8", tuning=flow(1, 160, 224))
        sim.step(64)
        torch.cuda.synchronize()
        try:
            sim.step(0)
        except ltl.LtlError as e:
            assert e.code == ltl.LTL_ERR_HIP and "timed out" in str(e)
            reported = True
        sim.close()
        if reported:
            break
    assert reported
    # with the default limit the same run is exact again
    monkeypatch.delenv("LTL_FLOW_SPIN_LIMIT")
    sim = ltl.Simulation(g0, inputs.BOSCO_M1, "cat_i8", tuning=flow(1, 160, 224))
    sim.step(3)
    got = sim.read().cpu().numpy()
    sim.close()
    ref = oracle.run(g0.cpu().numpy(), inputs.BOSCO_M1, 3)
    assert np.array_equal(got, ref)
