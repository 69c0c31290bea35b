"""GPU parity: the HIP library against the CPU oracle, cell for cell.

Counts are integers computed exactly (int8 MFMA with int32 accumulation), so the bar is
bit-exact equality of every cell after every step checked.
"""
import numpy as np
import pytest

import oracle
from paper_2406_17284_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ltl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_17284_amd import ltl as mod
    mod.load()
    return mod


def gpu_grid(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_and_compare_each_step(ltl, g0, rule, method, steps, tuning=None):
    sim = ltl.Simulation(gpu_grid(g0), rule, method, tuning=tuning)
    ref = g0.copy()
    for t in range(steps):
        sim.step(1)
        ref = oracle.step(ref, rule)
        got = sim.read().cpu().numpy()
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)
            raise AssertionError(f"{method} {rule.text()} tuning={tuning}: step {t + 1} differs at "
                                 f"{len(bad)} cells, first {bad[:5].tolist()}")
    sim.close()
    return ref


def run_and_compare(ltl, g0, rule, method, steps, tuning=None, chunks=None):
    sim = ltl.Simulation(gpu_grid(g0), rule, method, tuning=tuning)
    for n in (chunks or [steps]):
        sim.step(n)
    got = sim.read().cpu().numpy()
    pad = sim.current_padded().cpu().numpy()
    sim.close()
    ref = oracle.run(g0, rule, steps)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"{method} {rule.text()} tuning={tuning}: after {steps} steps {len(bad)} cells "
                             f"differ, first {bad[:5].tolist()}")
    # padding columns of the library layout stay dead
    assert not pad[:, g0.shape[1]:].any()


METHODS = ["cat_i8", "direct"]
ALL_METHODS = ["cat_i8", "cat_f16", "cat_f8", "direct"]


def f8_refuses(ltl, rule):
    """fp8-e4m3 counts are exact only for 2r+1 <= 16: larger radii must be refused."""
    if rule.R <= 7:
        return False
    with pytest.raises(ltl.LtlError) as e:
        ltl.Simulation(gpu_grid(np.zeros((8, 8), dtype=np.uint8)), rule, "cat_f8")
    assert e.value.code == ltl.LTL_ERR_INEXACT
    return True

SMALL_RULES = [
    inputs.LIFE,
    inputs.Rule(1, 2, 0, 2, 3, 3, 3),
    inputs.Rule(2, 0, 1, 7, 13, 8, 11),
    inputs.Rule(3, 0, 0, 15, 23, 14, 17),
    inputs.BOSCO_M1,
    inputs.Rule(5, 0, 0, 35, 59, 34, 45),
    inputs.Rule(6, 0, 1, 42, 76, 45, 57),
    inputs.Rule(8, 2, 0, 163, 223, 74, 252),
    inputs.Rule(11, 0, 1, 132, 238, 142, 179),
    inputs.Rule(16, 0, 0, 170, 296, 170, 300),
    inputs.Rule(16, 0, 1, 272, 490, 294, 370),
    inputs.Rule(3, 4, 1, 12, 22, 13, 16),
    inputs.Rule(16, 8, 0, 300, 500, 330, 420),
    inputs.Rule(2, 0, 1, 0, 3, 0, 2),      # birth at count 0: the dead halo must not be born
    inputs.Rule(4, 0, 1, 30, 10, 21, 27),  # empty survival range
]


@pytest.mark.parametrize("method", ALL_METHODS)
@pytest.mark.parametrize("rule", SMALL_RULES, ids=lambda r: r.text())
def test_every_step_small_ragged(ltl, method, rule):
    if method == "cat_f8" and f8_refuses(ltl, rule):
        return
    g0 = inputs.bernoulli_grid(83, 151, 0.5, seed=rule.R * 7 + rule.C)
    run_and_compare_each_step(ltl, g0, rule, method, 6)


@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (37, 1), (16, 32), (17, 33), (255, 257), (300, 65)])
@pytest.mark.parametrize("method", ALL_METHODS)
def test_shapes(ltl, shape, method):
    rule = inputs.Rule(3, 0, 1, 12, 22, 13, 16)
    g0 = inputs.bernoulli_grid(shape[0], shape[1], 0.5, seed=shape[0] * 1000 + shape[1])
    run_and_compare(ltl, g0, rule, method, 5)


def shape_feasible(r, T, TH, TW, waves=8, maxc=14, cell=1, lds_max=160 * 1024):
    """Whether the CAT kernel can run this launch shape: the LDS state tile fits and in every
    step the 32-column strips times the row segments (at most `maxc` 16-row blocks) fit the
    waves. int8 above r = 16 reads two more H blocks per segment (11 output blocks, margin
    + 32); cell = 2 marks fp16, which has no wide variant."""
    wide = r > 16 and cell == 1 and maxc == 14
    if wide:
        maxc = 9
    margin = -(-r * (T - 1) // 16) * 16 + (48 if wide else 16)
    rows, cols = TH + 2 * margin, TW + 2 * margin
    lds = -(-rows * (cols + 16) // 1024) * 1024
    if lds > lds_max:
        return False
    for t in range(1, T + 1):
        E = -(-r * (T - t) // 16) * 16
        nstrips = (TW + 2 * E) // 32
        nseg = -(-((TH + 2 * E) // 16) // maxc)
        if nstrips * nseg > waves:
            return False
    return True


@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8"])
@pytest.mark.parametrize("T", [1, 2, 3, 4, 7])
@pytest.mark.parametrize("r", [1, 2, 5, 6, 9, 16])
def test_temporal_blocking(ltl, T, r, method):
    rule = inputs.sweep_rule(r)
    if method == "cat_f8" and f8_refuses(ltl, rule):
        return
    g0 = inputs.bernoulli_grid(200, 333, 0.5, seed=100 + r)
    tuning = dict(steps_per_launch=T, tile_rows=64, tile_cols=64, waves=0)
    maxc = 5 if method == "cat_f16" else 14
    cell = 2 if method == "cat_f16" else 1
    if not shape_feasible(r, T, 64, 64, maxc=maxc, cell=cell):
        # the library must refuse a launch shape it cannot run
        with pytest.raises(ltl.LtlError) as e:
            run_and_compare(ltl, g0, rule, method, 9, tuning=tuning)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_and_compare(ltl, g0, rule, method, 9, tuning=tuning)


@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8"])
@pytest.mark.parametrize("T", [8, 12, 16, 33, 64])
@pytest.mark.parametrize("r", [1, 2])
def test_long_temporal_blocking(ltl, T, r, method):
    """Steps per launch above 7 (the autotuner takes T = 8 at r = 1) up to the 64 the tuning
    accepts: 2T + 3 steps (two whole launches and a shorter one) equal the oracle, on a dead halo
    and (int8) on a torus; launch shapes the kernel cannot hold are refused."""
    rule = inputs.sweep_rule(r)
    g0 = inputs.bernoulli_grid(200, 333, 0.5, seed=200 + r)
    n = 2 * T + 3
    tuning = dict(steps_per_launch=T, tile_rows=64, tile_cols=64, waves=0)
    maxc = 5 if method == "cat_f16" else 14
    if not shape_feasible(r, T, 64, 64, maxc=maxc):
        with pytest.raises(ltl.LtlError) as e:
            run_and_compare(ltl, g0, rule, method, n, tuning=tuning)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_and_compare(ltl, g0, rule, method, n, tuning=tuning)
    if method == "cat_i8":
        run_periodic(ltl, inputs.bernoulli_grid(208, 336, 0.5, seed=300 + r), rule, method, n, tuning=tuning,
                     every_step=False)


TALL_RULES = [inputs.sweep_rule(3), inputs.sweep_rule(12), inputs.Rule(6, 5, 0, 30, 70, 35, 50)]


@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8"])
@pytest.mark.parametrize("tile", [(512, 32), (448, 96), (320, 64), (272, 128)], ids=lambda t: f"{t[0]}x{t[1]}")
@pytest.mark.parametrize("rule", TALL_RULES, ids=lambda r: r.text())
def test_tall_tiles(ltl, rule, tile, method):
    """Tiles taller than one row segment (a 32-column strip split over several waves), up to the
    512 rows the tuning accepts, over byte, windowed and decay epilogues; a ragged last tile row
    (1100 = 2 x 512 + 76). Shapes the kernel cannot hold are refused."""
    if method == "cat_f8" and f8_refuses(ltl, rule):
        return
    g0 = (inputs.state_grid(1100, 150, rule.C, seed=31) if rule.C >= 3
          else inputs.bernoulli_grid(1100, 150, 0.5, seed=31))
    maxc = 5 if method == "cat_f16" else 14
    for T in (1, 3):
        tuning = dict(steps_per_launch=T, tile_rows=tile[0], tile_cols=tile[1], waves=0)
        if not shape_feasible(rule.R, T, *tile, maxc=maxc):
            with pytest.raises(ltl.LtlError) as e:
                run_and_compare(ltl, g0, rule, method, 7, tuning=tuning)
            assert e.value.code == ltl.LTL_ERR_ARG
            continue
        run_and_compare(ltl, g0, rule, method, 7, tuning=tuning)


@pytest.mark.parametrize("tile", [(16, 32), (32, 64), (64, 64), (128, 128), (48, 96), (192, 128), (128, 224), (80, 224)])
def test_tile_shapes(ltl, tile):
    rule = inputs.Rule(7, 0, 1, 56, 101, 60, 76)
    g0 = inputs.bernoulli_grid(301, 299, 0.5, seed=5)
    for T in (1, 3):
        tuning = dict(steps_per_launch=T, tile_rows=tile[0], tile_cols=tile[1], waves=0)
        run_and_compare(ltl, g0, rule, "cat_i8", 7, tuning=tuning)


# The fixed shape class (224-column tiles, 32-cell margin, 8 waves: separate kernel copies with
# these constants compiled in, 160-row tiles with the height fixed too): every epilogue, both
# tile heights, several tile rows and columns with ragged edges, launches of T steps and a
# shorter last launch.
FIXED_CLASS_CASES = [
    (inputs.sweep_rule(5), 4),                         # byte lanes
    (inputs.sweep_rule(5), 2),
    (inputs.sweep_rule(8), 3),                         # 7-bit window
    (inputs.sweep_rule(16), 2),                        # full-byte window
    (inputs.Rule(10, 0, 1, 100, 354, 120, 200), 2),    # span 255: 16-bit lanes
    (inputs.Rule(5, 12, 1, 34, 58, 34, 45), 4),        # decay, C > 8
    (inputs.Rule(5, 6, 0, 30, 60, 34, 45), 3),         # decay tables, C <= 8
    (inputs.Rule(16, 8, 0, 300, 500, 330, 420), 2),    # decay tables, full-byte window
]


@pytest.mark.parametrize("rows", [160, 192])
@pytest.mark.parametrize("case", FIXED_CLASS_CASES, ids=lambda c: f"{c[0].text()}-T{c[1]}")
def test_fixed_shape_class(ltl, case, rows):
    rule, T = case
    assert 1 <= rule.R * (T - 1) <= 16   # a 32-cell margin
    g0 = inputs.bernoulli_grid(700, 700, 0.5, seed=rule.R + 3 * T)
    tuning = dict(steps_per_launch=T, tile_rows=rows, tile_cols=224, waves=8)
    run_and_compare(ltl, g0, rule, "cat_i8", 2 * T + 1, tuning=tuning)


def test_fixed_shape_class_periodic(ltl):
    g0 = inputs.bernoulli_grid(700, 704, 0.5, seed=11)
    tuning = dict(steps_per_launch=4, tile_rows=160, tile_cols=224, waves=8)
    run_periodic(ltl, g0, inputs.sweep_rule(5), "cat_i8", 9, tuning=tuning, every_step=False)


def test_wave_count_must_cover_the_strips(ltl):
    g0 = inputs.bernoulli_grid(64, 64, 0.5, seed=1)
    sim = ltl.Simulation(gpu_grid(g0), inputs.Rule(7, 0, 1, 56, 101, 60, 76), "cat_i8")
    with pytest.raises(ltl.LtlError) as e:
        sim.set_tuning(steps_per_launch=3, tile_rows=64, tile_cols=128, waves=2)
    assert e.value.code == ltl.LTL_ERR_ARG
    sim.set_tuning(steps_per_launch=3, tile_rows=64, tile_cols=128, waves=0)
    assert sim.tuning()["waves"] == 8
    sim.close()


@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8"])
def test_decay_multistep(ltl, method):
    rule = inputs.Rule(5, 6, 0, 30, 54, 32, 41)
    g0 = inputs.state_grid(190, 230, 6, seed=12)
    for T in (1, 2, 4):
        run_and_compare(ltl, g0, rule, method, 8, tuning=dict(steps_per_launch=T, waves=0))
    run_and_compare(ltl, g0, rule, "direct", 8)


def test_resume_and_graph_chunks(ltl):
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(260, 270, 0.5, seed=77)
    tuning = dict(steps_per_launch=3, tile_rows=64, tile_cols=64, waves=0)
    run_and_compare(ltl, g0, rule, "cat_i8", 17, tuning=tuning, chunks=[0, 5, 1, 11, 0])
    run_and_compare(ltl, g0, rule, "cat_i8", 17, tuning=dict(tuning, use_graph=0), chunks=[5, 12])


@pytest.mark.parametrize("method", ["cat_i8", "direct"])
def test_long_runs_span_several_step_chunks(ltl, method):
    """A call runs as chunks of at most 64 launches (one cached graph each): 150 one-step launches
    (64 + 64 + 22) and 197 steps at three per launch (192 + 5), with and without graphs and split
    across calls, equal the oracle."""
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(128, 150, 0.5, seed=83)
    T = 1 if method == "direct" else 3
    n = 150 if T == 1 else 197
    base = dict(steps_per_launch=T) if method == "direct" else dict(steps_per_launch=T, tile_rows=64, tile_cols=64)
    for use_graph in (1, 0):
        run_and_compare(ltl, g0, rule, method, n, tuning=dict(base, use_graph=use_graph))
    run_and_compare(ltl, g0, rule, method, n, tuning=dict(base, use_graph=1), chunks=[130, n - 130])
    if method == "cat_i8":
        run_and_compare(ltl, g0, rule, method, 150, tuning=dict(base, steps_per_launch=1, use_graph=1))


def test_side_stream_and_read_into(ltl):
    """A handle on its own stream, created from a non-contiguous tensor (the binding's contiguous
    copy is made on the current stream), reads into a caller's tensor; a tensor of the wrong
    shape, type or layout is refused before any copy."""
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(150, 130, 0.5, seed=91)
    src = gpu_grid(np.ascontiguousarray(g0.T)).t()          # g0 as a transposed view
    assert not src.is_contiguous()
    side = torch.cuda.Stream()
    sim = ltl.Simulation(src, rule, "cat_i8", stream=side)
    sim.step(7)
    out = torch.full((150, 130), 255, dtype=torch.uint8, device="cuda")
    assert sim.read(out) is out
    side.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.run(g0, rule, 7))
    for bad in (torch.empty((150, 129), dtype=torch.uint8, device="cuda"),
                torch.empty((150, 130), dtype=torch.int32, device="cuda"),
                torch.empty((130, 150), dtype=torch.uint8, device="cuda").t(),
                torch.empty((150, 130), dtype=torch.uint8)):
        with pytest.raises(ValueError):
            sim.read(bad)
    sim.close()
    batch = ltl.Batch([gpu_grid(g0)], [rule], "cat_i8", stream=side)
    batch.step(7)
    with pytest.raises(ValueError):
        batch.read(0, torch.empty((150, 131), dtype=torch.uint8, device="cuda"))
    out2 = batch.read(0)
    side.synchronize()
    assert torch.equal(out2, out)
    batch.close()


def test_life_256_every_step(ltl):
    w = inputs.WORKLOADS["life256"]
    g0 = inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)
    for method in METHODS:
        run_and_compare_each_step(ltl, g0, w.rule, method, w.steps)


def test_life_patterns_on_gpu(ltl):
    # a glider crossing tile borders keeps its shape and velocity
    g0 = np.zeros((100, 100), dtype=np.uint8)
    g0[1:4, 1:4] = np.array([[0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=np.uint8)
    sim = ltl.Simulation(gpu_grid(g0), inputs.LIFE, "cat_i8", tuning=dict(steps_per_launch=4, tile_rows=32, tile_cols=32))
    sim.step(80)
    got = sim.read().cpu().numpy()
    sim.close()
    assert np.array_equal(got, np.roll(np.roll(g0, 20, 0), 20, 1))


def test_bosco_4096_full(ltl):
    """The Bosco workload in full (4096^2, 100 steps) against the oracle: CAT int8 in the launch
    shape the benchmark times (the library's own pick), the same shape in its persistent form,
    a fixed T = 4 160 x 224 shape, and the direct stencil."""
    w = inputs.WORKLOADS["bosco4096"]
    g0 = inputs.bernoulli_grid(w.H, w.W, w.p, w.seed)
    oracle.set_threads(0)
    ref = oracle.run(g0, w.rule, w.steps)
    probe = ltl.Simulation(gpu_grid(g0), w.rule, "cat_i8")
    timed = probe.tuning()
    probe.close()
    fixed = dict(steps_per_launch=4, tile_rows=160, tile_cols=224, waves=8)
    for method, tuning in (("cat_i8", timed), ("cat_i8", dict(timed, persistent=1)), ("cat_i8", fixed),
                           ("direct", None)):
        sim = ltl.Simulation(gpu_grid(g0), w.rule, method, tuning=tuning)
        sim.step(w.steps)
        got = sim.read().cpu().numpy()
        sim.close()
        assert np.array_equal(got, ref), (method, tuning)


# ------------------------------------------------------------------ periodic boundary (torus)
PERIODIC_SHAPES = [(16, 16), (1, 16), (5, 32), (48, 64), (83, 160), (200, 336)]
PERIODIC_RULES = [inputs.LIFE, inputs.BOSCO_M1, inputs.Rule(9, 0, 0, 90, 160, 97, 122),
                  inputs.Rule(3, 5, 1, 12, 22, 13, 16), inputs.Rule(16, 0, 1, 272, 490, 294, 370),
                  inputs.Rule(6, 0, 1, 42, 76, 45, 57)]


def run_periodic(ltl, g0, rule, method, steps, tuning=None, every_step=True):
    sim = ltl.Simulation(gpu_grid(g0), rule, method, tuning=tuning, boundary="periodic")
    ref = g0.copy()
    for t in range(steps if every_step else 1):
        n = 1 if every_step else steps
        sim.step(n)
        ref = oracle.run(ref, rule, n, periodic=True)
        got = sim.read().cpu().numpy()
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)
            raise AssertionError(f"periodic {method} {rule.text()} {g0.shape} tuning={tuning}: step {t + 1} "
                                 f"differs at {len(bad)} cells, first {bad[:5].tolist()}")
    assert not sim.current_padded()[:, g0.shape[1]:].any()
    sim.close()


@pytest.mark.parametrize("method", ALL_METHODS)
@pytest.mark.parametrize("rule", PERIODIC_RULES, ids=lambda r: r.text())
@pytest.mark.parametrize("shape", PERIODIC_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_periodic_every_step(ltl, method, rule, shape):
    if method == "cat_f8" and f8_refuses(ltl, rule):
        return
    H, W = shape
    g0 = (inputs.state_grid(H, W, rule.C, seed=H * 1000 + W) if rule.C >= 3
          else inputs.bernoulli_grid(H, W, 0.5, seed=H * 1000 + W))
    run_periodic(ltl, g0, rule, method, 4)


@pytest.mark.parametrize("method", ["cat_i8", "cat_f16"])
@pytest.mark.parametrize("T", [2, 3, 5, 7])
@pytest.mark.parametrize("r", [1, 5, 16])
def test_periodic_temporal_blocking(ltl, method, T, r):
    rule = inputs.sweep_rule(r)
    g0 = inputs.bernoulli_grid(200, 336, 0.5, seed=300 + r)
    tuning = dict(steps_per_launch=T, tile_rows=64, tile_cols=64, waves=0)
    maxc = 5 if method == "cat_f16" else 14
    cell = 2 if method == "cat_f16" else 1
    if not shape_feasible(r, T, 64, 64, maxc=maxc, cell=cell):
        # the library must refuse a launch shape it cannot run
        with pytest.raises(ltl.LtlError) as e:
            run_periodic(ltl, g0, rule, method, 9, tuning=tuning, every_step=False)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_periodic(ltl, g0, rule, method, 9, tuning=tuning, every_step=False)
    # a torus smaller than the loaded window (margins wrap several times)
    run_periodic(ltl, inputs.bernoulli_grid(24, 32, 0.5, seed=301 + r), rule, method, 7, tuning=tuning,
                 every_step=False)


def test_periodic_needs_width_multiple_of_16(ltl):
    sim = ltl.Simulation(gpu_grid(np.zeros((8, 40), dtype=np.uint8)), inputs.LIFE, "cat_i8")
    with pytest.raises(ltl.LtlError) as e:
        ltl.ltl_set_boundary(sim.handle, ltl.LTL_BOUNDARY_PERIODIC)
    assert e.value.code == ltl.LTL_ERR_UNSUPPORTED
    sim.close()


def test_periodic_glider_wraps_on_gpu(ltl):
    g0 = np.zeros((32, 48), dtype=np.uint8)
    g0[1:4, 1:4] = np.array([[0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=np.uint8)   # moves (+1, +1) per 4 steps
    for method in ("cat_i8", "direct"):
        sim = ltl.Simulation(gpu_grid(g0), inputs.LIFE, method, boundary="periodic")
        sim.step(4 * 96)          # lcm(32, 48) = 96 periods of (1, 1)
        assert np.array_equal(sim.read().cpu().numpy(), g0), method
        sim.close()


# ------------------------------------------------------------------ radius 17..32 (int8 wide)
WIDE_RULES = [inputs.sweep_rule(17), inputs.Rule(20, 5, 1, 300, 700, 320, 500), inputs.Rule(24, 0, 0, 600, 1100, 650, 900),
              inputs.Rule(31, 0, 1, 990, 1800, 1070, 1360), inputs.Rule(32, 0, 1, 1056, 1901, 1140, 1436)]


@pytest.mark.parametrize("method", ["cat_i8", "direct"])
@pytest.mark.parametrize("rule", WIDE_RULES, ids=lambda r: r.text())
def test_wide_radius_every_step(ltl, method, rule):
    g0 = (inputs.state_grid(83, 151, rule.C, seed=rule.R) if rule.C >= 3
          else inputs.bernoulli_grid(83, 151, 0.5, seed=rule.R))
    run_and_compare_each_step(ltl, g0, rule, method, 4)


@pytest.mark.parametrize("T", [1, 2, 3])
@pytest.mark.parametrize("r", [17, 24, 32])
@pytest.mark.parametrize("tile", [(64, 64), (128, 96), (48, 160)], ids=lambda t: f"{t[0]}x{t[1]}")
def test_wide_radius_launch_shapes(ltl, T, r, tile):
    rule = inputs.sweep_rule(r)
    g0 = inputs.bernoulli_grid(230, 301, 0.5, seed=500 + r)
    tuning = dict(steps_per_launch=T, tile_rows=tile[0], tile_cols=tile[1], waves=0)
    if not shape_feasible(r, T, tile[0], tile[1]):
        with pytest.raises(ltl.LtlError) as e:
            run_and_compare(ltl, g0, rule, "cat_i8", 5, tuning=tuning)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_and_compare(ltl, g0, rule, "cat_i8", 5, tuning=tuning)


def test_wide_radius_periodic(ltl):
    rule = inputs.sweep_rule(24)
    run_periodic(ltl, inputs.bernoulli_grid(64, 80, 0.5, seed=24), rule, "cat_i8", 3)
    run_periodic(ltl, inputs.bernoulli_grid(150, 208, 0.5, seed=25), rule, "cat_i8", 5,
                 tuning=dict(steps_per_launch=2, tile_rows=64, tile_cols=64), every_step=False)


def test_wide_radius_refusals(ltl):
    g = gpu_grid(np.zeros((8, 8), dtype=np.uint8))
    for method, code in (("cat_f16", ltl.LTL_ERR_UNSUPPORTED), ("cat_f8", ltl.LTL_ERR_INEXACT)):
        with pytest.raises(ltl.LtlError) as e:
            ltl.Simulation(g, inputs.sweep_rule(17), method)
        assert e.value.code == code
    with pytest.raises(ltl.LtlError) as e:
        ltl.Simulation(g, inputs.Rule(33, 0, 1, 1, 2, 1, 2), "cat_i8")
    assert e.value.code == ltl.LTL_ERR_RULE
    with pytest.raises(ltl.LtlError) as e:
        ltl.Batch([g, g], [inputs.LIFE, inputs.sweep_rule(17)], "cat_i8")
    assert e.value.code == ltl.LTL_ERR_UNSUPPORTED


def test_graph_replays_match_eager(ltl):
    """The cached hipGraph of an n-step call is replayed several times, with eager work (reads,
    a single eager step, synchronizations) between the replays; every replay must equal the
    eager launches of the same steps."""
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(300, 420, 0.5, seed=61)
    tun = dict(steps_per_launch=2, tile_rows=64, tile_cols=128)
    graph = ltl.Simulation(gpu_grid(g0), rule, "cat_i8", tuning=dict(tun, use_graph=1))
    eager = ltl.Simulation(gpu_grid(g0), rule, "cat_i8", tuning=dict(tun, use_graph=0))
    for k in range(4):
        graph.step(6)       # same n and parity each time: the same cached graph
        eager.step(6)
        torch.cuda.synchronize()
        a, b = graph.read(), eager.read()
        assert torch.equal(a, b), f"replay {k}"
        graph.step(2)        # eager-sized calls between the replays (two launches: a second graph)
        eager.step(2)
        _ = graph.read().sum().item()
    assert np.array_equal(graph.read().cpu().numpy(), oracle.run(g0, rule, 32))
    graph.close()
    eager.close()


# ------------------------------------------------------------------ cross neighbourhood (N_N)
CROSS_RULES = [inputs.Rule(1, 0, 1, 2, 3, 3, 3, "N"), inputs.Rule(2, 0, 0, 2, 5, 3, 4, "N"),
               inputs.Rule(5, 4, 1, 5, 12, 6, 9, "N"), inputs.Rule(9, 0, 1, 10, 22, 12, 17, "N"),
               inputs.Rule(16, 0, 1, 17, 40, 20, 30, "N"), inputs.Rule(7, 0, 1, 20, 10, 8, 14, "N")]


@pytest.mark.parametrize("method", ["cat_i8", "direct"])
@pytest.mark.parametrize("rule", CROSS_RULES, ids=lambda r: r.text())
def test_cross_every_step(ltl, method, rule):
    g0 = (inputs.state_grid(83, 151, rule.C, seed=rule.R + 40) if rule.C >= 3
          else inputs.bernoulli_grid(83, 151, 0.5, seed=rule.R + 40))
    run_and_compare_each_step(ltl, g0, rule, method, 4)


@pytest.mark.parametrize("T", [2, 3, 5])
@pytest.mark.parametrize("tile", [(64, 64), (96, 128), (32, 192)], ids=lambda t: f"{t[0]}x{t[1]}")
@pytest.mark.parametrize("r", [1, 5, 16])
def test_cross_launch_shapes(ltl, T, tile, r):
    rule = inputs.Rule(r, 0, 1, r, 3 * r, r + 1, 2 * r, "N")
    g0 = inputs.bernoulli_grid(200, 333, 0.5, seed=700 + r)
    tuning = dict(steps_per_launch=T, tile_rows=tile[0], tile_cols=tile[1], waves=0)
    if not shape_feasible(r, T, tile[0], tile[1], maxc=6):
        with pytest.raises(ltl.LtlError) as e:
            run_and_compare(ltl, g0, rule, "cat_i8", 7, tuning=tuning)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_and_compare(ltl, g0, rule, "cat_i8", 7, tuning=tuning)


def test_cross_periodic(ltl):
    rule = inputs.Rule(4, 0, 1, 4, 9, 5, 7, "N")
    for method in ("cat_i8", "direct"):
        run_periodic(ltl, inputs.bernoulli_grid(64, 80, 0.5, seed=81), rule, method, 4)
    run_periodic(ltl, inputs.bernoulli_grid(130, 224, 0.5, seed=82), rule, "cat_i8", 6,
                 tuning=dict(steps_per_launch=3, tile_rows=64, tile_cols=64), every_step=False)


def test_cross_refusals_and_direct_range(ltl):
    g = gpu_grid(np.zeros((8, 8), dtype=np.uint8))
    for method in ("cat_f16", "cat_f8"):
        with pytest.raises(ltl.LtlError) as e:
            ltl.Simulation(g, inputs.Rule(3, 0, 1, 3, 6, 4, 5, "N"), method)
        assert e.value.code == ltl.LTL_ERR_UNSUPPORTED
    with pytest.raises(ltl.LtlError) as e:
        ltl.Simulation(g, inputs.Rule(17, 0, 1, 20, 40, 25, 30, "N"), "cat_i8")
    assert e.value.code == ltl.LTL_ERR_UNSUPPORTED
    # the direct stencil covers the cross up to r = 32
    rule = inputs.Rule(24, 0, 1, 25, 60, 30, 45, "N")
    run_and_compare_each_step(ltl, inputs.bernoulli_grid(90, 140, 0.5, seed=24), rule, "direct", 3)


# ------------------------------------------------------------------ persistent (double-buffered) form
# The persistent form launches about one 8-wave workgroup per compute unit; with small tiles on
# a grid of ~1000 tiles every workgroup walks several tiles, so the double-buffered hand-over
# (load of tile i+1 while tile i computes) is exercised at every position of the walk.
PERSIST_GRID = (1000, 1008)     # ragged against 32-row / 32-column tiles; W % 16 == 0 for the torus


@pytest.mark.parametrize("boundary", ["dead", "periodic"])
@pytest.mark.parametrize("T", [1, 3])
@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8"])
def test_persistent_many_tiles(ltl, method, T, boundary):
    rule = inputs.BOSCO_M1
    g0 = inputs.bernoulli_grid(*PERSIST_GRID, 0.5, seed=41 + T)
    tuning = dict(steps_per_launch=T, tile_rows=32, tile_cols=32, waves=8, persistent=1)
    sim = ltl.Simulation(gpu_grid(g0), rule, method, tuning=tuning, boundary=boundary)
    assert sim.tuning()["persistent"] == 1
    for n in (3, 4):
        sim.step(n)
    got = sim.read().cpu().numpy()
    assert not sim.current_padded()[:, g0.shape[1]:].any()
    sim.close()
    ref = oracle.run(g0, rule, 7, periodic=(boundary == "periodic"))
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"persistent {method} T={T} {boundary}: {len(bad)} cells differ, first {bad[:5].tolist()}")


PERSIST_RULES = [inputs.Rule(3, 5, 0, 9, 20, 10, 14),            # decay states
                 inputs.Rule(24, 0, 0, 600, 1100, 650, 900),     # wide radius
                 inputs.Rule(5, 0, 1, 5, 12, 6, 9, "N"),         # cross neighbourhood
                 inputs.Rule(1, 0, 1, 3, 4, 3, 3)]               # Life: the smallest window


@pytest.mark.parametrize("rule", PERSIST_RULES, ids=lambda r: r.text())
@pytest.mark.parametrize("T", [1, 2])
def test_persistent_rules(ltl, rule, T):
    g0 = (inputs.state_grid(700, 704, rule.C, seed=rule.R) if rule.C >= 3
          else inputs.bernoulli_grid(700, 704, 0.5, seed=rule.R))
    tuning = dict(steps_per_launch=T, tile_rows=32, tile_cols=32, waves=8, persistent=1)
    run_and_compare(ltl, g0, rule, "cat_i8", 5, tuning=tuning, chunks=[2, 3])


@pytest.mark.parametrize("tile", [(16, 32), (64, 64), (96, 128), (160, 224)], ids=lambda t: f"{t[0]}x{t[1]}")
@pytest.mark.parametrize("T", [1, 4])
def test_persistent_tile_shapes(ltl, tile, T):
    """Few tiles (one per workgroup, some XCDs idle) up to many per workgroup."""
    rule = inputs.Rule(7, 0, 1, 56, 101, 60, 76)
    g0 = inputs.bernoulli_grid(301, 299, 0.5, seed=6)
    tuning = dict(steps_per_launch=T, tile_rows=tile[0], tile_cols=tile[1], waves=0, persistent=1)
    if not shape_feasible(7, T, tile[0], tile[1], lds_max=80 * 1024):
        with pytest.raises(ltl.LtlError) as e:
            run_and_compare(ltl, g0, rule, "cat_i8", 8, tuning=tuning)
        assert e.value.code == ltl.LTL_ERR_ARG
        return
    run_and_compare(ltl, g0, rule, "cat_i8", 8, tuning=tuning)


def test_persistent_tiny_grids(ltl):
    """Fewer tiles than XCDs: the surplus workgroups have no tile and exit."""
    rule = inputs.BOSCO_M1
    for shape in [(1, 1), (17, 33), (40, 100)]:
        g0 = inputs.bernoulli_grid(*shape, 0.5, seed=shape[1])
        run_and_compare(ltl, g0, rule, "cat_i8", 4, tuning=dict(steps_per_launch=2, tile_rows=16, tile_cols=32,
                                                                 waves=0, persistent=1))


def test_persistent_refused_where_absent(ltl):
    """The direct method has no persistent form; batches have no dataflow form (persistent = 2)
    and the batched direct method no persistent one."""
    g = gpu_grid(np.zeros((64, 64), dtype=np.uint8))
    with pytest.raises(ltl.LtlError) as e:
        ltl.Simulation(g, inputs.LIFE, "direct", tuning=dict(steps_per_launch=1, persistent=1))
    assert e.value.code == ltl.LTL_ERR_ARG
    with pytest.raises(ltl.LtlError) as e:
        ltl.Batch([g, g], [inputs.LIFE, inputs.LIFE], "cat_i8", tuning=dict(persistent=2))
    assert e.value.code == ltl.LTL_ERR_ARG
    with pytest.raises(ltl.LtlError) as e:
        ltl.Batch([g, g], [inputs.LIFE, inputs.LIFE], "direct", tuning=dict(persistent=1))
    assert e.value.code == ltl.LTL_ERR_ARG


# ------------------------------------------------------------------ windowed byte epilogues
# Two-state rules whose counts exceed 126 but whose finite range bounds all lie in a window
# c+1..c+126 run the byte epilogue on n - c clamped to 127 (int8 method); with a window up to
# c+254 the full-byte form (n - c clamped to 255, v_lerp_u8 range tests); the others keep
# 16-bit lanes. Each rule below sits on one side of these choices or at an edge of them; the
# grids are striped in density so that the counts sweep across the window bounds.
WINDOW_RULES = [
    inputs.Rule(6, 0, 1, 42, 76, 45, 57),            # sweep rule r = 6 (window 41..167)
    inputs.Rule(8, 0, 1, 100, 225, 150, 160),        # span exactly 126: 7-bit window
    inputs.Rule(8, 0, 1, 100, 226, 150, 160),        # span 127: full-byte window
    inputs.Rule(6, 0, 1, 10, 100, 0, 50),            # lower bound 0 (c = -1)
    inputs.Rule(6, 0, 1, 150, 169, 140, 160),        # upper bound at the largest count
    inputs.Rule(7, 0, 1, 60, 120, 9, 8),             # empty birth range
    inputs.Rule(6, 0, 1, 5, 4, 9, 8),                # both ranges empty
    inputs.Rule(9, 0, 0, 200, 250, 190, 260),        # M = 0: survival range moves up by one
    inputs.Rule(12, 0, 1, 156, 281, 168, 212),       # sweep rule r = 12 (span 126)
    inputs.Rule(16, 0, 1, 500, 560, 480, 600),       # r = 16, narrow window
    inputs.Rule(16, 0, 1, 272, 490, 294, 370),       # sweep rule r = 16 (full-byte window, span 219)
    inputs.Rule(10, 0, 1, 100, 353, 120, 200),       # span exactly 254: full-byte window
    inputs.Rule(10, 0, 1, 100, 354, 120, 200),       # span 255: 16-bit lanes
    inputs.Rule(9, 0, 1, 0, 253, 200, 253),          # full-byte window from count 0 (c = -1, span 254)
    inputs.Rule(11, 0, 0, 300, 529, 320, 9),         # M = 0, empty birth range, survival to the largest count
]


def striped_grid(H, W, seed):
    """Horizontal bands of Bernoulli densities 0.1 .. 0.9 (counts from low to high)."""
    ps = [0.1, 0.3, 0.35, 0.5, 0.65, 0.78, 0.9]
    band = -(-H // len(ps))
    parts = [inputs.bernoulli_grid(min(band, H - k * band), W, p, seed + k) for k, p in enumerate(ps) if k * band < H]
    return np.vstack(parts)


@pytest.mark.parametrize("rule", WINDOW_RULES, ids=lambda r: r.text())
def test_window_epilogue_every_step(ltl, rule):
    g0 = striped_grid(161, 203, seed=rule.R * 7 + rule.S2)
    run_and_compare_each_step(ltl, g0, rule, "cat_i8", 6)


@pytest.mark.parametrize("rule", WINDOW_RULES, ids=lambda r: r.text())
@pytest.mark.parametrize("form", ["T3", "persistent", "torus"])
def test_window_epilogue_launch_forms(ltl, rule, form):
    g0 = striped_grid(300, 336, seed=rule.R)
    if form == "torus":
        run_periodic(ltl, g0, rule, "cat_i8", 5, tuning=dict(steps_per_launch=2, tile_rows=64, tile_cols=64, waves=0),
                     every_step=False)
        return
    tuning = dict(steps_per_launch=3, tile_rows=64, tile_cols=96, waves=8, persistent=int(form == "persistent"))
    if not shape_feasible(rule.R, 3, 64, 96, lds_max=(80 if form == "persistent" else 160) * 1024):
        tuning["steps_per_launch"] = 1
    run_and_compare(ltl, g0, rule, "cat_i8", 7, tuning=tuning, chunks=[3, 4])


def test_window_epilogue_matches_half_lanes(ltl):
    """The same windowed rules through fp16 and fp8 (16-bit lanes) and the direct stencil."""
    g0 = striped_grid(257, 300, seed=77)
    for rule in WINDOW_RULES[:6]:
        ref = None
        for method in ["cat_i8", "cat_f16", "direct"] + (["cat_f8"] if rule.R <= 7 else []):
            sim = ltl.Simulation(gpu_grid(g0), rule, method)
            sim.step(9)
            got = sim.read().cpu().numpy()
            sim.close()
            if ref is None:
                ref = got
                assert np.array_equal(ref, oracle.run(g0, rule, 9)), rule.text()
            assert np.array_equal(got, ref), f"{method} {rule.text()}"


# ------------------------------------------------------------------ autotuner on small grids
@pytest.mark.parametrize("shape,boundary,rule", [
    ((1, 1), "dead", inputs.BOSCO_M1), ((37, 53), "dead", inputs.BOSCO_M1), ((64, 48), "periodic", inputs.LIFE),
    ((200, 336), "periodic", inputs.Rule(9, 4, 0, 90, 160, 97, 122)), ((150, 170), "dead", inputs.Rule(20, 0, 1, 300, 700, 320, 500)),
], ids=lambda x: str(x) if not hasattr(x, "text") else x.text())
def test_autotune_small_grids(ltl, shape, boundary, rule):
    """The autotuner (every steps-per-launch, tile, wave count and form it tries) runs on a
    copy, leaves the state untouched, and its pick computes the oracle's grid."""
    g0 = (inputs.state_grid(*shape, rule.C, seed=7) if rule.C >= 3 else inputs.bernoulli_grid(*shape, 0.5, seed=7))
    sim = ltl.Simulation(gpu_grid(g0), rule, "cat_i8", boundary=boundary)
    sim.step(2)
    before = sim.read().cpu().numpy()
    for bad in (0, 4097):                                         # probe length out of range
        with pytest.raises(ltl.LtlError) as e:
            sim.autotune(probe_steps=bad)
        assert e.value.code == ltl.LTL_ERR_ARG
    best = sim.autotune(probe_steps=3)
    assert np.array_equal(sim.read().cpu().numpy(), before)      # the probes ran on a copy
    assert sim.tuning() == best
    sim.step(5)
    got = sim.read().cpu().numpy()
    sim.close()
    assert np.array_equal(got, oracle.run(g0, rule, 7, periodic=(boundary == "periodic"))), best


@pytest.mark.parametrize("C", [3, 4, 7, 8, 9, 16, 255])
def test_decay_state_counts(ltl, C):
    """Decay rules around the 3-bit boundary of the state-table epilogue (C <= 8 on int8) and
    above it (C > 8: the SWAR decay epilogue), every method, dead and torus, several launch
    shapes; initial grids hold every state 0..C-1."""
    rng = np.random.default_rng(C)
    g0 = np.where(rng.random((200, 304)) < 0.45, 1, 0).astype(np.uint8)
    dec = rng.random(g0.shape) < 0.2
    g0[dec] = rng.integers(2, C, size=int(dec.sum()), dtype=np.uint8)
    for rule in (inputs.Rule(3, C, 0, 12, 22, 13, 16), inputs.Rule(16, C, 1, 300, 500, 330, 420)):
        for method in ("cat_i8", "cat_f16", "direct") + (("cat_f8",) if rule.R <= 7 else ()):
            for tuning in (None, dict(steps_per_launch=2, tile_rows=64, tile_cols=96, waves=8)):
                if method == "direct" and tuning:
                    continue
                run_and_compare(ltl, g0, rule, method, 7, tuning=tuning)
        sim = ltl.Simulation(gpu_grid(g0), rule, "cat_i8", boundary="periodic")
        sim.step(5)
        got = sim.read().cpu().numpy()
        sim.close()
        assert np.array_equal(got, oracle.run(g0, rule, 5, periodic=True))
