"""GPU parity by exhaustion.

* Every 5x5 neighbourhood (all 2^25 patterns, tiled as adjacent blocks of a 20480 x 40960
  grid): after one step the centre of each block must follow the rule applied to its block's
  popcount, through every method.
* Every count value through every epilogue: for radii 1..32, blocks of (2r+1)^2 cells with
  exactly k alive non-centre cells for each k, with a dead, an alive and (decay rules)
  decaying centres, and decaying neighbours that must not count. Each block's centre sees
  exactly its own block, so its next state is the rule's transition of that count — the
  windowed byte epilogue's window bounds and clamp, the 16-bit lanes and the decay path are
  all driven across their whole count range. Expected values come from the rule notation.
"""
import functools
import math

import numpy as np
import pytest

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


def transition(rule, s, n_box):
    """Next state from the rule notation: n_box counts the block's state-1 cells, centre included."""
    R, C, M, S1, S2, B1, B2 = rule.as_tuple()
    Cn = C if C >= 3 else 2
    alive = (s == 1)
    cnt = n_box - (alive.astype(np.int64) if M == 0 else 0)
    born = (B1 <= cnt) & (cnt <= B2)
    keep = (S1 <= cnt) & (cnt <= S2)
    nxt = np.where(s == 0, born.astype(np.int64),
                   np.where(alive, np.where(keep, 1, 2 if Cn > 2 else 0),
                            np.where(s + 1 < Cn, s + 1, 0)))
    return nxt.astype(np.uint8)


# ------------------------------------------------------------------ all 5x5 neighbourhoods
@pytest.fixture(scope="module")
def all_5x5(ltl):
    p = torch.arange(1 << 25, dtype=torch.int64, device="cuda").reshape(4096, 8192)
    g = torch.zeros((4096 * 5, 8192 * 5), dtype=torch.uint8, device="cuda")
    for di in range(5):
        for dj in range(5):
            g[di::5, dj::5] = ((p >> (5 * di + dj)) & 1).to(torch.uint8)
    pn = p.cpu().numpy()
    pop = np.bitwise_count(pn.astype(np.uint64)).astype(np.int64)
    centre = ((pn >> 12) & 1).astype(np.int64)
    return g, pop, centre


@pytest.mark.parametrize("rule", [inputs.Rule(2, 0, 1, 7, 13, 8, 11), inputs.Rule(2, 2, 0, 0, 24, 0, 6),
                                  inputs.Rule(2, 0, 0, 3, 17, 1, 1)], ids=lambda r: r.text())
@pytest.mark.parametrize("method", ["cat_i8", "cat_f16", "cat_f8", "direct"])
def test_all_5x5_neighbourhoods(ltl, all_5x5, rule, method):
    g, pop, centre = all_5x5
    sim = ltl.Simulation(g, rule, method)
    sim.step(1)
    got = sim.read()[2::5, 2::5].cpu().numpy()
    sim.close()
    want = transition(rule, centre, pop)
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{method} {rule.text()}: {len(bad)} of 2^25 patterns wrong, first {bad[:3].tolist()}"


# ------------------------------------------------------------------ every count value
@functools.lru_cache(maxsize=None)
def count_sweep(r, C, seed):
    """Grid of blocks (s, k): centre state s, exactly k alive non-centre cells (positions drawn
    from a seeded permutation), and with C >= 3 half of the remaining cells decaying."""
    d = 2 * r + 1
    N = d * d
    mid = r * d + r
    states = [0, 1] + ([2, C - 1] if C >= 3 else [])
    blocks = [(s, k) for s in states for k in range(N)]
    nbj = math.ceil(math.sqrt(len(blocks)))
    nbi = math.ceil(len(blocks) / nbj)
    g = np.zeros((nbi * d, nbj * d), dtype=np.uint8)
    rng = np.random.default_rng(seed)
    others = np.delete(np.arange(N), mid)
    for idx, (s, k) in enumerate(blocks):
        cells = np.zeros(N, dtype=np.uint8)
        pos = rng.permutation(others)
        cells[pos[:k]] = 1
        if C >= 3:
            rest = pos[k:]
            cells[rest[: len(rest) // 2]] = rng.integers(2, C, size=len(rest) // 2, dtype=np.uint8)
        cells[mid] = s
        bi, bj = divmod(idx, nbj)
        g[bi * d:(bi + 1) * d, bj * d:(bj + 1) * d] = cells.reshape(d, d)
    s_arr = np.array([b[0] for b in blocks], dtype=np.int64)
    n_box = np.array([b[1] + (b[0] == 1) for b in blocks], dtype=np.int64)
    return g, s_arr, n_box, nbj, d


def sweep_rules(r):
    N = (2 * r + 1) ** 2
    rules = [inputs.sweep_rule(r) if r <= 16 else inputs.Rule(r, 0, 1, N // 4, (45 * N) // 100, (27 * N) // 100,
                                                             (34 * N) // 100),
             inputs.Rule(r, 0, 0, N // 3, N // 3 + min(100, N // 3), N // 3 + 5, N // 3 + min(60, N // 4)),  # narrow
             inputs.Rule(r, 0, 1, N // 10, (9 * N) // 10, 0, N // 6),          # wide, lower bound 0
             inputs.Rule(r, 0, 1, N - min(N // 2, 90), N, N // 2, N - 1)]      # open upper bound
    # spans 127..254 from r = 8 on: the full-byte window
    rules.append(inputs.Rule(r, 0, 1, N // 5, N // 5 + min(240, N // 2), N // 5 + min(10, N // 4), N // 5 + min(250, N // 2)))
    rules.append(inputs.Rule(r, 5, 0, N // 4, N // 4 + min(120, N // 3), N // 5, N // 5 + min(40, N // 4)))  # decay
    # decay with a window wider than 254 counts (16-bit range test) where N allows it
    rules.append(inputs.Rule(r, 6, 1, N // 10, (8 * N) // 10, N // 5, N // 5 + min(60, N // 4)))
    # decay with the fewest states and with more states than the 3-bit state tables hold
    rules.append(inputs.Rule(r, 3, 1, N // 5, N // 5 + min(110, N // 3), N // 4, N // 4 + min(50, N // 4)))
    rules.append(inputs.Rule(r, 12, 0, N // 6, N // 6 + min(100, N // 3), N // 4, N // 4 + min(30, N // 5)))
    return rules


@pytest.mark.parametrize("r", [1, 2, 5, 6, 7, 8, 11, 12, 13, 16, 17, 24, 32])
def test_every_count_through_every_epilogue(ltl, r):
    for rule in sweep_rules(r):
        g, s_arr, n_box, nbj, d = count_sweep(r, rule.C, 1000 + r)
        want = transition(rule, s_arr, n_box)
        methods = ["cat_i8"] + (["cat_f16", "direct"] if r <= 16 else ["direct"] if r <= 24 else []) \
            + (["cat_f8"] if r <= 7 else [])
        for method in methods:
            for periodic in (False, True):
                if periodic and (g.shape[1] % 16 or method != "cat_i8"):
                    continue
                sim = ltl.Simulation(torch.from_numpy(g).cuda(), rule, method,
                                     boundary="periodic" if periodic else "dead")
                sim.step(1)
                out = sim.read().cpu().numpy()
                sim.close()
                idx = np.arange(len(s_arr))
                got = out[(idx // nbj) * d + r, (idx % nbj) * d + r]
                bad = np.flatnonzero(got != want)
                assert len(bad) == 0, (f"{method} {rule.text()} {'torus' if periodic else 'dead'}: {len(bad)} of "
                                       f"{len(want)} (state, count) blocks wrong, e.g. state {s_arr[bad[0]]} "
                                       f"count {n_box[bad[0]]}: got {got[bad[0]]}, want {want[bad[0]]}")


@functools.lru_cache(maxsize=None)
def cross_sweep(r, C, seed):
    """Blocks (s, k) for the cross neighbourhood: exactly k alive cells on the 4r arm cells of
    the centre's row and column, and random alive (or decaying) cells off the cross, which must
    not count."""
    d = 2 * r + 1
    mid = r * d + r
    arm = np.array([r * d + j for j in range(d) if j != r] + [i * d + r for i in range(d) if i != r])
    off = np.setdiff1d(np.arange(d * d), np.append(arm, mid))
    states = [0, 1] + ([2, C - 1] if C >= 3 else [])
    blocks = [(s, k) for s in states for k in range(4 * r + 1)]
    nbj = math.ceil(math.sqrt(len(blocks)))
    nbi = math.ceil(len(blocks) / nbj)
    g = np.zeros((nbi * d, nbj * d), dtype=np.uint8)
    rng = np.random.default_rng(seed)
    for idx, (s, k) in enumerate(blocks):
        cells = np.zeros(d * d, dtype=np.uint8)
        cells[off] = rng.integers(0, 2 if C < 3 else C, size=len(off), dtype=np.uint8)
        pos = rng.permutation(arm)
        cells[pos[:k]] = 1
        if C >= 3:
            cells[pos[k:]] = np.where(rng.random(len(arm) - k) < 0.5, 0, rng.integers(2, C, size=len(arm) - k))
        cells[mid] = s
        bi, bj = divmod(idx, nbj)
        g[bi * d:(bi + 1) * d, bj * d:(bj + 1) * d] = cells.reshape(d, d)
    s_arr = np.array([b[0] for b in blocks], dtype=np.int64)
    n_box = np.array([b[1] + (b[0] == 1) for b in blocks], dtype=np.int64)
    return g, s_arr, n_box, nbj, d


def cross_rules(r):
    n = 4 * r + 1
    return [inputs.Rule(r, 0, 1, n // 4, n // 2, n // 3, n // 2, "N"), inputs.Rule(r, 0, 0, 1, n - 2, n // 2, n, "N"),
            inputs.Rule(r, 4, 0, n // 5, (3 * n) // 5, 0, n // 4, "N")]


@pytest.mark.parametrize("r", [1, 2, 5, 9, 16])
def test_every_cross_count(ltl, r):
    for rule in cross_rules(r):
        g, s_arr, n_box, nbj, d = cross_sweep(r, rule.C, 2000 + r)
        want = transition(rule, s_arr, n_box)
        for method in ("cat_i8", "direct"):
            sim = ltl.Simulation(torch.from_numpy(g).cuda(), rule, method)
            sim.step(1)
            out = sim.read().cpu().numpy()
            sim.close()
            idx = np.arange(len(s_arr))
            got = out[(idx // nbj) * d + r, (idx % nbj) * d + r]
            bad = np.flatnonzero(got != want)
            assert len(bad) == 0, (f"{method} {rule.text()}: {len(bad)} of {len(want)} blocks wrong, e.g. state "
                                   f"{s_arr[bad[0]]} count {n_box[bad[0]]}: got {got[bad[0]]}, want {want[bad[0]]}")
